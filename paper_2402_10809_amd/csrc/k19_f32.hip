// D3Q19 kernels with float population storage.
#include "launch19.hpp"

LBM_INSTANTIATE19(float)
