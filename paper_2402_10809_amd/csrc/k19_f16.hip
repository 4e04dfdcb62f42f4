// D3Q19 kernels with _Float16 population storage.
#include "launch19.hpp"

LBM_INSTANTIATE19(_Float16)
