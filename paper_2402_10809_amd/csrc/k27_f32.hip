// D3Q27 kernels with float population storage.
#include "launch27.hpp"

LBM_INSTANTIATE27(float)
