// D3Q27 kernels with 16-bit population storage (FP16 and BF16).
#include "launch27.hpp"

LBM_INSTANTIATE27(_Float16)
LBM_INSTANTIATE27(__bf16)
