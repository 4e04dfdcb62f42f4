// D3Q19 kernels with __bf16 population storage.
#include "launch19.hpp"

LBM_INSTANTIATE19(__bf16)
