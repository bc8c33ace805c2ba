// Mixed-precision kernels (split-BF16 on MFMA); filled in below.
#include <hip/hip_runtime.h>

#include "ladder_types.hpp"
