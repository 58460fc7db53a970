// Mixed-precision contraction kernels (float32 and split-bfloat16 products with float64
// promotion).
#include <hip/hip_runtime.h>
