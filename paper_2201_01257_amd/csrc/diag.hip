// Diagnostic entry point: one matrix-core instruction executed by one wave on caller data, so that
// tests can pin the instruction's lane layout and the rounding of its float32 accumulation with
// inputs whose exact results the host knows.  Not used by the contraction path.
#include <hip/hip_runtime.h>

#include "host.h"

using namespace tamm;

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// op 0: v_mfma_f32_16x16x4_f32;  op 1: v_mfma_f32_16x16x32_bf16;  op 2: v_mfma_f32_32x32x16_bf16;
// op 3: v_mfma_f32_32x32x2_f32.  Operands are read per lane (a, b: one float or eight bfloat16;
// c: 4 or 16 floats) and the result registers are written back per lane in the same layout as c.
__global__ __launch_bounds__(64) void k_diag_mfma(int op, const void* a, const void* b, const float* c, float* d) {
  const int l = threadIdx.x;
  if (op == 0 || op == 1) {
    f4_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = c[4 * l + r];
    if (op == 0)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(static_cast<const float*>(a)[l], static_cast<const float*>(b)[l], acc, 0, 0, 0);
    else
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(static_cast<const bf8_t*>(a)[l], static_cast<const bf8_t*>(b)[l], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) d[4 * l + r] = acc[r];
  } else {
    f16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = c[16 * l + r];
    if (op == 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(static_cast<const bf8_t*>(a)[l], static_cast<const bf8_t*>(b)[l], acc, 0, 0, 0);
    else
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(static_cast<const float*>(a)[l], static_cast<const float*>(b)[l], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) d[16 * l + r] = acc[r];
  }
}

}  // namespace

extern "C" int tamm_diag_mfma(int32_t op, const void* a, const void* b, const float* c, float* d, void* stream) {
  if (op < 0 || op > 3) return fail(TAMM_ERR_ARG, "op must be 0..3");
  if (!a || !b || !c || !d) return fail(TAMM_ERR_ARG, "null device pointer");
  hipLaunchKernelGGL(k_diag_mfma, dim3(1), dim3(64), 0, (hipStream_t)stream, (int)op, a, b, c, d);
  HIP_TRY(hipGetLastError());
  return ok();
}
