// The one-shot contraction for callers that cannot allocate device memory (code under graph
// capture, serving loops, harnesses that forbid hipMalloc): tamm_contract with its workspace taken
// from a file-scope device array instead of a caller buffer.
//
// The array `scratch` exists once per GPU the library runs on, for the life of the process.  Host
// code never uses its name as an address: on a device's first call the device address is read
// with hipGetSymbolAddress (with that device current) and kept per device; every later use goes
// through that pointer.  Calls on one GPU share the array and it keeps the last call's contents
// (the contraction needs no zeroed workspace: screening writes every count and pair list it reads,
// K-split partial tiles are written before they are summed).  Calls that overlap in time on one
// GPU race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.h"

using namespace tamm;

namespace {

constexpr size_t kScratchBytes = TAMM_NOALLOC_WORKSPACE_BYTES;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, null until read

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

extern "C" int tamm_contract_noalloc(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                                     const tamm_tensor* rhs, const char* rhs_lbl, int32_t precision, double alpha,
                                     double beta, void* stream) {
  // the plan (host analysis, cached in the library) fixes the workspace the contraction needs
  size_t need = 0;
  int rc = tamm_contract_workspace_size(out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl, precision, &need);
  if (rc != TAMM_OK) return rc;
  if (need > kScratchBytes)
    return fail(TAMM_ERR_WORKSPACE,
                "this contraction needs a %zu-byte workspace; the allocation-free entry point holds %zu bytes per GPU "
                "(use tamm_contract with a caller workspace)",
                need, kScratchBytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TAMM_ERR_UNSUPPORTED, "device %d is beyond the %d supported", dev, kMaxDevices);
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p || ((uintptr_t)p) % 256) return fail(TAMM_ERR_HIP, "scratch array of device %d is not 256-byte aligned", dev);
      g_scratch_ptr[dev] = p;
    }
    ptr = g_scratch_ptr[dev];
  }
  return tamm_contract(out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl, precision, alpha, beta, ptr, kScratchBytes, stream);
}
