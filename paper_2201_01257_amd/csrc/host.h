// Host-side handle definitions and error helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/tamm_mi.h"
#include "internal.h"

namespace tamm {

int fail(int code, const char* fmt, ...);
int ok();

// Drops the cached one-shot plans that name tensor t (called when t is destroyed).
void contract_cache_evict(const tamm_tensor* t);

// AddOp enqueue (addop.cpp), shared with the scheduler.
int add_enqueue(tamm_add* a, double alpha, double beta, hipStream_t s);
const tamm_tensor* add_out(const tamm_add* a);
const tamm_tensor* add_in(const tamm_add* a);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SpaceData {
  std::vector<int64_t> size, offset;
  std::vector<int8_t> spin;
  int64_t extent = 0;
  bool same(const SpaceData& o) const { return size == o.size && spin == o.spin; }
  int ntiles() const { return (int)size.size(); }
};

}  // namespace tamm

#define HIP_TRY(expr)                                                                                     \
  do {                                                                                                    \
    hipError_t e_ = (expr);                                                                               \
    if (e_ != hipSuccess) return ::tamm::fail(TAMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

struct tamm_space {
  std::shared_ptr<tamm::SpaceData> d;
};

struct tamm_tensor {
  int rank = 0;
  std::vector<std::shared_ptr<tamm::SpaceData>> dims;
  std::vector<int64_t> tstride;      // tile-linear strides per dim
  std::vector<int64_t> tile_off;     // per tile-linear index: element offset, -1 = not stored
  std::vector<int32_t> block_tiles;  // stored blocks, rank entries each, lexicographic
  std::vector<int64_t> block_off;
  std::vector<int64_t> tile_offset_cat, tile_size_cat;  // per dim, concatenated
  std::vector<int32_t> dim_tile_base;
  int64_t numel = 0;
  int64_t max_block = 0;
  double* dev = nullptr;
  size_t dev_bytes = 0;
  bool bound = false;
};
