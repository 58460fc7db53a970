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
// AddOp chains (several AddOps into one out, one launch), built by the scheduler.
bool add_chain_accepts(const tamm_add* head, const tamm_add* b, int* ydim);
int add_chain_items(const std::vector<const tamm_add*>& m, int ydim, std::vector<AddItem>& items, bool* plane);
int add_chain_enqueue(const std::vector<tamm_add*>& m, const std::vector<double>& alpha, double beta, int ydim,
                      bool plane, const AddItem* items, int64_t n_items, hipStream_t s);

// Plans and groups (plan.cpp), shared with the scheduler.
void plan_io(const tamm_plan* p, tamm_tensor** out, const tamm_tensor** lhs, const tamm_tensor** rhs, int* precision);
bool plans_fusable(tamm_plan* a, tamm_plan* b);
int group_create_nodes(const std::vector<std::vector<tamm_plan*>>& nodes, tamm_group** out);
int group_enqueue(tamm_group* g, hipStream_t s);
int group_update_desc(tamm_group* g, const double* alpha, const double* beta, hipStream_t s, bool* changed);
int group_check_bound(tamm_group* g);
int group_autotune(tamm_group* g, hipStream_t s, const char* cache_path, int32_t reps);
size_t group_workspace_size(const tamm_group* g);
size_t group_autotune_workspace_size(tamm_group* g);
int group_bind_ws(tamm_group* g, void* ws, size_t bytes);
size_t group_node_count(const tamm_group* g);

// Denominator update (denominator.cpp), shared with the scheduler.
int denominator_enqueue(tamm_denominator* d, const double* const* energy, hipStream_t s);
void denominator_io(const tamm_denominator* d, tamm_tensor** out, const tamm_tensor** in);

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
