// Internal declarations of the mixed-precision path (operand split and contraction kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tamm_mi.h"
#include "internal.h"

namespace tamm {

// K window (in flattened K indices of a tile pair, starting at the pair's first index) over which
// float32 partial sums are kept before they are added to the float64 accumulators.  The aligned
// split also takes its per-(row, window) scale over the same windows.
constexpr int kSplitWindow = 256;

// One stored block of an operand, as the split kernel sees it: rows are the flattened M (A) or N
// (B) labels, k the flattened K labels, both through the plan's offset tables.
struct PrepBlock {
  int64_t off;     // element offset of the block
  int64_t item0;   // first split item of this block
  int32_t rows;    // flattened row extent
  int32_t kext;    // flattened K extent
  int32_t tab_row; // pool start of the row offset table
  int32_t tab_k;   // pool start of the K offset table
  int32_t nwin;    // K windows
  int32_t pad;
};
static_assert(sizeof(PrepBlock) == 40, "PrepBlock layout");

struct PrepParams {
  const double* x;        // float64 operand
  void* out;              // packed: one 64-bit word of slices per element at x's element offsets;
                          // planes: bfloat16 slice s of block b's element (row, k) at
                          // out[s * plane_stride + off_b + row * kext_b + k]
  const PrepBlock* blocks;
  const int32_t* pool;
  int64_t n_items;
  int64_t plane_stride;   // planes layout: elements per slice plane
  int32_t n_blocks;
  int32_t aligned;        // 1: aligned lead + 3 residual slices, 0: 3 plain slices
  int32_t planes;         // 1: planes layout, 0: packed
  int32_t pad;
};

struct MixedConfig {
  int mt, nt, kt, wgm, wgn;
  const char* name;
};

int mixed_config_count(int precision);
const MixedConfig& mixed_config(int precision, int id);

hipError_t launch_prep_split(const PrepParams& p, bool rows_along_lanes, hipStream_t s);
// layout: bits 0-1 as for the float64 kernels; kPlanesLayout: split operands in planes layout.
constexpr int kPlanesLayout = 8;
hipError_t launch_contract_mixed(int precision, int config, int layout, const ContractParams& p, hipStream_t s);

}  // namespace tamm
