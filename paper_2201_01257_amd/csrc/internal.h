// Internal data layouts shared by the host planner and the HIP kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tamm {

constexpr int kMaxRank = 8;

// Operand offset tables are followed by kTablePad entries holding kTableInvalid, so that the
// gathers may read a table up to a tile (or a K chunk) past its end.  A gathered element whose
// row or k entry is kTableInvalid lies at least 8 * kTableInvalid bytes = 1 GiB into its block,
// which is beyond every operand block (the planner rejects blocks of 2^27 or more elements), so
// the bounds-checked buffer load returns zero for it.
constexpr int32_t kTableInvalid = 1 << 27;
constexpr int kTablePad = 256;

// One stored block of the output tensor, as the contraction kernel and the screening kernel see
// it.  The flattened M (out&A) and N (out&B) extents and the offset tables that map a flattened
// row/column to an element offset inside the block are fixed by the block's tile sizes.
struct OutBlockDesc {
  int64_t c_off;      // element offset of the block in out's storage
  int32_t mext;       // flattened M extent (product of M-label tile sizes)
  int32_t next;       // flattened N extent
  int32_t c_tabM;     // start of out's M offset table (int32 pool)
  int32_t c_tabN;     // start of out's N offset table
  int32_t a_tbase;    // A-operand tile-linear index contributed by the M labels
  int32_t b_tbase;    // B-operand tile-linear index contributed by the N labels
  int32_t a_cbase;    // A-operand shape-class id contributed by the M labels
  int32_t b_cbase;    // B-operand shape-class id contributed by the N labels
  int32_t pair_base;  // first slot of this block's surviving-pair list
  int32_t pad;
};
static_assert(sizeof(OutBlockDesc) == 48, "OutBlockDesc layout");

// One surviving tile pair of an output block, written by the screening kernel.
struct PairDesc {
  int64_t a_off;   // element offset of the A-operand block
  int64_t b_off;   // element offset of the B-operand block
  int32_t kext;    // flattened K extent of the pair
  int32_t a_tabM;  // A's M offset table for this A block shape
  int32_t a_tabK;  // A's K offset table
  int32_t b_tabK;  // B's K offset table
  int32_t b_tabN;  // B's N offset table
  int32_t kt;      // index of the K tile tuple (lexicographic over the K labels)
};
static_assert(sizeof(PairDesc) == 40, "PairDesc layout");

// One output macro-tile (or one K split of it) processed by one workgroup.  A tile split into
// nsplit > 1 parts (each a contiguous range of its block's surviving pairs) writes partial tiles
// to workspace slots tile .. tile + nsplit - 1, which k_reduce sums in order; an unsplit tile
// runs the epilogue itself.
struct WorkItem {
  int32_t prob;   // problem index inside a group (0 for a single plan)
  int32_t ob;     // output block
  int32_t m0;     // first flattened row of the tile
  int32_t n0;     // first flattened column
  int32_t split;  // split index in bits 0-15, number of splits of the tile in bits 16-30 (0 = 1)
  int32_t tile;   // first partial-tile slot of the tile (split tiles only)
};
static_assert(sizeof(WorkItem) == 24, "WorkItem layout");

__host__ __device__ inline int32_t item_split(const WorkItem& w) { return w.split & 0xFFFF; }
__host__ __device__ inline int32_t item_nsplit(const WorkItem& w) { return (w.split >> 16) > 1 ? (w.split >> 16) : 1; }
__host__ __device__ inline int32_t encode_split(int32_t split, int32_t nsplit) { return split | (nsplit << 16); }

// Everything the contraction kernel needs about one contraction.
struct ProblemDesc {
  const double* A;
  const double* B;
  double* C;
  const OutBlockDesc* blocks;
  const PairDesc* pairs;
  const int32_t* counts;
  const int32_t* pool;
  double* partial;   // K-split partial tiles [tile][split][MT*NT], or null
  double alpha;
  double beta;
  int32_t k_splits;
  int32_t a_kc;      // 1: A's stride-1 label is summed (gather lanes run along k), 0: along m
  int32_t b_kc;      // 1: B's stride-1 label is summed, 0: along n
  int32_t pad;
  int64_t a_plane;   // split-bfloat16 planes: elements between the slice planes of A (else 0)
  int64_t b_plane;   // the same for B
};
static_assert(sizeof(ProblemDesc) == 112, "ProblemDesc layout");

struct ContractParams {
  ProblemDesc single;         // used when probs is null (one plan)
  const ProblemDesc* probs;   // group: per-problem descriptors in device memory
  const WorkItem* work;
  int32_t* next_item;         // persistent launch: work counter (starts at gridDim.x), else null
  int32_t n_work;
  int32_t pad;
};

// Screening of one contraction (a segment).  Several contractions that write the same output
// tiles (a fused node) screen as consecutive segments of one list: every segment appends its
// surviving pairs to the pair list of the first segment's output block, with its operand element
// offsets and table starts shifted so that they are relative to the first segment's operand base
// pointers and table pool.
struct ScreenDesc {
  const int64_t* a_tile_off;  // per A tile-linear index: element offset, -1 = not stored
  const int64_t* b_tile_off;
  const OutBlockDesc* blocks;
  PairDesc* pairs;            // pair list base (first segment's): block ob's pairs at ob * pair_stride
  int32_t* counts;            // surviving pairs per output block (first segment's)
  const int32_t* pool;        // this segment's int32 table pool
  int64_t a_base;             // added to the A block offsets of the pairs (elements)
  int64_t b_base;             // added to the B block offsets
  int32_t pool_base;          // added to the table starts of the pairs (int32 entries)
  int32_t pair_stride;        // pair capacity per output block
  int32_t next_seg;           // index of the next segment in ScreenParams::probs, -1: last
  int32_t n_blocks;
  int32_t n_kt;               // K tile tuples (pair capacity per output block)
  int32_t nk;                 // number of K labels
  int32_t k_ntiles[kMaxRank];
  int32_t a_tstride[kMaxRank];
  int32_t b_tstride[kMaxRank];
  int32_t a_cstride[kMaxRank];
  int32_t b_cstride[kMaxRank];
  int32_t k_size_tab[kMaxRank];  // pool start of the K label's tile-size list
  int32_t k_cls_tab[kMaxRank];   // pool start of the K label's tile size-class list
  int32_t a_cls_tabM;            // pool start of the per-A-class table starts (M)
  int32_t a_cls_tabK;
  int32_t b_cls_tabK;
  int32_t b_cls_tabN;
};

struct ScreenParams {
  ScreenDesc single;
  const ScreenDesc* probs;       // group: per-problem screen descriptors
  const int32_t* item_prob;      // group: problem of each screening item
  const int32_t* item_block;     // group: output block of each screening item
  int32_t n_items;               // single: = single.n_blocks
  int32_t pad;
};

struct ReduceItem {
  int32_t prob, ob, m0, n0;
  int32_t tile;    // first partial-tile slot
  int32_t nsplit;  // partial tiles to sum, in slot order
};

struct ReduceParams {
  ProblemDesc single;
  const ProblemDesc* probs;
  const ReduceItem* items;
  int32_t n_items;
  int32_t tile_m;
  int32_t tile_n;
  int32_t pad;
};

struct DenomParams {
  double* out;
  const double* in;
  const int64_t* block_off;    // per stored block: element offset
  const int32_t* block_tiles;  // per stored block: rank tile indices
  const int64_t* tile_offset;  // per dim: untiled start of each tile (concatenated)
  const int64_t* tile_size;
  const double* energy[kMaxRank];
  int32_t dim_tile_base[kMaxRank];
  int8_t sign[kMaxRank];
  int32_t rank;
  int32_t chunk;                // elements per workgroup
  const int32_t* item_block;    // per workgroup: block index
  const int32_t* item_start;    // per workgroup: first element inside the block
  int64_t n_items;              // workgroups
};

// AddOp (out = beta*out + alpha*in with permuted labels): one stored block of out and the block
// of in at the permuted tile tuple.
struct AddBlock {
  int64_t out_off;           // element offset of the out block
  int64_t in_off;            // element offset of the in block; -1: not stored (reads as zero)
  int32_t ext[kMaxRank];     // extents, out's dimension order
  int32_t istr[kMaxRank];    // in-block stride of the label of each out dimension
};

// Work item of the AddOp kernels.  Direct mode (out and in end in the same label): a = first
// element of a chunk.  Transpose mode: a = batch index over the dimensions other than the two
// stride-1 ones, b = first row (out dimension ydim), c = first column (out's last dimension).
struct AddItem {
  int32_t block, a, b, c;
};

struct AddParams {
  double* out;
  const double* in;
  const AddBlock* blocks;
  const AddItem* items;
  int64_t n_items;
  double alpha, beta;
  int32_t rank;
  int32_t ydim;   // transpose mode: out dimension of in's last label; -1: direct mode
  int32_t chunk;  // direct mode: elements per item
  int32_t pad;
};

hipError_t launch_add(const AddParams& p, hipStream_t s);

// A chain of AddOps into one out (the scheduler's fused element-wise node): out = beta*out +
// sum_t alpha_t*in_t(permuted), out read and written once.  Every term shares out's block list
// (blocks[t][b] describes out block b for term t).  trans[t] = 1 when in_t's last label is out
// dimension ydim (read through LDS), 0 when it is out's last label (read directly).  Items are
// transpose-mode tiles of the (ydim, last) plane, or, with plane = 1 (ydim = rank - 2, every
// input's last two labels are out's last two, planes of at most kAddPlaneMax elements), whole
// planes: block and batch index over the other dimensions.
constexpr int kMaxAddTerms = 8;
constexpr int kAddPlaneMax = 1024;
struct AddMultiParams {
  double* out;
  const double* in[kMaxAddTerms];
  const AddBlock* blocks[kMaxAddTerms];
  double alpha[kMaxAddTerms];
  int32_t trans[kMaxAddTerms];
  const AddItem* items;
  int64_t n_items;
  double beta;
  int32_t rank, ydim, nterms, plane;
};

hipError_t launch_add_multi(const AddMultiParams& p, hipStream_t s);
// SetOp: p[0 .. n) = value.
hipError_t launch_fill(double* p, int64_t n, double value, hipStream_t s);

// Kernel configuration of the FP64 contraction kernel family.
struct F64Config {
  int mt, nt, kt, wgm, wgn, occ;  // occ: minimum waves per SIMD the registers must allow
  const char* name;
};

int f64_config_count();
const F64Config& f64_config(int id);

// Launchers (kernels.hip).  Return hipError_t of the launch.  grid <= 0: one workgroup per item.
hipError_t launch_screen(const ScreenParams& p, hipStream_t s);
hipError_t launch_contract_f64(int config, int layout, const ContractParams& p, int grid, hipStream_t s);
// Resident workgroups per compute unit of one configuration and gather layout (at least 1).
int f64_occupancy(int config, int layout);
hipError_t launch_reduce(const ReduceParams& p, hipStream_t s);
hipError_t launch_set_counter(int32_t* counter, int32_t value, hipStream_t s);
hipError_t launch_denominator(const DenomParams& p, hipStream_t s);

}  // namespace tamm
