/* tamm_mi.h -- C ABI of the MI355X (gfx950) block-sparse tensor contraction library.
 *
 * The library implements the tensor-contraction operation of TAMM (arXiv 2201.01257,
 * "TAMM: Tensor Algebra for Many-body Methods") for one GPU:
 *
 *   - tiled index spaces with a spin attribute per tile (Sec. III-A, Fig. 1);
 *   - block-sparse tensors that store only structurally non-zero blocks, decided by spin
 *     symmetry or by a user-supplied non-zero check (Sec. III-A; non-zero-only block storage
 *     is the third distribution scheme of Sec. III-B);
 *   - the contraction C(..) = beta*C(..) + alpha * A(..) * B(..) of the operation grammar
 *     (Sec. III-A, Fig. 3 rule 8, Fig. 4), with "=" as beta = 0, "+=" as beta = 1 and "-=" as
 *     alpha -> -alpha;
 *   - deferred execution: an operation is analysed once into a plan and executed many times
 *     (the queue-then-execute scheduler of Sec. III-A, Fig. 4, and Sec. III-B), and several
 *     independent plans can be executed as one group.
 *
 * Conventions for every entry point:
 *   - Every function returns a tamm_status (0 = success).  Nothing throws or aborts across
 *     the ABI.  On failure tamm_last_error() returns a message for the calling thread.
 *   - Device memory is owned by the caller.  The library never allocates device memory: the
 *     caller binds tensor storage (tamm_tensor_bind) and plan/group workspace
 *     (tamm_plan_bind_workspace, tamm_group_bind_workspace) or passes it (tamm_contract).
 *     Handles own host metadata only.
 *   - Asynchronous calls take a hipStream_t (passed as void*; NULL = the null stream), enqueue
 *     their kernels on it and return without synchronising.  HIP launch errors are reported
 *     as TAMM_ERR_HIP.
 *   - Handles are not thread-safe; distinct handles may be used from distinct threads.  The
 *     one-shot plan cache behind tamm_contract is shared and lock-guarded.
 *   - Labels are strings of ASCII letters, one per tensor dimension, no letter twice in one
 *     tensor.  In a contraction every letter appears in exactly two of the three tensors and
 *     binds the same tiled space (same tile sizes and spins) wherever it appears.
 */
#ifndef TAMM_MI_H
#define TAMM_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TAMM_OK = 0,
  TAMM_ERR_ARG = -1,         /* null handle/pointer, negative size, out-of-range value        */
  TAMM_ERR_LABEL = -2,       /* label string malformed, or a letter binds different spaces    */
  TAMM_ERR_SHAPE = -3,       /* rank mismatch between a label string and its tensor           */
  TAMM_ERR_SPARSITY = -4,    /* block structure inconsistent with the request                 */
  TAMM_ERR_UNSUPPORTED = -5, /* valid request the library does not implement                  */
  TAMM_ERR_UNBOUND = -6,     /* tensor storage or workspace not bound, or bound too small     */
  TAMM_ERR_WORKSPACE = -7,   /* workspace pointer misaligned or too small                     */
  TAMM_ERR_HIP = -8          /* a HIP runtime call failed                                     */
} tamm_status;

/* Compute precision of a contraction.  Storage, the final accumulation and the epilogue are
 * always IEEE float64; float32 partial sums are promoted to float64 after every K window of 256
 * flattened summed indices (windows start at each tile pair's first index).
 *   F64    : float64 products and accumulation (v_mfma_f64_16x16x4_f64).
 *   F32    : operands rounded to float32 (round to nearest even) as they are gathered;
 *            float32 matrix-core products (v_mfma_f32_16x16x4_f32) summed in float32 per window.
 *   BF16X3 : each operand split into three bfloat16 terms, x ~ b0 + b1 + b2 with
 *            b_i = bf16(x - b_0 - ... - b_{i-1}) (round to nearest even); the six products
 *            b_i*b_j with i + j <= 2 on bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16),
 *            summed in float32 per window: b0*b0 in one accumulator, the other five in another.
 *   BF16X4_ALIGNED : the leading term of every element is x rounded to the fixed-point grid 8
 *            bits below the maximum exponent of its (row, window) -- exact in bfloat16 -- and the
 *            residual is split into three bfloat16 terms; the ten products of term order
 *            i + j <= 3.  Lead*lead products of one window sum exactly in float32 (kept in their
 *            own accumulator); only the residual products see float32 rounding.
 * The flattened summed indices of an operand block run over the summed labels in the dimension
 * order of the operand that does not hold out's last label, unless only the other operand has a
 * summed label as its last dimension (then in that operand's order); the last label varies
 * fastest.  Windows are consecutive 256-long runs of them within each (block, row), where a row
 * is one value of the operand's remaining (output) labels.
 * The split precisions first write the split operands into the plan workspace, as bfloat16
 * slice planes (slice s of every element in plane s, each block stored [row][k] over its
 * flattened row and K labels) when every operand block's flattened K extent is a multiple of 8,
 * otherwise as one packed 64-bit word of slices per element at the float64 element offsets
 * (tamm_plan_stats.gather_layout bit 3 tells which); their workspace is correspondingly larger. */
typedef enum { TAMM_PREC_F64 = 0, TAMM_PREC_F32 = 1, TAMM_PREC_BF16X3 = 2, TAMM_PREC_BF16X4_ALIGNED = 3 } tamm_precision;

/* User non-zero check (Sec. III-A: a user-defined non-zero check used both for allocation and
 * for operation execution).  Called once per tile tuple when a tensor is created, with the
 * tile index and tile spin of every dimension.  Returns 1 if the block is stored, 0 if it is a
 * structural zero.  When NULL, the spin rule is used: a block of a rank-2k tensor is stored
 * iff the spins of its first k tiles add up to the spins of its last k tiles; blocks of
 * odd-rank tensors are always stored. */
typedef int (*tamm_nonzero_fn)(const int32_t* tile_idx, const int8_t* tile_spin, int32_t rank, void* user);

typedef struct tamm_space tamm_space;
typedef struct tamm_tensor tamm_tensor;
typedef struct tamm_plan tamm_plan;
typedef struct tamm_group tamm_group;

/* Message describing the last failure on the calling thread ("" if none).  Valid until the
 * next library call on this thread. */
const char* tamm_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t tamm_version(void);

/* ------------------------------------------------------------------------------------------
 * Tiled index spaces (Sec. III-A, Fig. 1).
 * ------------------------------------------------------------------------------------------ */

/* Explicit tiling: ntiles tiles of the given positive sizes, covering [0, sum of sizes) in
 * order, each with a spin code (0 = alpha, 1 = beta; NULL = all 0).  Arrays are read during
 * the call only.  ERR_ARG on ntiles <= 0, a non-positive size or a null output pointer. */
int tamm_space_create(const int64_t* tile_sizes, const int8_t* tile_spin, int32_t ntiles, tamm_space** out);

/* Fixed-size tiling of one range (Fig. 1, "tN{N, 10}"): full tiles then one shorter remainder
 * tile, all with spin 0. */
int tamm_space_create_fixed(int64_t extent, int64_t tile, tamm_space** out);

/* Spin-blocked tiling: the alpha sub-space [0, n_alpha) then the beta sub-space, each tiled on
 * its own with tile size min(tile, sub-space size), remainder tile last; tiles never straddle
 * the two sub-spaces.  An empty sub-space contributes no tiles. */
int tamm_space_create_spin(int64_t n_alpha, int64_t n_beta, int64_t tile, tamm_space** out);

/* Number of tiles and total extent. */
int tamm_space_info(const tamm_space* s, int32_t* ntiles, int64_t* extent);

/* Copy out tile sizes, tile start offsets and tile spins (each array ntiles long; any may be
 * NULL). */
int tamm_space_tiles(const tamm_space* s, int64_t* tile_sizes, int64_t* tile_offsets, int8_t* tile_spin);

int tamm_space_destroy(tamm_space* s);

/* ------------------------------------------------------------------------------------------
 * Block-sparse tensors (Sec. III-A; non-zero-only storage, Sec. III-B).
 *
 * Storage layout: the stored blocks back to back in lexicographic order of their tile tuples;
 * each block row-major in the tensor's own dimension order with extents equal to its tile
 * sizes; float64 elements.  A tensor copies what it needs from its spaces, so spaces may be
 * destroyed after tensor creation.
 * ------------------------------------------------------------------------------------------ */

/* rank in [1, 8].  nonzero NULL selects the spin rule (see tamm_nonzero_fn). */
int tamm_tensor_create(tamm_space* const* dims, int32_t rank, tamm_nonzero_fn nonzero, void* user, tamm_tensor** out);

/* Number of stored elements and bytes (stored blocks only). */
int tamm_tensor_numel(const tamm_tensor* t, int64_t* numel);
int tamm_tensor_nbytes(const tamm_tensor* t, size_t* bytes);

/* Stored block table: *nblocks receives the count; if tile_idx is not NULL it receives
 * nblocks*rank tile indices (block-major), and if elem_off is not NULL it receives the element
 * offset of each block in the storage. */
int tamm_tensor_blocks(const tamm_tensor* t, int64_t* nblocks, int32_t* tile_idx, int64_t* elem_off);

/* Bind caller-owned device storage (not owned, not freed by the library).  ERR_UNBOUND if
 * bytes is smaller than tamm_tensor_nbytes; ERR_ARG if dev_ptr is NULL while numel > 0 or is
 * not 8-byte aligned. */
int tamm_tensor_bind(tamm_tensor* t, void* dev_ptr, size_t bytes);

/* Releases the handle (host memory only) and drops the cached one-shot plans (tamm_contract)
 * that name it.  Plans and groups created by the caller must be destroyed first. */
int tamm_tensor_destroy(tamm_tensor* t);

/* ------------------------------------------------------------------------------------------
 * Contraction plans (Sec. III-A, Fig. 3 rule 8; the block non-zero analysis of Sec. III-A).
 *
 * out(out_lbl) = beta * out(out_lbl) + alpha * lhs(lhs_lbl) * rhs(rhs_lbl), summed over the
 * letters of lhs and rhs that out does not carry, on the stored blocks of out.  Operands are
 * read as dense tensors whose unstored blocks are zero.  A stored out block that no tile pair
 * reaches becomes beta * out (0 when beta == 0).  Tile pairs whose out block is not stored
 * (possible only with a user non-zero check) are dropped and counted in the plan statistics.
 * beta == 0 never reads out (NaN/Inf in out do not propagate).
 *
 * The three tensors must outlive the plan; out must not alias lhs or rhs storage.  Plan
 * creation is host-only (no GPU call).
 * ------------------------------------------------------------------------------------------ */
int tamm_plan_create(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                     const tamm_tensor* rhs, const char* rhs_lbl, tamm_precision precision, tamm_plan** plan);

/* Device workspace needed by the plan (bytes, 256-byte aligned start required). */
int tamm_plan_workspace_size(const tamm_plan* p, size_t* bytes);

/* Bind caller-owned device workspace and upload the plan's static tables into it
 * (synchronous copy).  ERR_WORKSPACE if too small or misaligned. */
int tamm_plan_bind_workspace(tamm_plan* p, void* dev_ptr, size_t bytes);

typedef struct {
  int64_t out_blocks;     /* stored blocks of out                                              */
  int64_t candidates;     /* out blocks x tile tuples of the summed labels                     */
  int64_t tasks;          /* surviving tile pairs (host structural count)                      */
  int64_t dropped;        /* surviving pairs whose out block is not stored                     */
  double useful_flops;    /* 2 * sum over surviving tile triples of the product of extents     */
  double algorithmic_bytes; /* 8 * (stored lhs + stored rhs + 2 * stored out elements)         */
  int64_t work_items;     /* output macro-tiles times K splits scheduled by the kernel         */
  int32_t kernel_config;  /* active kernel configuration id                                    */
  int32_t k_splits;       /* K splits per output macro-tile                                    */
  int32_t gather_layout;  /* the operand holding out's last label is B, the other A.
                             bit 1: A's stride-1 label is summed (lanes gather along k);
                             bit 0: the same for B; bit 2: every pair of offset-table entries
                             the gathers group is adjacent in memory, so the float64 kernels
                             load two elements per lane (16-byte loads); bit 3: split-bfloat16
                             precisions store the split operands as slice planes, each block
                             [row][k], because every operand block's K extent is a multiple
                             of 8 (16-byte gathers of 8 slices)                              */
  int32_t xcd_chunk;      /* launch order over the eight dies: work items per die chunk (0: the
                             plain longest-first order); see tamm_plan_set_order                */
  int32_t tile_order;     /* 0: the tiles of a block row by row; 1: grouped by B column panel  */
  int32_t reserved;       /* zero                                                              */
} tamm_plan_stats;

int tamm_plan_stats_get(const tamm_plan* p, tamm_plan_stats* s);

/* Kernel configurations available for this plan's precision: *count receives the number; ids
 * are 0..count-1.  tamm_plan_set_config selects one (the autotuner uses this); k_splits >= 1
 * splits the pair range of the output tiles of the heaviest blocks (largest summed K extent)
 * into that many deterministic partial sums, and lighter blocks' tiles into proportionally
 * fewer (at least one); 0 lets the library choose.  Changing the configuration requires
 * re-querying the workspace size and re-binding. */
int tamm_plan_config_count(const tamm_plan* p, int32_t* count);
int tamm_plan_set_config(tamm_plan* p, int32_t config, int32_t k_splits);
/* Launch order of the work items (results do not depend on it, bit for bit).  The list is
 * longest first; among tiles of equal cost, tile_order 0 keeps the tiles of one output block
 * together, row by row (neighbours share A row panels), and tile_order 1 groups the tiles that
 * read the same B column panel across blocks and rows.  Then the list is cut into chunks of
 * `chunk` items for the chip's eight dies (each with its own L2), chunk c running on die c mod 8;
 * 0 keeps the list as it is; -1 restores the library default (32, or the TAMM_XCD_CHUNK
 * environment variable).  The autotuner searches both after the kernel configuration.  Requires
 * re-binding. */
int tamm_plan_set_order(tamm_plan* p, int32_t tile_order, int32_t chunk);
/* Declare operand `which` (0 = lhs, 1 = rhs) constant (constant != 0) or variable.  For the
 * split-bfloat16 precisions the split of a constant operand, made by the first execution, is
 * reused by later executions as long as the operand stays bound to the same storage and the
 * workspace is not re-bound; the caller promises not to change its values meanwhile (integrals
 * during coupled-cluster iterations, for example).  Calling it again (either value) forces a new
 * split at the next execution, after the caller changed the values.  No effect on other
 * precisions.  Host only. */
int tamm_plan_set_constant(tamm_plan* p, int32_t which, int32_t constant);
/* Human-readable name of a configuration (static string), e.g. "f64_m128n64k16_w2x2_o1". */
const char* tamm_config_name(int32_t precision, int32_t config);

/* Autotuner.  Measures every kernel configuration with K splits 1, 2, 4 and 8 that fits the
 * given workspace (hipEvents on stream; after one warm-up, the fastest of `reps` individually
 * timed executions counts; reps <= 0 means 3), then both tile orders with die chunks of 0, 16, 32,
 * 64 and 128 items (tamm_plan_set_order) for the three fastest of those, then times the three
 * fastest candidates of both passes again in turn (three rounds) and keeps the lowest median;
 * it leaves the plan configured and bound to `workspace`.  The first failing HIP call or launch
 * ends the search and its error is returned.  With K splits s > 1 the tiles of the blocks with
 * the largest summed K extent are split into s parts and lighter blocks' tiles into
 * proportionally fewer (at least one), so the parts cost about the same.  The trial executions
 * run with alpha = 0, beta = 1, so out keeps its values when the operands are finite.  With a non-empty cache_path the result is appended to that text file keyed by the
 * plan's structural signature, and a later call with the same structure reuses it without
 * measuring.  tamm_plan_autotune_workspace_size gives the largest workspace any candidate needs.
 * Synchronises the stream. */
int tamm_plan_autotune_workspace_size(const tamm_plan* p, size_t* bytes);
int tamm_plan_autotune(tamm_plan* p, void* workspace, size_t bytes, void* stream, const char* cache_path, int32_t reps);

/* Enqueue the whole operation on stream: tamm_plan_screen then tamm_plan_contract.
 * Requires bound storage on all three tensors and a bound workspace. */
int tamm_plan_execute(tamm_plan* p, double alpha, double beta, void* stream);

/* The two halves of tamm_plan_execute.  tamm_plan_screen enqueues the GPU tile-pair screening,
 * which writes the surviving pair list of every stored out block into the workspace (the block
 * non-zero analysis of Sec. III-A).  tamm_plan_contract enqueues the contraction kernel (and,
 * with K splits, the ordered reduction) that consumes the last screened pair list; it fails with
 * ERR_UNBOUND if the plan was never screened on its current workspace. */
int tamm_plan_screen(tamm_plan* p, void* stream);
int tamm_plan_contract(tamm_plan* p, double alpha, double beta, void* stream);

/* Copy the GPU screening results of the last execution to the host (synchronises stream):
 * per stored out block (in storage order) the number of surviving pairs; and optionally the
 * K tile-tuple index of every surviving pair (out block major, pairs in lexicographic order,
 * sum(counts) entries).  For tests and statistics. */
int tamm_plan_screen_result(tamm_plan* p, void* stream, int32_t* counts, int32_t* k_tuple_idx);

/* The operand split of a split-bfloat16 plan (BF16X3 or BF16X4_ALIGNED) exactly as its
 * contraction multiplies it.  For operand `which` (0 = lhs, 1 = rhs): one 64-bit word per stored
 * element, at the element's offset in that tensor's storage, holding slice s as bfloat16 bits in
 * bits 16s..16s+15 (three slices: bits 48..63 zero).  The windows of the aligned lead slice are
 * those described at tamm_precision.  `out_dev`: caller-owned device memory of at least 8 bytes
 * per stored element of the operand.  Enqueued on stream.  ERR_UNSUPPORTED for F64 and F32 plans,
 * ERR_UNBOUND without a bound workspace or tensor storage, ERR_WORKSPACE if `bytes` is too small.
 * For tests of the split (its values have an exact definition) and for inspecting it. */
int tamm_plan_split_operand(const tamm_plan* p, int32_t which, void* out_dev, size_t bytes, void* stream);

int tamm_plan_destroy(tamm_plan* p);

/* ------------------------------------------------------------------------------------------
 * One-shot contraction (the assignment and update statements of Sec. III-A, Fig. 3, issued
 * one at a time): out(out_lbl) = beta * out + alpha * lhs(lhs_lbl) * rhs(rhs_lbl), with the
 * semantics of tamm_plan_create / tamm_plan_execute.  The library keeps one plan per distinct
 * (out, lhs, rhs handles, labels, precision) in a process-wide cache, created on first use with
 * the default kernel configuration; tamm_tensor_destroy drops every cached plan naming that
 * tensor.  The cache is guarded by a lock: concurrent calls are serialised on the host.
 *
 * tamm_contract_workspace_size creates the cached plan if needed (host only, no GPU call) and
 * gives the bytes of device workspace tamm_contract needs for it.
 *
 * tamm_contract enqueues the contraction on stream.  `workspace`: caller-owned device memory,
 * 256-byte aligned, of at least that size (ERR_WORKSPACE otherwise).  The plan's tables are
 * uploaded into it (synchronous copy) unless the previous tamm_contract call given this same
 * (workspace, bytes) was for the same contraction, which then reuses them; so the library owns
 * the contents of a workspace between calls, and a caller that writes it or frees and reuses
 * the memory for another purpose calls tamm_contract_cache_clear before passing it again.
 * Handing a workspace (or memory overlapping one an earlier call used) to another contraction
 * synchronises the whole device before the upload, since earlier calls on any stream may still
 * read the old tables.  A separate workspace per contraction keeps repeated calls asynchronous.
 * Errors of plan creation (labels, shapes) are returned as by tamm_plan_create.
 *
 * tamm_contract_cache_count gives the number of cached plans; tamm_contract_cache_clear
 * drops them all (host memory only; work already enqueued is unaffected).
 * ------------------------------------------------------------------------------------------ */
int tamm_contract_workspace_size(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                                 const tamm_tensor* rhs, const char* rhs_lbl, int32_t precision, size_t* bytes);
int tamm_contract(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                  const tamm_tensor* rhs, const char* rhs_lbl, int32_t precision, double alpha, double beta,
                  void* workspace, size_t bytes, void* stream);
int tamm_contract_cache_count(int64_t* plans);
int tamm_contract_cache_clear(void);

/* For callers that cannot allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): tamm_contract with no workspace argument.  The workspace is a
 * file-scope device array of the library, TAMM_NOALLOC_WORKSPACE_BYTES (64 MiB) on each GPU the
 * library runs on, held until the process ends; the call allocates nothing (no
 * hipMalloc, no library allocation).  Same operation, arguments, plan cache and results as
 * tamm_contract on the current device; the stream must belong to that device.  ERR_WORKSPACE,
 * before anything is enqueued, when the contraction needs more workspace than the array holds
 * (host check, tamm_contract_workspace_size).  All calls on one GPU share its array, which keeps
 * the last call's contents (nothing in it needs to start zeroed); calls that overlap in time on one
 * GPU race on it and must be serialised by the caller.  Switching the array between contractions
 * re-uploads the plan tables after draining the device, as tamm_contract does. */
int tamm_contract_noalloc(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                          const tamm_tensor* rhs, const char* rhs_lbl, int32_t precision, double alpha, double beta,
                          void* stream);
#define TAMM_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)

/* ------------------------------------------------------------------------------------------
 * Groups: many independent plans executed together (the single-GPU analogue of running the
 * operations of one scheduler level at once, Sec. III-B): one screening launch over every
 * member, then one persistent contraction launch whose workgroups take output tiles of all
 * members, heaviest first, from a shared counter.  Members must be float64 plans; no member may
 * write storage that another member reads or writes (checked at execution, ERR_ARG).  Plans and
 * their tensors must outlive the group; the group uses its own workspace (the members' own
 * workspaces are not needed).  The group ignores the members' kernel configurations and runs
 * without K splits.  Members are grouped into classes by their gather layout (operand
 * orientations and 8- or 16-byte gathers, see tamm_plan_stats.gather_layout); each class has its
 * own persistent launch, kernel configuration (tile shape) and grid.
 * ------------------------------------------------------------------------------------------ */
int tamm_group_create(tamm_plan* const* plans, int32_t n, tamm_group** g);
int tamm_group_workspace_size(const tamm_group* g, size_t* bytes);
/* Bind caller-owned device workspace (256-byte aligned) and upload the members' static tables
 * (synchronous).  Drops a captured graph. */
int tamm_group_bind_workspace(tamm_group* g, void* dev_ptr, size_t bytes);
/* Select one kernel configuration for every class (-1 = each class's default: the least padding)
 * and the persistent grid size (0 = every resident slot: compute units x workgroups of the
 * configuration that fit on one).  Requires re-binding (the workspace size does not depend on
 * the configuration). */
int tamm_group_set_config(tamm_group* g, int32_t config, int32_t grid);
/* alpha and beta are host arrays of n values, read during the call.  If a graph was captured
 * with the same alpha/beta and the members' storage bindings are unchanged, the graph is
 * replayed; otherwise the kernels are launched directly (and any graph is dropped).  When the
 * coefficients or bindings differ from the previous call, the per-member descriptors in the
 * workspace are rewritten first: the stream is synchronised and the copy is synchronous (earlier
 * launches may still read the old descriptors); calls with unchanged values launch
 * asynchronously. */
int tamm_group_execute(tamm_group* g, const double* alpha, const double* beta, void* stream);
/* Capture the group's launches (counter reset, screening, persistent contraction; no memset or
 * copy nodes) into a hipGraph on an internal stream, with alpha/beta fixed at these values;
 * later tamm_group_execute calls with the same values replay it on their stream. */
int tamm_group_capture(tamm_group* g, const double* alpha, const double* beta, void* stream);
/* Autotuner for groups: for every class separately, every kernel configuration with persistent
 * grids of 1, 2 and 4 workgroups per compute unit and the occupancy-sized grid, the class's launch
 * timed on stream with alpha = 0, beta = 1; keeps each class's fastest and caches them in
 * cache_path (if non-empty) under the group's structural signature.  Needs a bound workspace.
 * Synchronises the stream. */
int tamm_group_autotune(tamm_group* g, void* stream, const char* cache_path, int32_t reps);
/* Configuration and persistent grid (0 = automatic) of the class with the most work items, and
 * the number of work items of all classes. */
int tamm_group_stats(const tamm_group* g, int32_t* config, int32_t* grid, int64_t* work_items);
int tamm_group_destroy(tamm_group* g);

/* ------------------------------------------------------------------------------------------
 * Orbital-energy denominator update (the Jacobi step of CD-CCSD named in Sec. IV-B-1, which
 * turns a residual into amplitudes), prepared once and executed many times:
 *   out[p] = in[p] / D(p),  D(p) = sum of energy[d][p_d] over dims with sign[d] > 0, in
 *   dimension order, then minus energy[d][p_d] over dims with sign[d] < 0, in dimension order
 *   (for R[a,b,i,j] with signs (-,-,+,+): ((e_i + e_j) - e_a) - e_b).  IEEE float64 division
 *   (correctly rounded), over the stored blocks.
 * out and in must have identical block structure and may be the same tensor; sign[d] in
 * {-1, 0, +1} (read during create), at least one non-zero.  The workspace (caller-owned,
 * 256-byte aligned) receives the block metadata at bind time (synchronous copy).
 * energy: host array of rank device pointers (read during the call), each indexing the full
 * untiled range of its dimension; a dimension with sign 0 may pass NULL.
 * ------------------------------------------------------------------------------------------ */
typedef struct tamm_denominator tamm_denominator;
int tamm_denominator_create(tamm_tensor* out, const tamm_tensor* in, const int8_t* sign, tamm_denominator** d);
int tamm_denominator_workspace_size(const tamm_denominator* d, size_t* bytes);
int tamm_denominator_bind_workspace(tamm_denominator* d, void* workspace, size_t bytes);
int tamm_denominator_execute(tamm_denominator* d, const double* const* energy, void* stream);
int tamm_denominator_destroy(tamm_denominator* d);

/* ------------------------------------------------------------------------------------------
 * Element-wise operations of the operation grammar (Sec. III-A, Fig. 3 rules 5-7; the SetOp and
 * AddOp lines of Fig. 4).  Both run over the stored blocks of out only and are bound by HBM
 * bandwidth.
 *
 * tamm_set (SetOp, rule 5, "A(i,l) = alpha"): every stored element of out becomes alpha.
 *   Enqueued on stream.  ERR_UNBOUND if out has no storage.
 *
 * tamm_add_* (AddOp, rules 6-7, "B(i,l) = A(i,l)", "B(i,l) += -1.0 * A(i,l)", and the addition
 *   "A(i,l) += alpha * D(l,i)" with a label permutation):
 *     out(out_lbl) = beta * out(out_lbl) + alpha * in(in_lbl),
 *   where in_lbl is a permutation of out_lbl and every letter binds the same tiled space in both
 *   tensors.  For each stored block of out, the block of in at the permuted tile tuple is read
 *   through the permutation; if that block is not stored it reads as zero (the out block becomes
 *   beta * out).  beta == 0 never reads out.  "=" is beta = 0, "+=" beta = 1, "-=" alpha -> -alpha.
 *   Prepared once (host only), bound to a caller-owned workspace (256-byte aligned; the block and
 *   work tables are copied in synchronously), executed many times.  out and in storage must be
 *   disjoint, except that with identical label strings they may be the same storage (an
 *   in-place scale); ERR_ARG at execution otherwise.  ERR_LABEL if in_lbl is not a permutation of
 *   out_lbl or a letter binds two different spaces; ERR_SHAPE on a rank mismatch.
 * ------------------------------------------------------------------------------------------ */
int tamm_set(tamm_tensor* out, double alpha, void* stream);

typedef struct tamm_add tamm_add;
int tamm_add_create(tamm_tensor* out, const char* out_lbl, const tamm_tensor* in, const char* in_lbl, tamm_add** a);
int tamm_add_workspace_size(const tamm_add* a, size_t* bytes);
int tamm_add_bind_workspace(tamm_add* a, void* workspace, size_t bytes);
int tamm_add_execute(tamm_add* a, double alpha, double beta, void* stream);
int tamm_add_destroy(tamm_add* a);

/* ------------------------------------------------------------------------------------------
 * Scheduler (Sec. III-A, Fig. 4: operations are queued on a scheduler and executed together;
 * Sec. III-B: a dataflow analysis over the queued operations finds the conflicts -- two
 * operations that share a tensor, at least one of them writing it -- and a levelized execution
 * runs the non-conflicting operations of a level together).
 *
 * Queue operations (host only, in program order; nothing runs yet):
 *   tamm_sched_set         SetOp          out = alpha on every stored element
 *   tamm_sched_add         AddOp          out = beta*out + alpha*in(permuted), a prepared tamm_add
 *   tamm_sched_contract    MultOp         out = beta*out + alpha*lhs*rhs, a float64 plan
 *                                         (ERR_UNSUPPORTED for other precisions)
 *   tamm_sched_denominator the denominator update of a prepared tamm_denominator; `energy` (rank
 *                          device pointers, as for tamm_denominator_execute) is copied at queue
 *                          time.
 * The queued objects (plans, AddOps, denominators, their tensors) must outlive the schedule, and
 * AddOps and denominators keep their own bound workspaces; plans' own workspaces are not used.
 *
 * tamm_sched_build (host only) analyses the queue once:
 *   - fusion: a contraction with beta = 1 whose output was last touched by a contraction (or a
 *     fused chain of them) with the same output tensor and the same alpha, whose plan splits the
 *     output into the same rows and columns, and with no operation queued in between that writes
 *     a tensor the chain reads, joins that chain: the chain is one node whose output tiles each
 *     run one K loop over the pairs of every member (same-output fusion).  Members must share
 *     alpha; a term whose coefficient differs is fused by scaling one of its operands upstream.
 *   - AddOp chains: an AddOp with beta = 1 whose output was last touched by an AddOp (or a chain
 *     of them) into the same output tensor joins that chain when its input's storage lies apart
 *     from the output, the output has rank >= 2, no operation queued in between writes a tensor
 *     the chain reads, the chain has fewer than 8 members, and its input ends (stride-1 label) in
 *     the output's last label or in the one other label that the chain's transposed members end
 *     in.  A chain is one node and one launch: out = beta_first*out + the members' alpha*in terms
 *     added in queue order, each output element read and written once (the antisymmetrisers
 *     P(ij)P(ab) written as permuted additions, Fig. 3).  Every product alpha*in and every
 *     partial sum is rounded on its own (no fused multiply-add): the arithmetic of the AddOps
 *     applied one after another in float64.
 *   - levels: nodes, in the order of their last queued operation, each go one level after the
 *     latest earlier node they conflict with (tensors compared by handle and by storage overlap).
 *   Every level runs as one group launch of its contraction nodes (screening, one persistent
 *   contraction launch per gather layout class) followed by its element-wise nodes; the
 *   result equals running the queue in program order (up to the rounding of fused sums).
 * tamm_sched_workspace_size / _bind_workspace: one caller-owned device workspace (256-byte
 *   aligned) for every level's group, sized so that the autotuner's candidates fit, and for the
 *   work items of every AddOp chain; binding copies the static tables in (synchronous).  Executing
 *   a chain fails with ERR_ARG if an input was rebound onto storage that overlaps its output.
 * tamm_sched_autotune: the group autotuner (tamm_group_autotune) on every level (outputs left
 *   unchanged for finite inputs; synchronises the stream).
 * tamm_sched_execute: enqueue every level on stream.  If a graph was captured and every tensor
 *   and energy array is still bound to the same storage, the graph is replayed; otherwise the
 *   launches are issued directly (descriptor refreshes synchronise the stream when bindings moved).
 * tamm_sched_capture: record the whole schedule into one hipGraph (no memset or copy nodes).
 * tamm_sched_info: levels, nodes, and operations inside fused nodes; tamm_sched_op_info: level and
 *   node of queued operation `op` (0-based, queue order).
 * ------------------------------------------------------------------------------------------ */
typedef struct tamm_sched tamm_sched;
int tamm_sched_create(tamm_sched** s);
int tamm_sched_set(tamm_sched* s, tamm_tensor* out, double alpha);
int tamm_sched_add(tamm_sched* s, tamm_add* a, double alpha, double beta);
int tamm_sched_contract(tamm_sched* s, tamm_plan* p, double alpha, double beta);
int tamm_sched_denominator(tamm_sched* s, tamm_denominator* d, const double* const* energy);
int tamm_sched_build(tamm_sched* s);
int tamm_sched_workspace_size(const tamm_sched* s, size_t* bytes);
int tamm_sched_bind_workspace(tamm_sched* s, void* workspace, size_t bytes);
int tamm_sched_autotune(tamm_sched* s, void* stream, const char* cache_path, int32_t reps);
int tamm_sched_execute(tamm_sched* s, void* stream);
int tamm_sched_capture(tamm_sched* s, void* stream);
int tamm_sched_info(const tamm_sched* s, int32_t* levels, int32_t* nodes, int32_t* fused_ops);
int tamm_sched_op_info(const tamm_sched* s, int32_t op, int32_t* level, int32_t* node);
int tamm_sched_destroy(tamm_sched* s);

/* ------------------------------------------------------------------------------------------
 * Row views (the view tensors of Sec. III-A: a tensor of another shape over existing storage,
 * no allocation).  *out receives a new tensor handle whose first dimension holds tiles
 * [tile_lo, tile_hi) of parent's first dimension (the other dimensions, the block rule and the
 * order of the blocks are parent's), and *elem_offset the element offset in parent's storage at
 * which the view's storage starts: parent's blocks whose first tile lies in the range are
 * contiguous there (lexicographic block order).  Bind the view to parent's storage plus
 * 8 * *elem_offset bytes.  Host only; the view does not track later rebinding of parent.
 * ERR_ARG on an empty or out-of-range tile range.  Destroy with tamm_tensor_destroy.
 * ------------------------------------------------------------------------------------------ */
int tamm_tensor_view_rows(const tamm_tensor* parent, int32_t tile_lo, int32_t tile_hi, tamm_tensor** out,
                          int64_t* elem_offset);

/* ------------------------------------------------------------------------------------------
 * Particle-particle ladder over integrals rebuilt from Cholesky vectors (Sec. IV-A-1, Eq. (cc12);
 * the integral tensor as a lambda tensor of Sec. III-A, computed where it is used):
 *
 *   R[a,b,i,j] = beta * R[a,b,i,j] + alpha * sum_cd V[a,b,c,d] T[c,d,i,j],
 *   V[a,b,c,d] = sum_L B[a,c,L] B[b,d,L] - B[a,d,L] B[b,c,L].
 *
 * R and T: rank 4 (vir, vir, occ, occ), one virtual space for both leading dimensions of R, T
 * and B, R and T sharing the occupied spaces.  B: rank 3 (vir, vir, aux), the vectors (pq|L),
 * stored with whatever non-zero check it was created with (spin-diagonal for molecular
 * integrals); unstored blocks read as zero.  V is never formed: the operation runs as
 *   Tm[c,d,i,j] = T[c,d,i,j] - T[d,c,i,j]                          (two AddOps, HBM-bound)
 * and, for each strip of `strip_tiles` tiles of a (0 = one tile per strip),
 *   G[a,c,b,d]  = sum_L B[a,c,L] B[b,d,L]                          (float64 matrix cores)
 *   R[a,b,i,j]  = beta R + alpha sum_cd G[a,c,b,d] Tm[c,d,i,j]     (float64 matrix cores)
 * which equals the definition (rename c <-> d in the second term).  G is stored only on the
 * blocks where some auxiliary tile pairs two stored B blocks.
 * Workspace (caller-owned, 256-byte aligned): Tm, one strip of G, and the tables of the strips'
 * plans (sized for any configuration the autotuner may pick); binding copies tables in
 * (synchronous).  R, T and B must outlive the handle and keep their storage disjoint from each
 * other and from the workspace; the handle reads their current bindings at every call.
 * Execute enqueues everything on stream.  Autotune runs the plan autotuner on every strip's two
 * plans (R unchanged for finite values; synchronises the stream).  Stats: useful flops of the pair
 * products and of the strip ladders, strips, largest G strip and Tm in elements (any pointer may
 * be NULL).  strip_plans exposes a strip's two plans (owned by the handle) for inspection.
 * ERR_SHAPE / ERR_LABEL when the tensors do not fit the pattern above.
 * ------------------------------------------------------------------------------------------ */
typedef struct tamm_chol tamm_chol;
int tamm_chol_ladder_create(tamm_tensor* r, const tamm_tensor* t, const tamm_tensor* b, int32_t strip_tiles,
                            tamm_chol** out);
int tamm_chol_ladder_workspace_size(const tamm_chol* c, size_t* bytes);
int tamm_chol_ladder_bind_workspace(tamm_chol* c, void* workspace, size_t bytes);
int tamm_chol_ladder_execute(tamm_chol* c, double alpha, double beta, void* stream);
int tamm_chol_ladder_autotune(tamm_chol* c, void* stream, const char* cache_path, int32_t reps);
int tamm_chol_ladder_stats(const tamm_chol* c, double* build_flops, double* ladder_flops, int64_t* strips,
                           int64_t* g_max_elements, int64_t* tm_elements);
int tamm_chol_ladder_strip_plans(const tamm_chol* c, int32_t strip, tamm_plan** build, tamm_plan** ladder);
int tamm_chol_ladder_destroy(tamm_chol* c);

/* ------------------------------------------------------------------------------------------
 * Diagnostic: execute one matrix-core instruction on one wave with caller data (device
 * pointers, enqueued on stream), for tests of its lane layout and of the rounding of its float32
 * accumulation on inputs whose exact results are known.  The contraction path never calls it.
 *   op 0: v_mfma_f32_16x16x4_f32    a, b: 64 floats (one per lane); c, d: 256 floats (4 per lane)
 *   op 1: v_mfma_f32_16x16x32_bf16  a, b: 512 bfloat16 (8 per lane);  c, d: 256 floats
 *   op 2: v_mfma_f32_32x32x16_bf16  a, b: 512 bfloat16 (8 per lane);  c, d: 1024 floats (16 per lane)
 *   op 3: v_mfma_f32_32x32x2_f32    a, b: 64 floats;                   c, d: 1024 floats
 * d receives the result registers, lane-major like c.  ERR_ARG on an unknown op or a null pointer.
 * ------------------------------------------------------------------------------------------ */
int tamm_diag_mfma(int32_t op, const void* a, const void* b, const float* c, float* d, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TAMM_MI_H */
