// Mixed-precision contraction kernels for gfx950: the bulk products run on float32 or bfloat16
// matrix cores with float32 accumulation inside K windows of 256, and every window's partial
// sums are promoted into float64 accumulators; the epilogue (beta*C + alpha*acc) is float64.
//
//   float32 (v_mfma_f32_16x16x4_f32): operands rounded to float32 (round to nearest even) while
//       they are gathered into LDS.
//   split bfloat16 (v_mfma_f32_16x16x32_bf16): each operand is first split by k_prep_split into
//       bfloat16 slices, stored either as slice planes (plane s holds slice s of every element,
//       each block [row][k]; used when every block's K extent is a multiple of 8) or as one packed
//       64-bit word per element (slice s in bits 16s..16s+15) at the float64 element offsets; the
//       contraction then multiplies selected slice pairs.
//         - three plain slices (x ~ b0 + b1 + b2, b_i = bf16(x - b_0 - ... - b_{i-1})), the six
//           products b_i*b_j with i + j <= 2; b0*b0 in one float32 accumulator per window, the
//           five smaller products in another;
//         - aligned lead: slice 0 is x rounded to a fixed-point grid of 8 bits below the maximum
//           exponent of its (row, window) -- an integer of magnitude <= 256 times a power of two,
//           exact in bfloat16 -- and slices 1..3 are bfloat16 slices of the residual; the ten
//           products of slice order i + j <= 3.  Within one 256-long window every lead*lead
//           product is an integer of at most 16 bits times the same power of two for a given
//           (m, n), so their sum (at most 2^24 in magnitude) is exact in float32; it is kept in
//           its own accumulator, and only the small residual products see float32 rounding.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "internal.h"
#include "mixed.h"

namespace tamm {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------------
// operand split
// ---------------------------------------------------------------------------------------------
// Round to nearest even at 8 significant bits (the bfloat16 precision), on the float64 bit pattern:
// adding half a unit of the kept part (less one ulp when the kept part is even) and clearing the
// 45 dropped mantissa bits rounds to nearest even; a carry out of the mantissa steps the exponent,
// which is the correctly rounded result.  Magnitudes below 2^-100 are flushed to zero (far below
// anything the slices can carry).  Finite inputs only.
__device__ __forceinline__ double round_bf16(double x) {
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  if (((u >> 52) & 0x7FF) < 1023 - 100) return 0.0;
  u += 0x00000FFFFFFFFFFFull + ((u >> 45) & 1u);
  u &= ~0x00001FFFFFFFFFFFull;
  return __builtin_bit_cast(double, u);
}

// Bits of a value that is exactly representable in bfloat16.
__device__ __forceinline__ uint64_t bf16_bits(double y) {
  const float f = (float)y;  // exact: y has at most 8 significant bits and a float exponent
  return (uint64_t)(__float_as_uint(f) >> 16);
}

__device__ __forceinline__ uint64_t split_plain(double x) {
  const double b0 = round_bf16(x);
  const double r1 = x - b0;
  const double b1 = round_bf16(r1);
  const double b2 = round_bf16(r1 - b1);
  return bf16_bits(b0) | (bf16_bits(b1) << 16) | (bf16_bits(b2) << 32);
}

// 2^p for -1022 <= p <= 1023
__device__ __forceinline__ double pow2(int p) { return __builtin_bit_cast(double, (uint64_t)(p + 1023) << 52); }

// Grid of a (row, window) with maximum magnitude mx: the exponent e with 2^(e-1) <= mx < 2^e
// (taken as -1000 for smaller maxima, whose slices are all zero in bfloat16 anyway); the lead
// slice is x rounded to multiples of 2^(e-8).
__device__ __forceinline__ int window_exponent(double mx) {
  const int bexp = (int)((__builtin_bit_cast(uint64_t, mx) >> 52) & 0x7FF);
  return max(bexp - 1022, -1000);
}

__device__ __forceinline__ uint64_t split_aligned(double x, int e) {
  const double lead = rint(x * pow2(8 - e)) * pow2(e - 8);  // an integer of magnitude <= 256 times 2^(e-8)
  const double r = x - lead;                                // exact
  const double s1 = round_bf16(r);
  const double r2 = r - s1;
  const double s2 = round_bf16(r2);
  const double s3 = round_bf16(r2 - s2);
  return bf16_bits(lead) | (bf16_bits(s1) << 16) | (bf16_bits(s2) << 32) | (bf16_bits(s3) << 48);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int find_block(const PrepBlock* blocks, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blocks[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Planes layout, lanes along k: a wave converts kPrepUnroll consecutive (block, row, window)
// items, 4 consecutive k of one row per lane and item.  The loads of all its items are issued
// before any of them is converted, so each wave keeps kPrepUnroll windows of reads in flight.
constexpr int kPrepUnroll = 4;

__device__ __forceinline__ void prep_planes_kc(const PrepParams& P, int64_t first, int lane) {
  static_assert(kSplitWindow == 4 * 64, "a wave converts one window, 4 k per lane");
  typedef double d2_t __attribute__((ext_vector_type(2)));
  const int32_t* __restrict__ pool = P.pool;
  double x[kPrepUnroll][4];
  int64_t pos[kPrepUnroll];
  bool live[kPrepUnroll];
#pragma unroll
  for (int u = 0; u < kPrepUnroll; ++u) {
    const int64_t item = first + u;
    live[u] = false;
    pos[u] = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) x[u][i] = 0.0;
    if (item >= P.n_items) continue;  // wave-uniform
    const PrepBlock pb = P.blocks[find_block(P.blocks, P.n_blocks, item)];
    const int64_t local = item - pb.item0;
    const int k0 = (int)(local % pb.nwin) * kSplitWindow, row = (int)(local / pb.nwin);
    const int k = k0 + 4 * lane;
    const int k1 = min(pb.kext, k0 + kSplitWindow);
    pos[u] = pb.off + (int64_t)row * pb.kext + k;
    live[u] = k < k1;  // k1 is a multiple of 8: all four k are inside or all outside
    if (!live[u]) continue;
    const int64_t rowoff = pb.off + pool[pb.tab_row + row];
    int32_t t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = pool[pb.tab_k + k + i];
    const int64_t a = rowoff + t[0];
    if (t[1] == t[0] + 1 && t[2] == t[0] + 2 && t[3] == t[0] + 3 && (a & 1) == 0) {
      // four consecutive elements at a 16-byte boundary: two 16-byte loads
      const d2_t lo = *reinterpret_cast<const d2_t*>(P.x + a), hi = *reinterpret_cast<const d2_t*>(P.x + a + 2);
      x[u][0] = lo[0];
      x[u][1] = lo[1];
      x[u][2] = hi[0];
      x[u][3] = hi[1];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) x[u][i] = P.x[rowoff + t[i]];
    }
  }
  const int ns = P.aligned ? 4 : 3;
  unsigned short* __restrict__ out = static_cast<unsigned short*>(P.out);
#pragma unroll
  for (int u = 0; u < kPrepUnroll; ++u) {
    if (first + u >= P.n_items) break;  // wave-uniform
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) mx = fmax(mx, fabs(x[u][i]));
    const int e = window_exponent(wave_max(mx));
    if (!live[u]) continue;
    uint64_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = P.aligned ? split_aligned(x[u][i], e) : split_plain(x[u][i]);
    for (int sl = 0; sl < ns; ++sl) {
      uint64_t v = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) v |= ((w[i] >> (16 * sl)) & 0xFFFFull) << (16 * i);
      *reinterpret_cast<uint64_t*>(out + sl * P.plane_stride + pos[u]) = v;
    }
  }
}

// One wave per item.  ROWS_ALONG_LANES = false: the operand's stride-1 label is summed, so an item
// is one (block, row, window) and the lanes run along k (coalesced); the window maximum is a wave
// reduction.  ROWS_ALONG_LANES = true: an item is (block, 64 rows, window), each lane owns a row
// and walks the window (lanes coalesce along the row label).
template <bool ROWS_ALONG_LANES>
__global__ __launch_bounds__(256) void k_prep_split(PrepParams P) {
  const int lane = threadIdx.x & 63;
  if (!ROWS_ALONG_LANES && P.planes) {
    prep_planes_kc(P, ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kPrepUnroll, lane);
    return;
  }
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= P.n_items) return;
  const int b = find_block(P.blocks, P.n_blocks, item);
  const PrepBlock pb = P.blocks[b];
  const int64_t local = item - pb.item0;
  const int win = (int)(local % pb.nwin);
  const int rg = (int)(local / pb.nwin);
  const int k0 = win * kSplitWindow;
  const int k1 = min(pb.kext, k0 + kSplitWindow);
  const int32_t* __restrict__ pool = P.pool;
  if (P.planes) {
    // planes layout (every K extent a multiple of 8): a lane converts 4 (lanes along k) or 8
    // (lanes along rows) consecutive k of one row and writes each slice plane's part at once
    const int ns = P.aligned ? 4 : 3;
    unsigned short* __restrict__ out = static_cast<unsigned short*>(P.out);
    {  // lanes along rows (lanes along k: prep_planes_kc)
      const int row = rg * 64 + lane;
      if (row >= pb.rows) return;
      const int64_t rowoff = pb.off + pool[pb.tab_row + row];
      double mx = 0.0;
      if (P.aligned)
        for (int k = k0; k < k1; ++k) mx = fmax(mx, fabs(P.x[rowoff + pool[pb.tab_k + k]]));
      const int e = window_exponent(mx);
      for (int k = k0; k < k1; k += 8) {
        uint64_t w[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const double v = P.x[rowoff + pool[pb.tab_k + k + i]];
          w[i] = P.aligned ? split_aligned(v, e) : split_plain(v);
        }
        const int64_t pos = pb.off + (int64_t)row * pb.kext + k;
        for (int sl = 0; sl < ns; ++sl) {
          u4_t v;
#pragma unroll
          for (int h = 0; h < 4; ++h)
            v[h] = (uint32_t)((w[2 * h] >> (16 * sl)) & 0xFFFFu) | ((uint32_t)((w[2 * h + 1] >> (16 * sl)) & 0xFFFFu) << 16);
          *reinterpret_cast<u4_t*>(out + sl * P.plane_stride + pos) = v;
        }
      }
    }
    return;
  }
  if (!ROWS_ALONG_LANES) {
    const int row = rg;
    const int64_t rowoff = pb.off + pool[pb.tab_row + row];
    double x[kSplitWindow / 64];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < kSplitWindow / 64; ++j) {
      const int k = k0 + lane + 64 * j;
      x[j] = (k < k1) ? P.x[rowoff + pool[pb.tab_k + k]] : 0.0;
      mx = fmax(mx, fabs(x[j]));
    }
    const int e = window_exponent(wave_max(mx));
#pragma unroll
    for (int j = 0; j < kSplitWindow / 64; ++j) {
      const int k = k0 + lane + 64 * j;
      if (k < k1)
        static_cast<uint64_t*>(P.out)[rowoff + pool[pb.tab_k + k]] = P.aligned ? split_aligned(x[j], e) : split_plain(x[j]);
    }
  } else {
    const int row = rg * 64 + lane;
    if (row >= pb.rows) return;
    const int64_t rowoff = pb.off + pool[pb.tab_row + row];
    double mx = 0.0;
    if (P.aligned)
      for (int k = k0; k < k1; ++k) mx = fmax(mx, fabs(P.x[rowoff + pool[pb.tab_k + k]]));
    const int e = window_exponent(mx);
    for (int k = k0; k < k1; ++k) {
      const int64_t a = rowoff + pool[pb.tab_k + k];
      const double v = P.x[a];
      static_cast<uint64_t*>(P.out)[a] = P.aligned ? split_aligned(v, e) : split_plain(v);
    }
  }
}

hipError_t launch_prep_split(const PrepParams& p, bool rows_along_lanes, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  const int64_t per_block = (!rows_along_lanes && p.planes) ? 4 * kPrepUnroll : 4;  // items per workgroup
  const dim3 g((unsigned)((p.n_items + per_block - 1) / per_block)), b(256);
  if (rows_along_lanes) hipLaunchKernelGGL(k_prep_split<true>, g, b, 0, s, p);
  else hipLaunchKernelGGL(k_prep_split<false>, g, b, 0, s, p);
  return hipGetLastError();
}

// Epilogue shared by the mixed kernels: float64 accumulators in the float32 MFMA layout (D[m][n]
// in lane n + 16*(m/4), register m%4).
template <int MT, int NT, int WM, int WN, int FM, int FN>
__device__ __forceinline__ void epilogue_f32layout(const ProblemDesc& pr, const WorkItem& w, const OutBlockDesc& blk,
                                                   d4_t (&acc)[FM][FN], int wm, int wn, int lr, int lq) {
  if (item_nsplit(w) > 1) {
    double* part = pr.partial + ((int64_t)w.tile + item_split(w)) * (MT * NT);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[(wm * WM + i * 16 + 4 * lq + r) * NT + wn * WN + j * 16 + lr] = acc[i][j][r];
    return;
  }
  // through out's offset tables: every table entry first (the tables are padded, so rows and
  // columns past the block read in bounds), then per row block the old values (beta != 0), then
  // the results, so that no load waits behind the use of another
  const double alpha = pr.alpha, beta = pr.beta;
  const int32_t* pool = pr.pool;
  __attribute__((address_space(1))) double* __restrict__ Cg = (__attribute__((address_space(1))) double*)pr.C;
  const int mb = w.m0 + wm * WM + 4 * lq, nb = w.n0 + wn * WN + lr;
  int32_t rt[FM][4], ct[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) rt[i][r] = pool[blk.c_tabM + mb + i * 16 + r];
#pragma unroll
  for (int j = 0; j < FN; ++j) ct[j] = pool[blk.c_tabN + nb + j * 16];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    double old[4][FN];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bool live = mb + i * 16 + r < blk.mext && nb + j * 16 < blk.next;
        old[r][j] = (beta != 0.0 && live) ? Cg[blk.c_off + rt[i][r] + ct[j]] : 0.0;
      }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bool live = mb + i * 16 + r < blk.mext && nb + j * 16 < blk.next;
        const double v = alpha * acc[i][j][r];
        if (live) Cg[blk.c_off + rt[i][r] + ct[j]] = (beta == 0.0) ? v : beta * old[r][j] + v;
      }
  }
}

// ---------------------------------------------------------------------------------------------
// float32 products (v_mfma_f32_16x16x4_f32), float32 window sums promoted to float64.
// ---------------------------------------------------------------------------------------------
template <int MT, int NT, int KT, int WGM, int WGN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(64 * WGM * WGN) void k_contract_f32(ContractParams P) {
  constexpr int NTHR = 64 * WGM * WGN;
  constexpr int WM = MT / WGM, WN = NT / WGN, FM = WM / 16, FN = WN / 16;
  constexpr int LD = KT + 4;  // floats; rows 16 apart land on distinct banks for the 4 k lanes
  static_assert(kSplitWindow % KT == 0, "chunks tile the promotion window");
  using G = Gather<MT, NT, KT, NTHR, A_KC, B_KC, double>;
  __shared__ float As[2][MT * LD];
  __shared__ float Bs[2][NT * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM, lr = lane & 15, lq = lane >> 4;
  const int a_frag = (wm * WM + lr) * LD + lq, b_frag = (wn * WN + lr) * LD + lq;
  const int item = blockIdx.x;
  if (item >= P.n_work) return;
  const WorkItem w = wave_uniform(sload(P.work + item));
  const ProblemDesc pr = wave_uniform(P.probs ? sload(P.probs + w.prob) : P.single);
  const OutBlockDesc blk = wave_uniform(sload(pr.blocks + w.ob));
  const int32_t* __restrict__ pool = pr.pool;
  const PairDesc* __restrict__ pairs = pr.pairs + blk.pair_base;
  const int cnt = wave_uniform(gload(pr.counts + w.ob));
  const int nsplit = item_nsplit(w), split = item_split(w);
  const int pb = (int)(((int64_t)cnt * split) / nsplit), pe = (int)(((int64_t)cnt * (split + 1)) / nsplit);
  G g;
  g.init(tid);
  d4_t acc[FM][FN];
  f4_t part[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc[i][j] = (d4_t){0.0, 0.0, 0.0, 0.0};
      part[i][j] = (f4_t){0.f, 0.f, 0.f, 0.f};
    }
  if (pb < pe) {
    auto store = [&](int b) {
#pragma unroll
      for (int e = 0; e < G::AE; ++e) As[b][g.a_lds_row(e) * LD + g.a_lds_k(e)] = (float)g.ra[e];
#pragma unroll
      for (int e = 0; e < G::BE; ++e) Bs[b][g.b_lds_row(e) * LD + g.b_lds_k(e)] = (float)g.rb[e];
    };
    auto compute = [&](int b, bool flush, auto&& stage, auto&& post) {
      const float* as = As[b] + a_frag;
      const float* bs = Bs[b] + b_frag;
      float af[2][FM], bf[2][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[0][i] = as[i * 16 * LD];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[0][j] = bs[j * 16 * LD];
      __builtin_amdgcn_s_setprio(1);  // MFMA phase first when waves of two workgroups compete
#pragma unroll
      for (int s = 0; s < KT / 4; ++s) {  // zeros beyond a ragged chunk's K extent
        const int cur = s & 1, nxt = cur ^ 1;
        if (s + 1 < KT / 4) {
#pragma unroll
          for (int i = 0; i < FM; ++i) af[nxt][i] = as[i * 16 * LD + 4 * (s + 1)];
#pragma unroll
          for (int j = 0; j < FN; ++j) bf[nxt][j] = bs[j * 16 * LD + 4 * (s + 1)];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[cur][i], bf[cur][j], part[i][j], 0, 0, 0);
        if (s == 0) stage();
      }
      __builtin_amdgcn_s_setprio(0);
      post();  // bookkeeping of the next chunk while the MFMAs drain
      if (flush) {  // end of a promotion window or of a pair: float32 sums into float64
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              acc[i][j][r] += (double)part[i][j][r];
              part[i][j][r] = 0.f;
            }
      }
    };
    chunk_pipeline<KT, kSplitWindow>(g, pairs, pb, pe, pool, pr.A, pr.B, w.m0, w.n0, blk.mext, blk.next, store, compute);
  }
  epilogue_f32layout<MT, NT, WM, WN, FM, FN>(pr, w, blk, acc, wm, wn, lr, lq);
}

// ---------------------------------------------------------------------------------------------
// Gather of split operands in the planes layout: plane s holds bfloat16 slice s of every element,
// each block as [row][k] (flattened M or N rows, flattened K, k fastest) at the block's element
// offset.  A lane moves 8 consecutive k of one row and plane with one 16-byte load and one
// 16-byte LDS store.  The planner uses this layout only when every operand block's K extent is a
// multiple of 8, so a group of 8 is either inside the block or wholly past its K extent; groups
// past the rows or the K extent read zeros (offset beyond the buffer resource).
// Same interface as Gather, for chunk_pipeline.
// ---------------------------------------------------------------------------------------------
// LDS layout of a chunk in the planes layout: per plane, the 16-byte units (8 k of one row) are
// stored k-group major, unit (k-group q, row r) at q*ROWS + (r ^ 2q).  An MFMA operand read (16
// rows, one k-group per 16 lanes) is then a permutation of one aligned 256-byte block per 16
// lanes, which the LDS serves without bank conflicts; the gather's stores (4 lanes per row, one
// k-group each) put every 8 consecutive lanes on 8 distinct 16-byte bank groups.
template <int ROWS>
__device__ __forceinline__ int lds_unit(int r, int q) { return q * ROWS + (r ^ (2 * q)); }

template <int MT, int NT, int KT, int NTHR, int NS>
struct PlaneGather {
  static constexpr int KG = KT / 8;           // 16-byte groups per row of a chunk
  static constexpr int AJ = (MT * KG + NTHR - 1) / NTHR;  // loads per plane and thread
  static constexpr int BJ = (NT * KG + NTHR - 1) / NTHR;
  static_assert(KT % 8 == 0 && (MT * KG % NTHR == 0 || NTHR % (MT * KG) == 0) &&
                    (NT * KG % NTHR == 0 || NTHR % (NT * KG) == 0), "plane gather mapping");
  // a load slot past the tile (fewer 16-byte groups than threads): whole waves skip it
  __device__ static bool a_live(int p) { return MT * KG % NTHR == 0 || p < MT * KG; }
  __device__ static bool b_live(int p) { return NT * KG % NTHR == 0 || p < NT * KG; }
  static constexpr uint32_t kPast = 0x80000000u;  // byte offset beyond every block

  int tid;
  int64_t a_plane, b_plane;
  const __bf16* a_base;
  const __bf16* b_base;
  int m0, n0, mext, next, kext, kbase;
  u4_t ra[NS][AJ], rb[NS][BJ];

  __device__ void init(int t, int64_t ap, int64_t bp) {
    tid = t;
    a_plane = ap;
    b_plane = bp;
  }
  __device__ void setup_pair(const PairDesc& d, const int32_t*, const __bf16* A, const __bf16* B, int m0_, int n0_,
                             int mext_, int next_) {
    a_base = A + d.a_off;
    b_base = B + d.b_off;
    m0 = m0_;
    n0 = n0_;
    mext = mext_;
    next = next_;
    kext = d.kext;
  }
  __device__ void load_tables(const PairDesc&, const int32_t*, int kb) { kbase = kb; }
  __device__ void load_data() {
    const uint32_t a_bytes = (uint32_t)mext * (uint32_t)kext * 2u, b_bytes = (uint32_t)next * (uint32_t)kext * 2u;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const __amdgpu_buffer_rsrc_t ar = block_rsrc(a_base + sl * a_plane, a_bytes);
      const __amdgpu_buffer_rsrc_t br = block_rsrc(b_base + sl * b_plane, b_bytes);
#pragma unroll
      for (int j = 0; j < AJ; ++j) {
        const int p = tid + j * NTHR, r = m0 + p / KG, k = kbase + 8 * (p % KG);
        if (!a_live(p)) continue;
        const uint32_t off = (r < mext && k < kext) ? (uint32_t)(r * kext + k) * 2u : kPast;
        ra[sl][j] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(ar, (int)off, 0, 0));
      }
#pragma unroll
      for (int j = 0; j < BJ; ++j) {
        const int p = tid + j * NTHR, r = n0 + p / KG, k = kbase + 8 * (p % KG);
        if (!b_live(p)) continue;
        const uint32_t off = (r < next && k < kext) ? (uint32_t)(r * kext + k) * 2u : kPast;
        rb[sl][j] = __builtin_bit_cast(u4_t, __builtin_amdgcn_raw_buffer_load_b128(br, (int)off, 0, 0));
      }
    }
  }
  // LDS position (row, first k) of load j
  __device__ int lds_row(int j) const { return (tid + j * NTHR) / KG; }
  __device__ int lds_k(int j) const { return 8 * ((tid + j * NTHR) % KG); }
};

// ---------------------------------------------------------------------------------------------
// split bfloat16 products (v_mfma_f32_16x16x32_bf16).  LDS holds NS slice planes per operand: in
// the planes layout as 16-byte units placed by lds_unit; in the packed layout as [row][k] bfloat16
// with a row stride of KT+8 elements (an odd number of 16-byte units).
// ---------------------------------------------------------------------------------------------
template <int MT, int NT, int KT, int WGM, int WGN, bool ALIGNED, bool A_KC, bool B_KC, bool PLANES>
__global__ __launch_bounds__(64 * WGM * WGN) void k_contract_bf16s(ContractParams P) {
  constexpr int NTHR = 64 * WGM * WGN;
  constexpr int WM = MT / WGM, WN = NT / WGN, FM = WM / 16, FN = WN / 16;
  constexpr int NS = ALIGNED ? 4 : 3;
  // LDS rows of KT bfloat16.  Packed layout: padded to an odd number of 16-byte units.  Planes
  // layout: a plane of MT (NT) rows x KT holds MT*KT elements, unit (q, r) at lds_unit.
  constexpr int LD = PLANES ? KT : KT + 8;
  static_assert(KT % 32 == 0 && kSplitWindow % KT == 0, "chunks of whole MFMA k-steps tile the window");
  static_assert(PLANES ? KT == 32 : ((LD * 2) / 16) % 2 == 1, "LDS row layout");
  using G = std::conditional_t<PLANES, PlaneGather<MT, NT, KT, NTHR, NS>, Gather<MT, NT, KT, NTHR, A_KC, B_KC, uint64_t>>;
  using E = std::conditional_t<PLANES, __bf16, uint64_t>;  // element type of the split operands
  __shared__ __attribute__((aligned(16))) __bf16 As[2][NS * MT * LD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][NS * NT * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM, lr = lane & 15, lq = lane >> 4;
  // operand read offsets of this lane (row block i / j, MFMA k-step 0)
  int a_frag[FM], b_frag[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int r = wm * WM + i * 16 + lr;
    a_frag[i] = PLANES ? 8 * lds_unit<MT>(r, lq) : r * LD + 8 * lq;
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int r = wn * WN + j * 16 + lr;
    b_frag[j] = PLANES ? 8 * lds_unit<NT>(r, lq) : r * LD + 8 * lq;
  }
  const int item = blockIdx.x;
  if (item >= P.n_work) return;
  const WorkItem w = wave_uniform(sload(P.work + item));
  const ProblemDesc pr = wave_uniform(P.probs ? sload(P.probs + w.prob) : P.single);
  const OutBlockDesc blk = wave_uniform(sload(pr.blocks + w.ob));
  const int32_t* __restrict__ pool = pr.pool;
  const PairDesc* __restrict__ pairs = pr.pairs + blk.pair_base;
  const E* Ap = reinterpret_cast<const E*>(pr.A);
  const E* Bp = reinterpret_cast<const E*>(pr.B);
  const int cnt = wave_uniform(gload(pr.counts + w.ob));
  const int nsplit = item_nsplit(w), split = item_split(w);
  const int pb = (int)(((int64_t)cnt * split) / nsplit), pe = (int)(((int64_t)cnt * (split + 1)) / nsplit);
  G g;
  if constexpr (PLANES) g.init(tid, pr.a_plane, pr.b_plane);
  else g.init(tid);
  d4_t acc[FM][FN];
  f4_t lead[FM][FN], rest[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc[i][j] = (d4_t){0.0, 0.0, 0.0, 0.0};
      lead[i][j] = (f4_t){0.f, 0.f, 0.f, 0.f};
      rest[i][j] = (f4_t){0.f, 0.f, 0.f, 0.f};
    }
  if (pb < pe) {
    auto store = [&](int b) {
      if constexpr (PLANES) {  // 8 slices of one plane per 16-byte store
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
          for (int j = 0; j < G::AJ; ++j) {
            if (!G::a_live(tid + j * NTHR)) continue;
            *reinterpret_cast<u4_t*>(&As[b][s * MT * LD + 8 * lds_unit<MT>(g.lds_row(j), g.lds_k(j) / 8)]) = g.ra[s][j];
          }
#pragma unroll
          for (int j = 0; j < G::BJ; ++j) {
            if (!G::b_live(tid + j * NTHR)) continue;
            *reinterpret_cast<u4_t*>(&Bs[b][s * NT * LD + 8 * lds_unit<NT>(g.lds_row(j), g.lds_k(j) / 8)]) = g.rb[s][j];
          }
        }
      } else {  // one packed element: its NS slices to NS planes
        unsigned short* As16 = reinterpret_cast<unsigned short*>(As[b]);
        unsigned short* Bs16 = reinterpret_cast<unsigned short*>(Bs[b]);
#pragma unroll
        for (int e = 0; e < G::AE; ++e) {
          const int o = g.a_lds_row(e) * LD + g.a_lds_k(e);
#pragma unroll
          for (int s = 0; s < NS; ++s) As16[s * MT * LD + o] = (unsigned short)(g.ra[e] >> (16 * s));
        }
#pragma unroll
        for (int e = 0; e < G::BE; ++e) {
          const int o = g.b_lds_row(e) * LD + g.b_lds_k(e);
#pragma unroll
          for (int s = 0; s < NS; ++s) Bs16[s * NT * LD + o] = (unsigned short)(g.rb[e] >> (16 * s));
        }
      }
    };
    auto compute = [&](int b, bool flush, auto&& stage, auto&& post) {
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int st = 0; st < KT / 32; ++st) {  // zeros beyond a ragged chunk's K extent
        bf8_t af[NS][FM], bfr[NS][FN];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
            af[s][i] = *reinterpret_cast<const bf8_t*>(&As[b][s * MT * LD + a_frag[i] + 32 * st]);
#pragma unroll
          for (int j = 0; j < FN; ++j)
            bfr[s][j] = *reinterpret_cast<const bf8_t*>(&Bs[b][s * NT * LD + b_frag[j] + 32 * st]);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            f4_t r = rest[i][j];
            if (ALIGNED) {
              // lead x lead is exact in float32 and kept apart; nine residual products
              lead[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], lead[i][j], 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[0][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[NS - 1][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[NS - 1][i], bfr[0][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[2][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[1][j], r, 0, 0, 0);
            } else {
              // b0 x b0 carries almost all of the sum: its own accumulator, so that its running
              // sum is rounded once per k-step rather than once per product plane
              lead[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], lead[i][j], 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[0][j], r, 0, 0, 0);
              r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], r, 0, 0, 0);
            }
            rest[i][j] = r;
          }
        if (st == 0) stage();
      }
      __builtin_amdgcn_s_setprio(0);
      post();  // bookkeeping of the next chunk while the MFMAs drain
      if (flush) {  // end of a promotion window or of a pair: float32 sums into float64
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              acc[i][j][r] += (double)lead[i][j][r] + (double)rest[i][j][r];
              lead[i][j][r] = 0.f;
              rest[i][j][r] = 0.f;
            }
      }
    };
    chunk_pipeline<KT, kSplitWindow>(g, pairs, pb, pe, pool, Ap, Bp, w.m0, w.n0, blk.mext, blk.next, store, compute);
  }
  epilogue_f32layout<MT, NT, WM, WN, FM, FN>(pr, w, blk, acc, wm, wn, lr, lq);
}

// ---------------------------------------------------------------------------------------------
// configurations and dispatch
// ---------------------------------------------------------------------------------------------
static const MixedConfig kF32Configs[] = {
    {64, 64, 16, 2, 2, "f32_m64n64k16_w2x2"},
    {128, 64, 16, 2, 2, "f32_m128n64k16_w2x2"},
    {64, 128, 16, 2, 2, "f32_m64n128k16_w2x2"},
    {128, 128, 16, 2, 2, "f32_m128n128k16_w2x2"},
    {128, 128, 16, 4, 2, "f32_m128n128k16_w4x2"},
    {128, 128, 16, 2, 4, "f32_m128n128k16_w2x4"},
};
static const MixedConfig kBf16Configs[] = {
    {64, 64, 32, 2, 2, "bf16s_m64n64k32_w2x2"},
    {128, 64, 32, 2, 2, "bf16s_m128n64k32_w2x2"},
    {64, 128, 32, 2, 2, "bf16s_m64n128k32_w2x2"},
    {128, 64, 32, 4, 2, "bf16s_m128n64k32_w4x2"},
    {64, 128, 32, 2, 4, "bf16s_m64n128k32_w2x4"},
    {128, 128, 32, 4, 2, "bf16s_m128n128k32_w4x2"},
    {128, 128, 32, 2, 4, "bf16s_m128n128k32_w2x4"},
};

int mixed_config_count(int precision) {
  if (precision == TAMM_PREC_F32) return (int)(sizeof(kF32Configs) / sizeof(kF32Configs[0]));
  return (int)(sizeof(kBf16Configs) / sizeof(kBf16Configs[0]));
}

const MixedConfig& mixed_config(int precision, int id) {
  return precision == TAMM_PREC_F32 ? kF32Configs[id] : kBf16Configs[id];
}

template <int MT, int NT, int KT, int WGM, int WGN>
static hipError_t launch_f32(int layout, const ContractParams& p, hipStream_t s) {
  const dim3 g(p.n_work), b(64 * WGM * WGN);
  switch (layout) {
    case 3: hipLaunchKernelGGL((k_contract_f32<MT, NT, KT, WGM, WGN, true, true>), g, b, 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_contract_f32<MT, NT, KT, WGM, WGN, true, false>), g, b, 0, s, p); break;
    case 1: hipLaunchKernelGGL((k_contract_f32<MT, NT, KT, WGM, WGN, false, true>), g, b, 0, s, p); break;
    default: hipLaunchKernelGGL((k_contract_f32<MT, NT, KT, WGM, WGN, false, false>), g, b, 0, s, p); break;
  }
  return hipGetLastError();
}

template <int MT, int NT, int KT, int WGM, int WGN, bool AL>
static hipError_t launch_bf(int layout, const ContractParams& p, hipStream_t s) {
  const dim3 g(p.n_work), b(64 * WGM * WGN);
  switch (layout) {
    case kPlanesLayout: hipLaunchKernelGGL((k_contract_bf16s<MT, NT, KT, WGM, WGN, AL, false, false, true>), g, b, 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_contract_bf16s<MT, NT, KT, WGM, WGN, AL, true, true, false>), g, b, 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_contract_bf16s<MT, NT, KT, WGM, WGN, AL, true, false, false>), g, b, 0, s, p); break;
    case 1: hipLaunchKernelGGL((k_contract_bf16s<MT, NT, KT, WGM, WGN, AL, false, true, false>), g, b, 0, s, p); break;
    default: hipLaunchKernelGGL((k_contract_bf16s<MT, NT, KT, WGM, WGN, AL, false, false, false>), g, b, 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_contract_mixed(int precision, int config, int layout, const ContractParams& p, hipStream_t s) {
  if (p.n_work <= 0) return hipSuccess;
  if (precision == TAMM_PREC_F32) {
    switch (config) {
      case 0: return launch_f32<64, 64, 16, 2, 2>(layout, p, s);
      case 1: return launch_f32<128, 64, 16, 2, 2>(layout, p, s);
      case 2: return launch_f32<64, 128, 16, 2, 2>(layout, p, s);
      case 3: return launch_f32<128, 128, 16, 2, 2>(layout, p, s);
      case 4: return launch_f32<128, 128, 16, 4, 2>(layout, p, s);
      case 5: return launch_f32<128, 128, 16, 2, 4>(layout, p, s);
      default: return hipErrorInvalidValue;
    }
  }
  const bool al = precision == TAMM_PREC_BF16X4_ALIGNED;
  switch (config) {
    case 0: return al ? launch_bf<64, 64, 32, 2, 2, true>(layout, p, s) : launch_bf<64, 64, 32, 2, 2, false>(layout, p, s);
    case 1: return al ? launch_bf<128, 64, 32, 2, 2, true>(layout, p, s) : launch_bf<128, 64, 32, 2, 2, false>(layout, p, s);
    case 2: return al ? launch_bf<64, 128, 32, 2, 2, true>(layout, p, s) : launch_bf<64, 128, 32, 2, 2, false>(layout, p, s);
    case 3: return al ? launch_bf<128, 64, 32, 4, 2, true>(layout, p, s) : launch_bf<128, 64, 32, 4, 2, false>(layout, p, s);
    case 4: return al ? launch_bf<64, 128, 32, 2, 4, true>(layout, p, s) : launch_bf<64, 128, 32, 2, 4, false>(layout, p, s);
    case 5: return al ? launch_bf<128, 128, 32, 4, 2, true>(layout, p, s) : launch_bf<128, 128, 32, 4, 2, false>(layout, p, s);
    case 6: return al ? launch_bf<128, 128, 32, 2, 4, true>(layout, p, s) : launch_bf<128, 128, 32, 2, 4, false>(layout, p, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tamm
