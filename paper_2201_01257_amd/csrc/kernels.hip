// HIP kernels for gfx950: tile-pair screening, the FP64 block-sparse contraction (index-permuted
// LDS gathers feeding v_mfma_f64_16x16x4_f64, atomic-free epilogue), the ordered K-split
// reduction and the orbital-energy denominator update.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace tamm {

typedef double d4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------------
// Tile-pair screening.  One wave per stored output block walks the K tile tuples in
// lexicographic order, keeps a pair when both operand blocks are stored, and compacts the
// survivors in order with a wave ballot (deterministic, no atomics).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_screen(ScreenParams p) {
  const int ob = blockIdx.x;
  if (ob >= p.n_blocks) return;
  const int lane = threadIdx.x;
  const OutBlockDesc blk = p.blocks[ob];
  int count = 0;
  for (int kt0 = 0; kt0 < p.n_kt; kt0 += 64) {
    const int kt = kt0 + lane;
    bool keep = false;
    int64_t aoff = -1, boff = -1;
    int kext = 1, acls = blk.a_cbase, bcls = blk.b_cbase;
    if (kt < p.n_kt) {
      int rem = kt, alin = blk.a_tbase, blin = blk.b_tbase;
      for (int k = p.nk - 1; k >= 0; --k) {
        const int t = rem % p.k_ntiles[k];
        rem /= p.k_ntiles[k];
        alin += t * p.a_tstride[k];
        blin += t * p.b_tstride[k];
        const int c = p.pool[p.k_cls_tab[k] + t];
        acls += c * p.a_cstride[k];
        bcls += c * p.b_cstride[k];
        kext *= p.pool[p.k_size_tab[k] + t];
      }
      aoff = p.a_tile_off[alin];
      boff = p.b_tile_off[blin];
      keep = aoff >= 0 && boff >= 0;
    }
    const unsigned long long mask = __ballot(keep);
    if (keep) {
      const int rank = __popcll(mask & ((1ull << lane) - 1ull));
      PairDesc d;
      d.a_off = aoff;
      d.b_off = boff;
      d.kext = kext;
      d.a_tabM = p.pool[p.a_cls_tabM + acls];
      d.a_tabK = p.pool[p.a_cls_tabK + acls];
      d.b_tabK = p.pool[p.b_cls_tabK + bcls];
      d.b_tabN = p.pool[p.b_cls_tabN + bcls];
      d.kt = kt;
      p.pairs[blk.pair_base + count + rank] = d;
    }
    count += __popcll(mask);
  }
  if (lane == 0) p.counts[ob] = count;
}

hipError_t launch_screen(const ScreenParams& p, hipStream_t s) {
  if (p.n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_screen, dim3(p.n_blocks), dim3(64), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// FP64 contraction.
//
// One workgroup owns one output macro-tile (MT x NT of the flattened M x N of one stored output
// block) and, for a K split, one contiguous range of that block's surviving pairs.  The K loop
// runs over the pairs and, inside a pair, over chunks of KT flattened K indices.  Each chunk is
// gathered from the operand blocks through the plan's offset tables straight into LDS, with
// the thread-to-element mapping following the operand's stride-1 label (so global reads
// coalesce) and the LDS layout chosen so that the MFMA operand reads are conflict-free.  There
// is no separate permutation pass.  Global loads of chunk c+1 are issued before the MFMAs of
// chunk c (register prefetch).  Accumulation is in float64 MFMA registers; the epilogue writes
// beta*C + alpha*acc through out's offset tables, each element by exactly one workgroup.
//
// v_mfma_f64_16x16x4_f64 lane layout (gfx950): A[m][k] from lane m + 16k, B[k][n] from lane
// n + 16k, result D[m][n] in lane n + 16*(m%4), register m/4.
// ---------------------------------------------------------------------------------------------

// LDS row strides (in doubles) chosen for conflict-free MFMA operand reads:
//   "KM" layout (row = k, contiguous m): stride = 16 (mod 32) so rows k and k+1 use disjoint halves
//   of the 64 banks;  "MK" layout (row = m, contiguous k): stride = 2 (mod 4).
template <int M>
struct KMStride {
  static constexpr int value = (M % 32 == 16) ? M : (M + (48 - M % 32) % 32);
};
template <int K>
struct MKStride {
  static constexpr int value = K + 2;
};

template <int MT, int NT, int KT, int WGM, int WGN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(64 * WGM * WGN) void k_contract_f64(ContractParams p) {
  constexpr int NTHR = 64 * WGM * WGN;
  constexpr int WM = MT / WGM, WN = NT / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert(KT % 4 == 0, "KT multiple of 4");
  // A chunk: MT x KT.  K-contiguous operand: lanes along k.  M-contiguous: lanes along m.
  static_assert(!A_KC || (NTHR % KT == 0 && MT % (NTHR / KT) == 0), "A K-contiguous mapping");
  static_assert(A_KC || (NTHR % MT == 0 && KT % (NTHR / MT) == 0), "A M-contiguous mapping");
  static_assert(!B_KC || (NTHR % KT == 0 && NT % (NTHR / KT) == 0), "B K-contiguous mapping");
  static_assert(B_KC || (NTHR % NT == 0 && KT % (NTHR / NT) == 0), "B N-contiguous mapping");
  constexpr int AE = MT * KT / NTHR;
  constexpr int BE = NT * KT / NTHR;
  constexpr int A_LD = A_KC ? MKStride<KT>::value : KMStride<MT>::value;
  constexpr int B_LD = B_KC ? MKStride<KT>::value : KMStride<NT>::value;
  constexpr int A_LDS = A_KC ? MT * A_LD : KT * A_LD;
  constexpr int B_LDS = B_KC ? NT * B_LD : KT * B_LD;
  __shared__ double As[A_LDS];
  __shared__ double Bs[B_LDS];

  const WorkItem w = p.work[blockIdx.x];
  const OutBlockDesc blk = p.blocks[w.ob];
  const int cnt = p.counts[w.ob];
  int pb = 0, pe = cnt;
  if (p.k_splits > 1) {
    pb = (int)(((int64_t)cnt * w.split) / p.k_splits);
    pe = (int)(((int64_t)cnt * (w.split + 1)) / p.k_splits);
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int32_t* __restrict__ pool = p.pool;
  const double* __restrict__ Ag = p.A;
  const double* __restrict__ Bg = p.B;

  // fixed per-thread gather coordinates inside a chunk
  const int a_k = A_KC ? tid % KT : tid / MT;  // first k (M-contig: + e*(NTHR/MT))
  const int a_m = A_KC ? tid / KT : tid % MT;  // first m (K-contig: + e*(NTHR/KT))
  const int b_k = B_KC ? tid % KT : tid / NT;
  const int b_n = B_KC ? tid / KT : tid % NT;

  d4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (d4_t){0.0, 0.0, 0.0, 0.0};

  double ra[AE], rb[BE];
  // per-pair row/column offsets (element offsets of the fixed m/n of this thread)
  int64_t a_rowoff[A_KC ? AE : 1];
  int64_t b_coloff[B_KC ? BE : 1];
  bool a_rowok[A_KC ? AE : 1];
  bool b_colok[B_KC ? BE : 1];

  PairDesc pd;
  int pi = pb, k0 = 0;

  auto setup_pair = [&](const PairDesc& d) {
    if (A_KC) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int m = w.m0 + a_m + e * (NTHR / KT);
        a_rowok[e] = m < blk.mext;
        a_rowoff[e] = d.a_off + (a_rowok[e] ? pool[d.a_tabM + m] : 0);
      }
    } else {
      const int m = w.m0 + a_m;
      a_rowok[0] = m < blk.mext;
      a_rowoff[0] = d.a_off + (a_rowok[0] ? pool[d.a_tabM + m] : 0);
    }
    if (B_KC) {
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        const int n = w.n0 + b_n + e * (NTHR / KT);
        b_colok[e] = n < blk.next;
        b_coloff[e] = d.b_off + (b_colok[e] ? pool[d.b_tabN + n] : 0);
      }
    } else {
      const int n = w.n0 + b_n;
      b_colok[0] = n < blk.next;
      b_coloff[0] = d.b_off + (b_colok[0] ? pool[d.b_tabN + n] : 0);
    }
  };

  auto load_chunk = [&](const PairDesc& d, int kbase) {
    const int kc = min(KT, d.kext - kbase);
    if (A_KC) {
      const bool kok = a_k < kc;
      const int64_t koff = kok ? pool[d.a_tabK + kbase + a_k] : 0;
#pragma unroll
      for (int e = 0; e < AE; ++e) ra[e] = (kok && a_rowok[e]) ? Ag[a_rowoff[e] + koff] : 0.0;
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int k = a_k + e * (NTHR / MT);
        const bool ok = a_rowok[0] && k < kc;
        ra[e] = ok ? Ag[a_rowoff[0] + pool[d.a_tabK + kbase + k]] : 0.0;
      }
    }
    if (B_KC) {
      const bool kok = b_k < kc;
      const int64_t koff = kok ? pool[d.b_tabK + kbase + b_k] : 0;
#pragma unroll
      for (int e = 0; e < BE; ++e) rb[e] = (kok && b_colok[e]) ? Bg[b_coloff[e] + koff] : 0.0;
    } else {
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        const int k = b_k + e * (NTHR / NT);
        const bool ok = b_colok[0] && k < kc;
        rb[e] = ok ? Bg[b_coloff[0] + pool[d.b_tabK + kbase + k]] : 0.0;
      }
    }
    return kc;
  };

  if (pi < pe) {
    pd = p.pairs[blk.pair_base + pi];
    setup_pair(pd);
    int kc = load_chunk(pd, 0);
    while (true) {
      __syncthreads();  // previous chunk's LDS reads are complete
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        if (A_KC) As[(a_m + e * (NTHR / KT)) * A_LD + a_k] = ra[e];
        else As[(a_k + e * (NTHR / MT)) * A_LD + a_m] = ra[e];
      }
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        if (B_KC) Bs[(b_n + e * (NTHR / KT)) * B_LD + b_k] = rb[e];
        else Bs[(b_k + e * (NTHR / NT)) * B_LD + b_n] = rb[e];
      }
      __syncthreads();
      const int ksteps = (kc + 3) >> 2;
      // advance to the next chunk and issue its global loads before this chunk's MFMAs
      k0 += KT;
      bool more = true;
      if (k0 >= pd.kext) {
        ++pi;
        k0 = 0;
        if (pi < pe) {
          pd = p.pairs[blk.pair_base + pi];
          setup_pair(pd);
        } else {
          more = false;
        }
      }
      int kc_next = 0;
      if (more) kc_next = load_chunk(pd, k0);

      const int lr = lane & 15, lk = lane >> 4;
      for (int s = 0; s < ksteps; ++s) {
        const int k = 4 * s + lk;
        double af[FM], bf[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const int m = wm * WM + i * 16 + lr;
          af[i] = A_KC ? As[m * A_LD + k] : As[k * A_LD + m];
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int n = wn * WN + j * 16 + lr;
          bf[j] = B_KC ? Bs[n * B_LD + k] : Bs[k * B_LD + n];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      if (!more) break;
      kc = kc_next;
    }
  }

  // epilogue: lane holds D[m][n] for m = 4r + lane/16 (register r), n = lane%16
  const int lr = lane & 15, lq = lane >> 4;
  if (p.k_splits > 1) {
    double* part = p.partial + (int64_t)blockIdx.x * (MT * NT);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = wm * WM + i * 16 + 4 * r + lq;
          const int n = wn * WN + j * 16 + lr;
          part[m * NT + n] = acc[i][j][r];
        }
    return;
  }
  const double alpha = p.alpha, beta = p.beta;
  double* __restrict__ Cg = p.C;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = w.m0 + wm * WM + i * 16 + 4 * r + lq;
      if (m >= blk.mext) continue;
      const int64_t rowoff = blk.c_off + pool[blk.c_tabM + m];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = w.n0 + wn * WN + j * 16 + lr;
        if (n >= blk.next) continue;
        const int64_t idx = rowoff + pool[blk.c_tabN + n];
        const double v = alpha * acc[i][j][r];
        Cg[idx] = (beta == 0.0) ? v : beta * Cg[idx] + v;
      }
    }
}

// Ordered reduction of K-split partial tiles (split 0, 1, ... in order) and the epilogue.
__global__ __launch_bounds__(256) void k_reduce(ReduceParams p) {
  const int t = blockIdx.x;
  if (t >= p.n_tiles) return;
  const WorkItem w = p.work[(int64_t)t * p.k_splits];  // the K splits of a tile are adjacent
  const OutBlockDesc blk = p.blocks[w.ob];
  const int tile = p.tile_m * p.tile_n;
  for (int e = threadIdx.x; e < tile; e += blockDim.x) {
    const int m = w.m0 + e / p.tile_n, n = w.n0 + e % p.tile_n;
    if (m >= blk.mext || n >= blk.next) continue;
    double s = 0.0;
    for (int k = 0; k < p.k_splits; ++k) s += p.partial[((int64_t)t * p.k_splits + k) * tile + e];
    const int64_t idx = blk.c_off + p.pool[blk.c_tabM + m] + p.pool[blk.c_tabN + n];
    const double v = p.alpha * s;
    p.C[idx] = (p.beta == 0.0) ? v : p.beta * p.C[idx] + v;
  }
}

hipError_t launch_reduce(const ReduceParams& p, hipStream_t s) {
  if (p.n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(p.n_tiles), dim3(256), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Configurations and dispatch
// ---------------------------------------------------------------------------------------------
static const F64Config kF64Configs[] = {
    {64, 64, 16, 2, 2, "f64_m64n64k16_w2x2"},
    {128, 64, 16, 2, 2, "f64_m128n64k16_w2x2"},
    {64, 128, 16, 2, 2, "f64_m64n128k16_w2x2"},
    {128, 128, 16, 2, 2, "f64_m128n128k16_w2x2"},
    {32, 64, 16, 2, 2, "f64_m32n64k16_w2x2"},
};

int f64_config_count() { return (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0])); }
const F64Config& f64_config(int id) { return kF64Configs[id]; }

template <int MT, int NT, int KT, int WGM, int WGN>
static hipError_t launch_cfg(bool akc, bool bkc, const ContractParams& p, hipStream_t s) {
  dim3 grid(p.n_work), block(64 * WGM * WGN);
  if (akc && bkc) hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, true, true>), grid, block, 0, s, p);
  else if (akc) hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, true, false>), grid, block, 0, s, p);
  else if (bkc) hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, false, true>), grid, block, 0, s, p);
  else hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, false, false>), grid, block, 0, s, p);
  return hipGetLastError();
}

hipError_t launch_contract_f64(int config, bool akc, bool bkc, const ContractParams& p, hipStream_t s) {
  if (p.n_work <= 0) return hipSuccess;
  switch (config) {
    case 0: return launch_cfg<64, 64, 16, 2, 2>(akc, bkc, p, s);
    case 1: return launch_cfg<128, 64, 16, 2, 2>(akc, bkc, p, s);
    case 2: return launch_cfg<64, 128, 16, 2, 2>(akc, bkc, p, s);
    case 3: return launch_cfg<128, 128, 16, 2, 2>(akc, bkc, p, s);
    case 4: return launch_cfg<32, 64, 16, 2, 2>(akc, bkc, p, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// Orbital-energy denominator update: one workgroup per stored block; IEEE float64 division.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_denominator(DenomParams p) {
  const int64_t b = blockIdx.x;
  if (b >= p.n_blocks) return;
  const int rank = p.rank;
  int64_t lo[kMaxRank], ext[kMaxRank];
  int64_t n = 1;
  for (int d = 0; d < rank; ++d) {
    const int t = p.block_tiles[b * rank + d];
    lo[d] = p.tile_offset[p.dim_tile_base[d] + t];
    ext[d] = p.tile_size[p.dim_tile_base[d] + t];
    n *= ext[d];
  }
  const int64_t base = p.block_off[b];
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    int64_t rem = e, idx[kMaxRank];
    for (int d = rank - 1; d >= 0; --d) {
      idx[d] = lo[d] + rem % ext[d];
      rem /= ext[d];
    }
    double den = 0.0;
    bool first = true;
    for (int d = 0; d < rank; ++d)
      if (p.sign[d] > 0) {
        den = first ? p.energy[d][idx[d]] : den + p.energy[d][idx[d]];
        first = false;
      }
    for (int d = 0; d < rank; ++d)
      if (p.sign[d] < 0) {
        den = first ? -p.energy[d][idx[d]] : den - p.energy[d][idx[d]];
        first = false;
      }
    p.out[base + e] = p.in[base + e] / den;
  }
}

hipError_t launch_denominator(const DenomParams& p, int64_t /*max_block_elems*/, hipStream_t s) {
  if (p.n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_denominator, dim3((unsigned)p.n_blocks), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace tamm
