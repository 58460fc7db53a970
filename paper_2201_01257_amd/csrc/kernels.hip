// HIP kernels for gfx950: tile-pair screening, the FP64 block-sparse contraction (index-permuted
// LDS gathers feeding v_mfma_f64_16x16x4_f64, atomic-free epilogue), the ordered K-split
// reduction and the orbital-energy denominator update.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "internal.h"

namespace tamm {

typedef double d4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------------
// Tile-pair screening (the block non-zero analysis).  One wave per stored output block walks the
// K tile tuples in lexicographic order, keeps a pair when both operand blocks are stored, and
// compacts the survivors in order with a wave ballot (deterministic, no atomics).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_screen(ScreenParams P) {
  const int item = blockIdx.x;
  if (item >= P.n_items) return;
  const ScreenDesc& S = P.probs ? P.probs[P.item_prob[item]] : P.single;
  const int ob = P.probs ? P.item_block[item] : item;
  const int lane = threadIdx.x;
  const OutBlockDesc blk = S.blocks[ob];
  int count = 0;
  for (int kt0 = 0; kt0 < S.n_kt; kt0 += 64) {
    const int kt = kt0 + lane;
    bool keep = false;
    int64_t aoff = -1, boff = -1;
    int kext = 1, acls = blk.a_cbase, bcls = blk.b_cbase;
    if (kt < S.n_kt) {
      int rem = kt, alin = blk.a_tbase, blin = blk.b_tbase;
      for (int k = S.nk - 1; k >= 0; --k) {
        const int t = rem % S.k_ntiles[k];
        rem /= S.k_ntiles[k];
        alin += t * S.a_tstride[k];
        blin += t * S.b_tstride[k];
        const int c = S.pool[S.k_cls_tab[k] + t];
        acls += c * S.a_cstride[k];
        bcls += c * S.b_cstride[k];
        kext *= S.pool[S.k_size_tab[k] + t];
      }
      aoff = S.a_tile_off[alin];
      boff = S.b_tile_off[blin];
      keep = aoff >= 0 && boff >= 0;
    }
    const unsigned long long mask = __ballot(keep);
    if (keep) {
      const int rank = __popcll(mask & ((1ull << lane) - 1ull));
      PairDesc d;
      d.a_off = aoff;
      d.b_off = boff;
      d.kext = kext;
      d.a_tabM = S.pool[S.a_cls_tabM + acls];
      d.a_tabK = S.pool[S.a_cls_tabK + acls];
      d.b_tabK = S.pool[S.b_cls_tabK + bcls];
      d.b_tabN = S.pool[S.b_cls_tabN + bcls];
      d.kt = kt;
      S.pairs[blk.pair_base + count + rank] = d;
    }
    count += __popcll(mask);
  }
  if (lane == 0) S.counts[ob] = count;
}

hipError_t launch_screen(const ScreenParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_screen, dim3(p.n_items), dim3(64), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// FP64 contraction.
//
// A workgroup owns one output macro-tile (MT x NT of the flattened M x N of one stored output
// block) and, with K splits, one contiguous range of that block's surviving pairs.  The K loop
// runs over the pairs and, inside a pair, over chunks of KT flattened K indices.  Each chunk is
// gathered from the operand blocks through the plan's offset tables straight into LDS; the
// thread-to-element mapping follows the operand's stride-1 label (lanes along k when it is a
// summed label, along m/n otherwise) so that global reads coalesce.  Both operands sit in LDS as
// [row][k] with a row stride of KT+2 doubles, which keeps the MFMA operand reads free of bank
// conflicts.  There is no separate permutation pass.
//
// Software pipeline (three chunks in flight): while the MFMAs of chunk c run from LDS, the data
// of chunk c+1 is in flight into registers and the offset-table entries of chunk c+2 are in
// flight too, so no dependent table->data load chain sits in front of the MFMAs.
//
// v_mfma_f64_16x16x4_f64 lane layout (gfx950, checked on the device): A[m][k] comes from lane
// m + 16k, B[k][n] from lane n + 16k, and D[m][n] lands in lane n + 16*(m%4), register m/4.
//
// The epilogue writes beta*C + alpha*acc through out's offset tables; every element is written
// by exactly one workgroup (beta == 0 never reads C).  With K splits, partial tiles go to the
// workspace and k_reduce sums them in split order.  Results are bitwise reproducible.
//
// Launch modes: one workgroup per work item, or a persistent grid whose workgroups take items
// from a counter (the grouped launch); the item order is the plan's longest-first order.  The
// operands' gather layouts (A_KC, B_KC) are template parameters: "layout" = 2*A_KC + B_KC.
// ---------------------------------------------------------------------------------------------
template <int MT, int NT, int KT, int WGM, int WGN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(64 * WGM * WGN) void k_contract_f64(ContractParams P) {
  constexpr int NTHR = 64 * WGM * WGN;
  constexpr int WM = MT / WGM, WN = NT / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LD = KT + 2;  // LDS row stride in doubles
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert(KT % 4 == 0, "KT multiple of 4");
  using G = Gather<MT, NT, KT, NTHR, A_KC, B_KC, double>;
  __shared__ double As[MT * LD];
  __shared__ double Bs[NT * LD];
  __shared__ int s_next;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int lr = lane & 15, lq = lane >> 4;
  G g;
  g.init(tid);

  int item = blockIdx.x;
  while (item < P.n_work) {
    // work-item descriptors are the same for the whole wave: keep them in scalar registers
    const WorkItem w = wave_uniform(sload(P.work + item));
    const ProblemDesc pr = wave_uniform(P.probs ? sload(P.probs + w.prob) : P.single);
    const OutBlockDesc blk = wave_uniform(sload(pr.blocks + w.ob));
    const int32_t* __restrict__ pool = pr.pool;
    const PairDesc* __restrict__ pairs = pr.pairs + blk.pair_base;
    const int cnt = wave_uniform(gload(pr.counts + w.ob));
    int pb = 0, pe = cnt;
    if (pr.k_splits > 1) {
      pb = (int)(((int64_t)cnt * w.split) / pr.k_splits);
      pe = (int)(((int64_t)cnt * (w.split + 1)) / pr.k_splits);
    }
    // MFMA blocks of this wave that hold at least one valid row / column (uniform per wave)
    const int fm_valid = wave_uniform(min(FM, max(0, (blk.mext - w.m0 - wm * WM + 15) >> 4)));
    const int fn_valid = wave_uniform(min(FN, max(0, (blk.next - w.n0 - wn * WN + 15) >> 4)));
    const bool full = fm_valid == FM && fn_valid == FN;

    d4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = (d4_t){0.0, 0.0, 0.0, 0.0};

    if (pb < pe) {
      // chunk cursors: c = next into LDS, n1 = data in flight, n2 = table entries in flight
      PairDesc d1 = wave_uniform(sload(pairs + pb));
      int p1 = pb, k1 = 0;
      g.setup_pair(d1, pool, pr.A, pr.B, w.m0, w.n0, blk.mext, blk.next);
      g.load_tables(d1, pool, 0);
      g.load_data();
      auto advance = [&]() {
        k1 += KT;
        if (k1 >= d1.kext) {
          ++p1;
          k1 = 0;
          if (p1 >= pe) return false;
          d1 = wave_uniform(sload(pairs + p1));
          g.setup_pair(d1, pool, pr.A, pr.B, w.m0, w.n0, blk.mext, blk.next);
        }
        g.load_tables(d1, pool, k1);
        return true;
      };
      bool has1 = advance();
      while (true) {
        __syncthreads();  // the previous chunk's LDS reads are complete
#pragma unroll
        for (int e = 0; e < G::AE; ++e) As[g.a_lds_row(e) * LD + g.a_lds_k(e)] = g.ra[e];
#pragma unroll
        for (int e = 0; e < G::BE; ++e) Bs[g.b_lds_row(e) * LD + g.b_lds_k(e)] = g.rb[e];
        __syncthreads();
        bool has2 = false;
        if (has1) {
          g.load_data();  // chunk n1 (its table entries arrived during the previous MFMA phase)
          has2 = advance();
        }
        // All KT/4 k-steps run, unrolled so that the LDS reads of step s+1 overlap the MFMAs of
        // step s; a ragged last chunk of a pair holds zeros beyond its K extent.  MFMA blocks
        // wholly outside the output block are skipped.
#pragma unroll
        for (int s = 0; s < KT / 4; ++s) {
          const int k = 4 * s + lq;
          double af[FM], bf[FN];
#pragma unroll
          for (int i = 0; i < FM; ++i) af[i] = As[(wm * WM + i * 16 + lr) * LD + k];
#pragma unroll
          for (int j = 0; j < FN; ++j) bf[j] = Bs[(wn * WN + j * 16 + lr) * LD + k];
          if (full) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
              for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          } else {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
              for (int j = 0; j < FN; ++j)
                if (i < fm_valid && j < fn_valid)
                  acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          }
        }
        if (!has1) break;
        has1 = has2;
      }
    }

    // epilogue: lane holds D[m][n] for m = 4r + lane/16 (register r), n = lane%16
    if (pr.k_splits > 1) {
      double* part = pr.partial + ((int64_t)w.tile * pr.k_splits + w.split) * (MT * NT);
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
    } else {
      const double alpha = pr.alpha, beta = pr.beta;
      double* __restrict__ Cg = pr.C;
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
    if (!P.next_item) break;
    __syncthreads();  // LDS and s_next are free
    if (tid == 0) s_next = atomicAdd(P.next_item, 1);
    __syncthreads();
    item = s_next;
  }
}

__global__ void k_set_counter(int32_t* c, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = v;
}

hipError_t launch_set_counter(int32_t* counter, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, s, counter, value);
  return hipGetLastError();
}

// Ordered reduction of K-split partial tiles (split 0, 1, ... in order) and the epilogue.
__global__ __launch_bounds__(256) void k_reduce(ReduceParams P) {
  const int t = blockIdx.x;
  if (t >= P.n_items) return;
  const ReduceItem it = P.items[t];
  const ProblemDesc& pr = P.probs ? P.probs[it.prob] : P.single;
  const OutBlockDesc blk = pr.blocks[it.ob];
  const int tile = P.tile_m * P.tile_n;
  const double* part = pr.partial + (int64_t)it.tile * pr.k_splits * tile;
  for (int e = threadIdx.x; e < tile; e += blockDim.x) {
    const int m = it.m0 + e / P.tile_n, n = it.n0 + e % P.tile_n;
    if (m >= blk.mext || n >= blk.next) continue;
    double s = 0.0;
    for (int k = 0; k < pr.k_splits; ++k) s += part[(int64_t)k * tile + e];
    const int64_t idx = blk.c_off + pr.pool[blk.c_tabM + m] + pr.pool[blk.c_tabN + n];
    const double v = pr.alpha * s;
    pr.C[idx] = (pr.beta == 0.0) ? v : pr.beta * pr.C[idx] + v;
  }
}

hipError_t launch_reduce(const ReduceParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(p.n_items), dim3(256), 0, s, p);
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
    {128, 128, 32, 2, 2, "f64_m128n128k32_w2x2"},
    {128, 64, 32, 2, 2, "f64_m128n64k32_w2x2"},
    {64, 128, 32, 2, 2, "f64_m64n128k32_w2x2"},
    {32, 256, 16, 1, 4, "f64_m32n256k16_w1x4"},
    {256, 32, 16, 4, 1, "f64_m256n32k16_w4x1"},
};

int f64_config_count() { return (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0])); }
const F64Config& f64_config(int id) { return kF64Configs[id]; }

template <int MT, int NT, int KT, int WGM, int WGN>
static hipError_t launch_cfg(int layout, const ContractParams& p, int grid, hipStream_t s) {
  const dim3 g(grid > 0 ? grid : p.n_work), b(64 * WGM * WGN);
  switch (layout) {
    case 3: hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, true, true>), g, b, 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, true, false>), g, b, 0, s, p); break;
    case 1: hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, false, true>), g, b, 0, s, p); break;
    default: hipLaunchKernelGGL((k_contract_f64<MT, NT, KT, WGM, WGN, false, false>), g, b, 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_contract_f64(int config, int layout, const ContractParams& p, int grid, hipStream_t s) {
  if (p.n_work <= 0) return hipSuccess;
  switch (config) {
    case 0: return launch_cfg<64, 64, 16, 2, 2>(layout, p, grid, s);
    case 1: return launch_cfg<128, 64, 16, 2, 2>(layout, p, grid, s);
    case 2: return launch_cfg<64, 128, 16, 2, 2>(layout, p, grid, s);
    case 3: return launch_cfg<128, 128, 16, 2, 2>(layout, p, grid, s);
    case 4: return launch_cfg<32, 64, 16, 2, 2>(layout, p, grid, s);
    case 5: return launch_cfg<128, 128, 32, 2, 2>(layout, p, grid, s);
    case 6: return launch_cfg<128, 64, 32, 2, 2>(layout, p, grid, s);
    case 7: return launch_cfg<64, 128, 32, 2, 2>(layout, p, grid, s);
    case 8: return launch_cfg<32, 256, 16, 1, 4>(layout, p, grid, s);
    case 9: return launch_cfg<256, 32, 16, 4, 1>(layout, p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// Orbital-energy denominator update.  Each workgroup handles `chunk` consecutive elements of one
// stored block; IEEE float64 division; the denominator is summed in the documented order.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_denominator(DenomParams P) {
  const int64_t it = blockIdx.x;
  if (it >= P.n_items) return;
  const int b = P.item_block[it];
  const int rank = P.rank;
  int lo[kMaxRank], ext[kMaxRank];
  int n = 1;
  for (int d = 0; d < rank; ++d) {
    const int t = P.block_tiles[(int64_t)b * rank + d];
    lo[d] = (int)P.tile_offset[P.dim_tile_base[d] + t];
    ext[d] = (int)P.tile_size[P.dim_tile_base[d] + t];
    n *= ext[d];
  }
  const int64_t base = P.block_off[b];
  const int e0 = P.item_start[it];
  const int e1 = min(n, e0 + P.chunk);
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    int rem = e, idx[kMaxRank];
    for (int d = rank - 1; d >= 0; --d) {
      idx[d] = lo[d] + rem % ext[d];
      rem /= ext[d];
    }
    double den = 0.0;
    bool first = true;
    for (int d = 0; d < rank; ++d)
      if (P.sign[d] > 0) {
        den = first ? P.energy[d][idx[d]] : den + P.energy[d][idx[d]];
        first = false;
      }
    for (int d = 0; d < rank; ++d)
      if (P.sign[d] < 0) {
        den = first ? -P.energy[d][idx[d]] : den - P.energy[d][idx[d]];
        first = false;
      }
    P.out[base + e] = P.in[base + e] / den;
  }
}

hipError_t launch_denominator(const DenomParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_denominator, dim3((unsigned)p.n_items), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace tamm
