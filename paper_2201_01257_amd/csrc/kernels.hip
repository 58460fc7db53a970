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
// compacts the survivors in order with a wave ballot (deterministic, no atomics).  A fused node
// (several contractions into the same output tiles) walks its segments one after another and
// appends to one list, so that one output tile's K loop later runs over every segment's pairs.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_screen(ScreenParams P) {
  const int item = blockIdx.x;
  if (item >= P.n_items) return;
  const ScreenDesc* S = P.probs ? P.probs + P.item_prob[item] : &P.single;
  const int ob = P.probs ? P.item_block[item] : item;
  const int lane = threadIdx.x;
  PairDesc* __restrict__ out = S->pairs + (int64_t)ob * S->pair_stride;
  int32_t* counts = S->counts;
  int count = 0;
  while (true) {  // segments of a fused node append to one list, in order
    const OutBlockDesc blk = S->blocks[ob];
    for (int kt0 = 0; kt0 < S->n_kt; kt0 += 64) {
      const int kt = kt0 + lane;
      bool keep = false;
      int64_t aoff = -1, boff = -1;
      int kext = 1, acls = blk.a_cbase, bcls = blk.b_cbase;
      if (kt < S->n_kt) {
        int rem = kt, alin = blk.a_tbase, blin = blk.b_tbase;
        for (int k = S->nk - 1; k >= 0; --k) {
          const int t = rem % S->k_ntiles[k];
          rem /= S->k_ntiles[k];
          alin += t * S->a_tstride[k];
          blin += t * S->b_tstride[k];
          const int c = S->pool[S->k_cls_tab[k] + t];
          acls += c * S->a_cstride[k];
          bcls += c * S->b_cstride[k];
          kext *= S->pool[S->k_size_tab[k] + t];
        }
        aoff = S->a_tile_off[alin];
        boff = S->b_tile_off[blin];
        keep = aoff >= 0 && boff >= 0;
      }
      const unsigned long long mask = __ballot(keep);
      if (keep) {
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        PairDesc d;
        d.a_off = aoff + S->a_base;
        d.b_off = boff + S->b_base;
        d.kext = kext;
        d.a_tabM = S->pool[S->a_cls_tabM + acls] + S->pool_base;
        d.a_tabK = S->pool[S->a_cls_tabK + acls] + S->pool_base;
        d.b_tabK = S->pool[S->b_cls_tabK + bcls] + S->pool_base;
        d.b_tabN = S->pool[S->b_cls_tabN + bcls] + S->pool_base;
        d.kt = kt;
        out[count + rank] = d;
      }
      count += __popcll(mask);
    }
    if (S->next_seg < 0) break;
    S = P.probs + S->next_seg;
  }
  if (lane == 0) counts[ob] = count;
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
// summed label, along m/n otherwise) so that global reads coalesce.  Each operand chunk sits in
// LDS in the layout LdsLayout chooses for its orientation and size, which keeps the MFMA operand
// reads and the gather stores free of bank conflicts.  There is no separate permutation pass.
//
// Software pipeline with one barrier per chunk: LDS holds two chunk buffers.  While the MFMAs
// of chunk c run from one buffer, the registers holding chunk c+1 (loaded during the previous
// chunk's MFMAs) are stored into the other buffer, the global loads of chunk c+2 are issued into
// the same registers, and the offset-table entries of chunk c+3 are fetched.  Inside a chunk the
// MFMA operands of k-step s+1 are read from LDS while the MFMAs of step s run.  In a tile inside
// its block every MFMA block runs (padding k positions hold zeros) and the MFMA stream has no
// branches; a tile that runs past its block deals its live output fragments over the waves
// (see below).
//
// v_mfma_f64_16x16x4_f64 lane layout (gfx950, checked on the device): A[m][k] comes from lane
// m + 16k, B[k][n] from lane n + 16k, and D[m][n] lands in lane n + 16*(m%4), register m/4.
//
// The epilogue writes beta*C + alpha*acc through out's offset tables; every element is written
// by exactly one workgroup (beta == 0 never reads C).  With K splits, partial tiles go to the
// workspace and k_reduce sums them in split order.  Results are bitwise reproducible.
//
// Launch modes: one workgroup per work item, or a persistent grid whose workgroups take items
// from a counter (the grouped launch); the item order is the plan's.  The operands' gather
// layouts (A_KC, B_KC) are template parameters: "layout" = 2*A_KC + B_KC.
// ---------------------------------------------------------------------------------------------
// LDS layout of one operand chunk (ROWS rows x KT summed indices, float64), chosen by the LDS's
// measured service pattern on gfx950 (8-byte reads: 32 lanes per cycle over 64 four-byte banks;
// 8-byte writes: 16 lanes per cycle over 32 banks; 16-byte writes: 8 lanes per cycle over 32
// banks) for the MFMA operand reads (8 bytes per lane: lanes 16q + r read row R0 + r at k-step
// position q) and the gather's stores:
//   kind 0, an operand whose stride-1 label is summed (lanes gather along k), up to 128 rows:
//     [row][k] with a row stride of KT + 2 doubles -- half the stride is odd, so the 16 rows x 2 k
//     of a read cycle land on 32 distinct 8-byte bank pairs, and a lane's two adjacent k go in
//     one aligned 16-byte store;
//   kind 1, the other operands with rows = 16 mod 32 or at least 128 rows: [k][row] with a k
//     stride of rows + pad (16 mod 32 doubles) -- 16 consecutive rows of one k fill half the
//     banks and the next k the other half, and a lane's two adjacent rows go in one store;
//   kind 2, otherwise (where that padding would cost LDS occupancy): [row][k] with an odd row
//     stride KT + 1, reads two-way conflicted.
template <int ROWS, int KT, bool KC>
struct LdsLayout {
  static constexpr int KIND = KC ? (ROWS <= 128 ? 0 : 2) : ((ROWS % 32 == 16 || ROWS >= 128) ? 1 : 2);
  static constexpr int LDR = ROWS + ((48 - ROWS % 32) % 32);  // kind 1: k stride, 16 mod 32
  static constexpr int RS = KIND == 1 ? 1 : (KIND == 0 ? KT + 2 : KT + 1);  // element stride between rows
  static constexpr int KS = KIND == 1 ? LDR : 1;                            // ... between k positions
  static constexpr int SIZE = KIND == 1 ? KT * LDR : ROWS * RS;             // doubles per buffer
  static constexpr int PAIR = KC ? KS : RS;  // distance of the two elements of a 16-byte gather load
  static constexpr bool STORE16 = PAIR == 1 && (KC ? RS : KS) % 2 == 0;  // they go in one aligned store
  static_assert(KIND != 1 || LDR % 32 == 16, "kind 1 stride");
  static_assert(KIND != 0 || (RS / 2) % 2 == 1, "kind 0 stride");
  static_assert(SIZE % 2 == 0, "16-byte aligned buffers");
  __device__ static constexpr int at(int row, int k) { return row * RS + k * KS; }
};

// A gather load's VEC elements into LDS: one 16-byte store when they are adjacent and aligned,
// else one store each, PAIR elements apart
template <int VEC, int PAIR, bool STORE16>
__device__ __forceinline__ void lds_store(double* dst, const double* v) {
  if constexpr (VEC == 2 && STORE16) {
    typedef double d2_t __attribute__((ext_vector_type(2)));
    *reinterpret_cast<d2_t*>(dst) = (d2_t){v[0], v[1]};
  } else {
    dst[0] = v[0];
    if constexpr (VEC == 2) dst[PAIR] = v[1];
  }
}

template <int MT, int NT, int KT, int WGM, int WGN, int OCC, bool A_KC, bool B_KC, int VEC>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(OCC))) void k_contract_f64(ContractParams P) {
  constexpr int NTHR = 64 * WGM * WGN;
  constexpr int WM = MT / WGM, WN = NT / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int NS = KT / 4;  // MFMA k-steps per chunk
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert(KT % 4 == 0 && NS >= 2, "KT a multiple of 4, at least 8");
  using G = Gather<MT, NT, KT, NTHR, A_KC, B_KC, double, VEC>;
  using LA = LdsLayout<MT, KT, A_KC>;
  using LB = LdsLayout<NT, KT, B_KC>;
  __shared__ __attribute__((aligned(16))) double As[2][LA::SIZE];
  __shared__ __attribute__((aligned(16))) double Bs[2][LB::SIZE];
  __shared__ int s_next;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int lr = lane & 15, lq = lane >> 4;
  const int a_frag = LA::at(wm * WM + lr, lq);  // this lane's operand reads at k-step 0
  const int b_frag = LB::at(wn * WN + lr, lq);
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
    const int nsplit = item_nsplit(w), split = item_split(w);
    const int pb = (int)(((int64_t)cnt * split) / nsplit), pe = (int)(((int64_t)cnt * (split + 1)) / nsplit);

    d4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = (d4_t){0.0, 0.0, 0.0, 0.0};

    // A tile that runs past its block holds fewer live 16 x 16 output fragments than waves x
    // fragments per wave.  When dealing the live ones round-robin over the waves (fragment f to
    // wave f % NW, slot f / NW) shortens the longest wave's share, each wave multiplies only its
    // dealt fragments: the workgroup's barrier-to-barrier time is set by that longest share.
    // Every output element is still summed by one wave in the same k order, so the results are
    // the same bits either way.
    constexpr int NW = WGM * WGN, NSLOT = FM * FN;
    const int fml = min(MT / 16, (blk.mext - w.m0 + 15) >> 4), fnl = min(NT / 16, (blk.next - w.n0 + 15) >> 4);
    const bool dealt = (fml * fnl + NW - 1) / NW < NSLOT;
    const int wv = wave_uniform(wave);
    const int nslot = dealt ? max(0, min(NSLOT, (fml * fnl - wv + NW - 1) / NW)) : NSLOT;

    if (pb < pe) {
      auto store = [&](int b) {
#pragma unroll
        for (int e = 0; e < G::AE; e += VEC)
          lds_store<VEC, LA::PAIR, LA::STORE16>(&As[b][LA::at(g.a_lds_row(e), g.a_lds_k(e))], &g.ra[e]);
#pragma unroll
        for (int e = 0; e < G::BE; e += VEC)
          lds_store<VEC, LB::PAIR, LB::STORE16>(&Bs[b][LB::at(g.b_lds_row(e), g.b_lds_k(e))], &g.rb[e]);
      };
      auto compute = [&](int b, bool, auto&& stage, auto&& post) {
        const double* as = As[b] + a_frag;
        const double* bs = Bs[b] + b_frag;
        double af[2][FM], bf[2][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) af[0][i] = as[i * 16 * LA::RS];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[0][j] = bs[j * 16 * LB::RS];
        __builtin_amdgcn_s_setprio(1);  // MFMA phase first when waves of two workgroups compete
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int cur = s & 1, nxt = cur ^ 1;
          if (s + 1 < NS) {  // operands of the next k-step while this step's MFMAs run
#pragma unroll
            for (int i = 0; i < FM; ++i) af[nxt][i] = as[i * 16 * LA::RS + 4 * (s + 1) * LA::KS];
#pragma unroll
            for (int j = 0; j < FN; ++j) bf[nxt][j] = bs[j * 16 * LB::RS + 4 * (s + 1) * LB::KS];
          }
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[cur][i], bf[cur][j], acc[i][j], 0, 0, 0);
          if (s == 0) stage();
        }
        __builtin_amdgcn_s_setprio(0);
        post();
      };
      if (!dealt) {
        chunk_pipeline<KT, 0>(g, pairs, pb, pe, pool, pr.A, pr.B, w.m0, w.n0, blk.mext, blk.next, store, compute);
      } else {
        // LDS offsets of this wave's dealt fragments: the fragment's first row (the same for the
        // whole wave) plus the lane's own row and k-step position
        int sa[NSLOT], sb[NSLOT];
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
          const int f = wv + q * NW, fi = f / fnl, fj = f - fi * fnl;
          sa[q] = wave_uniform(fi * 16 * LA::RS);
          sb[q] = wave_uniform(fj * 16 * LB::RS);
        }
        auto compute_dealt = [&](int b, bool, auto&& stage, auto&& post) {
          const double* as = As[b] + LA::at(lr, lq);
          const double* bs = Bs[b] + LB::at(lr, lq);
          __builtin_amdgcn_s_setprio(1);
#pragma unroll
          for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q)
              if (q < nslot)
                acc[q / FN][q % FN] =
                    __builtin_amdgcn_mfma_f64_16x16x4f64(as[sa[q] + 4 * s * LA::KS], bs[sb[q] + 4 * s * LB::KS],
                                                         acc[q / FN][q % FN], 0, 0, 0);
            if (s == 0) stage();
          }
          __builtin_amdgcn_s_setprio(0);
          post();
        };
        chunk_pipeline<KT, 0>(g, pairs, pb, pe, pool, pr.A, pr.B, w.m0, w.n0, blk.mext, blk.next, store, compute_dealt);
      }
    }

    // epilogue: lane holds D[m][n] for m = 4r + lane/16 (register r), n = lane%16
    if (dealt) {
      // per dealt fragment: its rows and columns, then the same writes as below
      const double alpha = pr.alpha, beta = pr.beta;
      __attribute__((address_space(1))) double* __restrict__ Cg = (__attribute__((address_space(1))) double*)pr.C;
#pragma unroll
      for (int q = 0; q < NSLOT; ++q) {
        if (q >= nslot) continue;
        const int f = wv + q * NW, fi = f / fnl, fj = f - fi * fnl;
        const int n = fj * 16 + lr;
        if (nsplit > 1) {
          double* part = pr.partial + ((int64_t)w.tile + split) * (MT * NT);
#pragma unroll
          for (int r = 0; r < 4; ++r) part[(fi * 16 + 4 * r + lq) * NT + n] = acc[q / FN][q % FN][r];
        } else {
          const int ct = gload(pool + blk.c_tabN + w.n0 + n);
          int32_t rt[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) rt[r] = gload(pool + blk.c_tabM + w.m0 + fi * 16 + 4 * r + lq);
          double old[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const bool live = w.m0 + fi * 16 + 4 * r + lq < blk.mext && w.n0 + n < blk.next;
            old[r] = (beta != 0.0 && live) ? Cg[blk.c_off + rt[r] + ct] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const bool live = w.m0 + fi * 16 + 4 * r + lq < blk.mext && w.n0 + n < blk.next;
            const double v = alpha * acc[q / FN][q % FN][r];
            if (live) Cg[blk.c_off + rt[r] + ct] = (beta == 0.0) ? v : beta * old[r] + v;
          }
        }
      }
    } else if (nsplit > 1) {
      double* part = pr.partial + ((int64_t)w.tile + split) * (MT * NT);
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
      // through out's offset tables: every table entry first (the tables are padded, so rows and
      // columns past the block read in bounds), then per row block the old values (beta != 0),
      // then the results, so that no load waits behind the use of another
      const double alpha = pr.alpha, beta = pr.beta;
      __attribute__((address_space(1))) double* __restrict__ Cg = (__attribute__((address_space(1))) double*)pr.C;
      const int mb = w.m0 + wm * WM + lq, nb = w.n0 + wn * WN + lr;
      int32_t rt[FM][4], ct[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) rt[i][r] = gload(pool + blk.c_tabM + mb + i * 16 + 4 * r);
#pragma unroll
      for (int j = 0; j < FN; ++j) ct[j] = gload(pool + blk.c_tabN + nb + j * 16);
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        double old[4][FN];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const bool live = mb + i * 16 + 4 * r < blk.mext && nb + j * 16 < blk.next;
            old[r][j] = (beta != 0.0 && live) ? Cg[blk.c_off + rt[i][r] + ct[j]] : 0.0;
          }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const bool live = mb + i * 16 + 4 * r < blk.mext && nb + j * 16 < blk.next;
            const double v = alpha * acc[i][j][r];
            if (live) Cg[blk.c_off + rt[i][r] + ct[j]] = (beta == 0.0) ? v : beta * old[r][j] + v;
          }
      }
    }
    if (!P.next_item) break;
    __syncthreads();  // s_next is free
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

// Ordered reduction of K-split partial tiles (split 0, 1, ... in order) and the epilogue.  A
// thread takes kReduceUnroll elements at a time and issues all their loads (table entries, then
// the partials and old values) before any use.
constexpr int kReduceUnroll = 4;

__global__ __launch_bounds__(256) void k_reduce(ReduceParams P) {
  const int t = blockIdx.x;
  if (t >= P.n_items) return;
  const ReduceItem it = P.items[t];
  const ProblemDesc& pr = P.probs ? P.probs[it.prob] : P.single;
  const OutBlockDesc blk = pr.blocks[it.ob];
  const int tile = P.tile_m * P.tile_n;
  const double* part = pr.partial + (int64_t)it.tile * tile;
  const double alpha = pr.alpha, beta = pr.beta;
  __attribute__((address_space(1))) double* __restrict__ Cg = (__attribute__((address_space(1))) double*)pr.C;
  for (int e0 = threadIdx.x; e0 < tile; e0 += kReduceUnroll * blockDim.x) {
    int64_t idx[kReduceUnroll];
    bool live[kReduceUnroll];
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u) {
      const int e = e0 + u * blockDim.x;
      const int m = it.m0 + e / P.tile_n, n = it.n0 + e % P.tile_n;
      live[u] = e < tile && m < blk.mext && n < blk.next;
      idx[u] = live[u] ? blk.c_off + pr.pool[blk.c_tabM + m] + pr.pool[blk.c_tabN + n] : 0;
    }
    double s[kReduceUnroll], old[kReduceUnroll];
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u) {
      old[u] = (beta != 0.0 && live[u]) ? Cg[idx[u]] : 0.0;
      s[u] = 0.0;
    }
    for (int k = 0; k < it.nsplit; ++k) {  // split order; the elements' loads of one split together
#pragma unroll
      for (int u = 0; u < kReduceUnroll; ++u) {
        const int e = e0 + u * blockDim.x;
        s[u] += live[u] ? part[(int64_t)k * tile + e] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kReduceUnroll; ++u) {
      const double v = alpha * s[u];
      if (live[u]) Cg[idx[u]] = (beta == 0.0) ? v : beta * old[u] + v;
    }
  }
}

hipError_t launch_reduce(const ReduceParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(p.n_items), dim3(256), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Configurations and dispatch.  X(id, MT, NT, KT, WGM, WGN, OCC): OCC is the minimum number of
// waves per SIMD the register allocation must allow (1 = no constraint).
// ---------------------------------------------------------------------------------------------
#define TAMM_F64_CONFIGS(X)            \
  X(0, 64, 64, 16, 2, 2, 1)            \
  X(1, 128, 64, 16, 2, 2, 1)           \
  X(2, 64, 128, 16, 2, 2, 1)           \
  X(3, 128, 128, 16, 2, 2, 1)          \
  X(4, 32, 64, 16, 2, 2, 1)            \
  X(5, 128, 80, 16, 4, 1, 1)           \
  X(6, 80, 128, 16, 1, 4, 1)           \
  X(7, 64, 80, 16, 4, 1, 1)            \
  X(8, 32, 256, 16, 1, 4, 1)           \
  X(9, 256, 32, 16, 4, 1, 1)           \
  X(10, 128, 128, 32, 2, 2, 1)         \
  X(11, 128, 80, 32, 4, 1, 1)          \
  X(12, 64, 80, 32, 4, 1, 1)           \
  X(13, 64, 64, 32, 2, 2, 1)           \
  X(14, 128, 128, 16, 2, 2, 2)

#define TAMM_CFG_ENTRY(id, mt, nt, kt, wgm, wgn, occ) \
  {mt, nt, kt, wgm, wgn, occ, "f64_m" #mt "n" #nt "k" #kt "_w" #wgm "x" #wgn "_o" #occ},
static const F64Config kF64Configs[] = {TAMM_F64_CONFIGS(TAMM_CFG_ENTRY)};
#undef TAMM_CFG_ENTRY

int f64_config_count() { return (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0])); }
const F64Config& f64_config(int id) { return kF64Configs[id]; }

// Gather layout index: bit 1 = A k-contiguous, bit 0 = B k-contiguous, bit 2 = 16-byte gathers.
// A tile shape whose chunks do not split into pairs runs the 8-byte gather for bit 2 as well.
template <int MT, int NT, int KT, int WGM, int WGN, int OCC, int LAYOUT>
static constexpr auto contract_kernel() {
  constexpr bool akc = (LAYOUT & 2) != 0, bkc = (LAYOUT & 1) != 0;
  constexpr int nthr = 64 * WGM * WGN;
  constexpr bool pairs = (LAYOUT & 4) != 0 && gather_pairs_fit<MT, KT, nthr, akc>() && gather_pairs_fit<NT, KT, nthr, bkc>();
  return k_contract_f64<MT, NT, KT, WGM, WGN, OCC, akc, bkc, pairs ? 2 : 1>;
}

template <int MT, int NT, int KT, int WGM, int WGN, int OCC>
static auto contract_kernel_for(int layout) {
  using K = decltype(contract_kernel<MT, NT, KT, WGM, WGN, OCC, 0>());
  static const K table[8] = {contract_kernel<MT, NT, KT, WGM, WGN, OCC, 0>(), contract_kernel<MT, NT, KT, WGM, WGN, OCC, 1>(),
                             contract_kernel<MT, NT, KT, WGM, WGN, OCC, 2>(), contract_kernel<MT, NT, KT, WGM, WGN, OCC, 3>(),
                             contract_kernel<MT, NT, KT, WGM, WGN, OCC, 4>(), contract_kernel<MT, NT, KT, WGM, WGN, OCC, 5>(),
                             contract_kernel<MT, NT, KT, WGM, WGN, OCC, 6>(), contract_kernel<MT, NT, KT, WGM, WGN, OCC, 7>()};
  return table[layout & 7];
}

template <int MT, int NT, int KT, int WGM, int WGN, int OCC>
static hipError_t launch_cfg(int layout, const ContractParams& p, int grid, hipStream_t s) {
  const dim3 g(grid > 0 ? grid : p.n_work), b(64 * WGM * WGN);
  const auto kernel = contract_kernel_for<MT, NT, KT, WGM, WGN, OCC>(layout);
  hipLaunchKernelGGL(kernel, g, b, 0, s, p);
  return hipGetLastError();
}

template <int MT, int NT, int KT, int WGM, int WGN, int OCC>
static int occupancy_cfg(int layout) {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &n, contract_kernel_for<MT, NT, KT, WGM, WGN, OCC>(layout), 64 * WGM * WGN, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

int f64_occupancy(int config, int layout) {
  switch (config) {
#define TAMM_CFG_OCC(id, mt, nt, kt, wgm, wgn, occ) \
  case id: return occupancy_cfg<mt, nt, kt, wgm, wgn, occ>(layout);
    TAMM_F64_CONFIGS(TAMM_CFG_OCC)
#undef TAMM_CFG_OCC
    default: return 1;
  }
}

hipError_t launch_contract_f64(int config, int layout, const ContractParams& p, int grid, hipStream_t s) {
  if (p.n_work <= 0) return hipSuccess;
  switch (config) {
#define TAMM_CFG_LAUNCH(id, mt, nt, kt, wgm, wgn, occ) \
  case id: return launch_cfg<mt, nt, kt, wgm, wgn, occ>(layout, p, grid, s);
    TAMM_F64_CONFIGS(TAMM_CFG_LAUNCH)
#undef TAMM_CFG_LAUNCH
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// Orbital-energy denominator update.  Each workgroup handles `chunk` consecutive elements of one
// stored block; IEEE float64 division; the denominator is summed in the documented order (the
// energies of the +1 dimensions in dimension order, then minus those of the -1 dimensions).
// A thread splits its first element into per-dimension indices once and then steps by the
// workgroup size with a mixed-radix add, so no integer division runs per element.  Elements go in
// batches of kDenomUnroll per thread whose loads are all issued before any division, so each wave
// keeps that many coalesced loads in flight.
// ---------------------------------------------------------------------------------------------
constexpr int kDenomUnroll = 4;

template <int RANK>
__device__ __forceinline__ void denominator_block(const DenomParams& P, int b, int e0, int e1) {
  int lo[RANK], ext[RANK], idx[RANK], step[RANK];
#pragma unroll
  for (int d = 0; d < RANK; ++d) {
    const int t = P.block_tiles[(int64_t)b * RANK + d];
    lo[d] = (int)P.tile_offset[P.dim_tile_base[d] + t];
    ext[d] = (int)P.tile_size[P.dim_tile_base[d] + t];
  }
  int rem = e0 + (int)threadIdx.x, srem = (int)blockDim.x;
#pragma unroll
  for (int d = RANK - 1; d >= 0; --d) {
    idx[d] = rem % ext[d];
    rem /= ext[d];
    step[d] = srem % ext[d];
    srem /= ext[d];
  }
  const double* __restrict__ in = P.in + P.block_off[b];
  double* __restrict__ out = P.out + P.block_off[b];
  for (int e = e0 + (int)threadIdx.x; e < e1; e += kDenomUnroll * (int)blockDim.x) {
    // all loads of the batch first (the element and its energies), then the arithmetic: no
    // load waits behind another's use
    double x[kDenomUnroll], ev[kDenomUnroll][RANK];
#pragma unroll
    for (int u = 0; u < kDenomUnroll; ++u) {
      const int eu = e + u * (int)blockDim.x;
      x[u] = eu < e1 ? in[eu] : 1.0;
#pragma unroll
      for (int d = 0; d < RANK; ++d) ev[u][d] = P.sign[d] != 0 ? P.energy[d][lo[d] + idx[d]] : 0.0;
      int carry = 0;  // idx += step in the block's mixed radix (each digit stays below 2*ext)
#pragma unroll
      for (int d = RANK - 1; d >= 0; --d) {
        idx[d] += step[d] + carry;
        carry = idx[d] >= ext[d] ? 1 : 0;
        idx[d] -= carry ? ext[d] : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < kDenomUnroll; ++u) {
      double den = 0.0;  // 0 + v and 0 - v are exact: the first term enters unchanged
#pragma unroll
      for (int d = 0; d < RANK; ++d)
        if (P.sign[d] > 0) den += ev[u][d];
#pragma unroll
      for (int d = 0; d < RANK; ++d)
        if (P.sign[d] < 0) den -= ev[u][d];
      const int eu = e + u * (int)blockDim.x;
      if (eu < e1) out[eu] = x[u] / den;
    }
  }
}

template <int RANK>
__global__ __launch_bounds__(256) void k_denominator(DenomParams P) {
  const int64_t it = blockIdx.x;
  if (it >= P.n_items) return;
  const int b = P.item_block[it];
  int n = 1;
#pragma unroll
  for (int d = 0; d < RANK; ++d) n *= (int)P.tile_size[P.dim_tile_base[d] + P.block_tiles[(int64_t)b * RANK + d]];
  const int e0 = P.item_start[it];
  denominator_block<RANK>(P, b, e0, min(n, e0 + P.chunk));
}

hipError_t launch_denominator(const DenomParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  const dim3 g((unsigned)p.n_items), blk(256);
  switch (p.rank) {
    case 1: hipLaunchKernelGGL(k_denominator<1>, g, blk, 0, s, p); break;
    case 2: hipLaunchKernelGGL(k_denominator<2>, g, blk, 0, s, p); break;
    case 3: hipLaunchKernelGGL(k_denominator<3>, g, blk, 0, s, p); break;
    case 4: hipLaunchKernelGGL(k_denominator<4>, g, blk, 0, s, p); break;
    case 5: hipLaunchKernelGGL(k_denominator<5>, g, blk, 0, s, p); break;
    case 6: hipLaunchKernelGGL(k_denominator<6>, g, blk, 0, s, p); break;
    case 7: hipLaunchKernelGGL(k_denominator<7>, g, blk, 0, s, p); break;
    case 8: hipLaunchKernelGGL(k_denominator<8>, g, blk, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tamm
