// Device helpers shared by the contraction kernels: bounds-checked buffer loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tamm {

// Largest block the gathers address through one buffer resource (bytes, exclusive): every table
// sum that involves kTableInvalid lands at or beyond it.
constexpr int64_t kMaxBlockBytes = (int64_t)kTableInvalid * 8;

// Loads through explicit address spaces: per-lane table reads as global loads (not flat), and
// wave-uniform descriptor reads as scalar loads from the constant address space (the descriptors
// are never written while a kernel runs).
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ T sload(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized descriptor");
  const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)(p);
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = q[i];
  return __builtin_bit_cast(T, w);
}

// Values the whole wave agrees on, moved to scalar registers (descriptors loaded through
// pointers are not provably uniform to the compiler; a buffer resource in vector registers would
// need a per-lane loop around every load).
__device__ __forceinline__ uint32_t wave_uniform(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
  const uint64_t v = (uint64_t)x;
  return (int64_t)(((uint64_t)wave_uniform((uint32_t)(v >> 32)) << 32) | wave_uniform((uint32_t)v));
}
template <typename T>
__device__ __forceinline__ T* wave_uniform(T* p) {
  return reinterpret_cast<T*>(wave_uniform((int64_t)reinterpret_cast<uintptr_t>(p)));
}
__device__ __forceinline__ PairDesc wave_uniform(const PairDesc& d) {
  PairDesc u;
  u.a_off = wave_uniform(d.a_off);
  u.b_off = wave_uniform(d.b_off);
  u.kext = wave_uniform(d.kext);
  u.a_tabM = wave_uniform(d.a_tabM);
  u.a_tabK = wave_uniform(d.a_tabK);
  u.b_tabK = wave_uniform(d.b_tabK);
  u.b_tabN = wave_uniform(d.b_tabN);
  u.kt = wave_uniform(d.kt);
  return u;
}

__device__ __forceinline__ double wave_uniform(double x) {
  return __builtin_bit_cast(double, wave_uniform(__builtin_bit_cast(int64_t, x)));
}
__device__ __forceinline__ ProblemDesc wave_uniform(const ProblemDesc& d) {
  ProblemDesc u;
  u.A = wave_uniform(d.A);
  u.B = wave_uniform(d.B);
  u.C = wave_uniform(d.C);
  u.blocks = wave_uniform(d.blocks);
  u.pairs = wave_uniform(d.pairs);
  u.counts = wave_uniform(d.counts);
  u.pool = wave_uniform(d.pool);
  u.partial = wave_uniform(d.partial);
  u.alpha = wave_uniform(d.alpha);
  u.beta = wave_uniform(d.beta);
  u.k_splits = wave_uniform(d.k_splits);
  u.a_kc = wave_uniform(d.a_kc);
  u.b_kc = wave_uniform(d.b_kc);
  u.pad = 0;
  u.a_plane = wave_uniform(d.a_plane);
  u.b_plane = wave_uniform(d.b_plane);
  return u;
}
__device__ __forceinline__ WorkItem wave_uniform(const WorkItem& w) {
  return WorkItem{wave_uniform(w.prob), wave_uniform(w.ob), wave_uniform(w.m0), wave_uniform(w.n0), wave_uniform(w.split),
                  wave_uniform(w.tile)};
}
__device__ __forceinline__ OutBlockDesc wave_uniform(const OutBlockDesc& b) {
  OutBlockDesc u;
  u.c_off = wave_uniform(b.c_off);
  u.mext = wave_uniform(b.mext);
  u.next = wave_uniform(b.next);
  u.c_tabM = wave_uniform(b.c_tabM);
  u.c_tabN = wave_uniform(b.c_tabN);
  u.a_tbase = wave_uniform(b.a_tbase);
  u.b_tbase = wave_uniform(b.b_tbase);
  u.a_cbase = wave_uniform(b.a_cbase);
  u.b_cbase = wave_uniform(b.b_cbase);
  u.pair_base = wave_uniform(b.pair_base);
  u.pad = 0;
  return u;
}

// Raw buffer resource over [base, base + bytes) (gfx9 buffer descriptor, 32-bit data format word).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(wave_uniform(base)), (short)0, (int)wave_uniform(bytes),
                                           0x00020000);
}

template <typename T>
__device__ __forceinline__ T buffer_load8(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  static_assert(sizeof(T) == 8, "8-byte element");
  return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}

// V consecutive 8-byte elements (V = 1 or 2) from one bounds-checked buffer load.
template <typename T, int V>
__device__ __forceinline__ void buffer_load_vec(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, T* out) {
  static_assert(sizeof(T) == 8 && (V == 1 || V == 2), "one or two 8-byte elements");
  if constexpr (V == 1) {
    out[0] = buffer_load8<T>(r, byte_off);
  } else {
    struct Pair {
      T x, y;
    };
    const Pair p = __builtin_bit_cast(Pair, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
    out[0] = p.x;
    out[1] = p.y;
  }
}

}  // namespace tamm

namespace tamm {

// Per-thread gather state of one contraction workgroup (shared by the float64 and mixed kernels).
//
// A chunk of A is MT rows x KT summed indices, of B NT rows x KT.  With a k-contiguous operand
// (its stride-1 label is summed) the lanes run along k: a thread owns one group of V
// consecutive k and AE/V rows.  Otherwise the lanes run along the rows: load q of a thread is
// the flat position tid + q*NTHR of the [k][row group] chunk (row groups of V consecutive rows),
// so consecutive lanes read consecutive rows.  When the row-group count divides the thread count
// a thread keeps one row group and AE/V k positions; otherwise (e.g. 80 rows, 256 threads) every
// load has its own row and k.  V = 2 (16-byte loads) is used when the planner has checked that
// every pair of table entries it groups is adjacent in memory.
//
// Everything is branch-free: rows, columns and k positions outside the block read the padding
// entries of the offset tables (kTableInvalid), whose element offset is beyond the buffer
// resource, and the buffer hardware returns zero for them.  Table entries are fetched a chunk
// ahead of the data, so no dependent table->data chain sits in front of the MFMAs.
template <int R, int KT, int NTHR, bool KC, int V>
struct GatherMap {
  static constexpr int E = R * KT / NTHR;                       // elements per thread
  static constexpr int L = E / V;                               // loads per thread
  static constexpr int KG = KT / V;                             // k groups per row (lanes along k)
  static constexpr int RG = R / V;                              // row groups (lanes along rows)
  static constexpr bool ROW_FIXED = !KC && (NTHR % RG == 0);    // one row group per thread
  static constexpr int NR = KC ? L : (ROW_FIXED ? 1 : L);       // distinct row-table entries
  static constexpr int NK = KC ? 1 : L;                         // distinct k-table entries
  static_assert(R * KT % NTHR == 0 && E % V == 0 && R % V == 0 && KT % V == 0, "chunk must split evenly");
  static_assert(KC || (RG * KT) % NTHR == 0, "row-group gather mapping");
  static_assert(!KC || (NTHR % KG == 0 && R % (NTHR / KG) == 0), "k-contiguous gather mapping");
  // row and k of element v of load q
  __device__ static int row(int tid, int q, int v) {
    return KC ? tid / KG + q * (NTHR / KG) : ((tid + q * NTHR) % RG) * V + v;
  }
  __device__ static int k(int tid, int q, int v) { return KC ? (tid % KG) * V + v : (tid + q * NTHR) / RG; }
  __device__ static int ridx(int q) { return KC ? q : (ROW_FIXED ? 0 : q); }  // row entry of load q
  __device__ static int kidx(int q) { return KC ? 0 : q; }                    // k entry of load q
};

// Whether a chunk of R rows x KT splits into 16-byte (two-element) loads under the mapping above.
template <int R, int KT, int NTHR, bool KC>
constexpr bool gather_pairs_fit() {
  const int e = R * KT / NTHR;
  if (R * KT % NTHR != 0 || e % 2 != 0 || R % 2 != 0 || KT % 2 != 0) return false;
  return KC ? (NTHR % (KT / 2) == 0 && R % (NTHR / (KT / 2)) == 0) : ((R / 2) * KT % NTHR == 0);
}

template <int MT, int NT, int KT, int NTHR, bool A_KC, bool B_KC, typename T, int V = 1>
struct Gather {
  using MA = GatherMap<MT, KT, NTHR, A_KC, V>;
  using MB = GatherMap<NT, KT, NTHR, B_KC, V>;
  static constexpr int AE = MA::E, BE = MB::E;
  static constexpr int A_NR = MA::NR, A_NK = MA::NK, B_NR = MB::NR, B_NK = MB::NK;

  int tid;
  const T* a_base;                        // current pair's operand blocks
  const T* b_base;
  uint32_t a_bytes, b_bytes;
  int a_rt[A_NR], b_rt[B_NR];             // row table entries (elements; kTableInvalid past the block)
  int a_kt[A_NK], b_kt[B_NK];             // k table entries (elements; kTableInvalid past the block)
  T ra[AE], rb[BE];                       // element q*V + v: element v of load q

  __device__ void init(int t) { tid = t; }
  __device__ void setup_pair(const PairDesc& d, const int32_t* pool, const T* A, const T* B, int m0, int n0, int mext,
                             int next) {
    a_base = A + d.a_off;
    b_base = B + d.b_off;
    a_bytes = (uint32_t)((int64_t)mext * d.kext * 8);
    b_bytes = (uint32_t)((int64_t)next * d.kext * 8);
#pragma unroll
    for (int q = 0; q < A_NR; ++q) a_rt[q] = gload(pool + d.a_tabM + m0 + MA::row(tid, q, 0));
#pragma unroll
    for (int q = 0; q < B_NR; ++q) b_rt[q] = gload(pool + d.b_tabN + n0 + MB::row(tid, q, 0));
  }
  __device__ void load_tables(const PairDesc& d, const int32_t* pool, int kbase) {
#pragma unroll
    for (int q = 0; q < A_NK; ++q) a_kt[q] = gload(pool + d.a_tabK + kbase + MA::k(tid, q, 0));
#pragma unroll
    for (int q = 0; q < B_NK; ++q) b_kt[q] = gload(pool + d.b_tabK + kbase + MB::k(tid, q, 0));
  }
  __device__ void load_data() {
    // resources built here from wave-uniform values, so that they live in scalar registers
    const __amdgpu_buffer_rsrc_t a_rsrc = block_rsrc(a_base, a_bytes);
    const __amdgpu_buffer_rsrc_t b_rsrc = block_rsrc(b_base, b_bytes);
#pragma unroll
    for (int q = 0; q < MA::L; ++q)
      buffer_load_vec<T, V>(a_rsrc, (uint32_t)(a_rt[MA::ridx(q)] + a_kt[MA::kidx(q)]) * 8u, ra + q * V);
#pragma unroll
    for (int q = 0; q < MB::L; ++q)
      buffer_load_vec<T, V>(b_rsrc, (uint32_t)(b_rt[MB::ridx(q)] + b_kt[MB::kidx(q)]) * 8u, rb + q * V);
  }
  __device__ int a_lds_row(int e) const { return MA::row(tid, e / V, e % V); }
  __device__ int a_lds_k(int e) const { return MA::k(tid, e / V, e % V); }
  __device__ int b_lds_row(int e) const { return MB::row(tid, e / V, e % V); }
  __device__ int b_lds_k(int e) const { return MB::k(tid, e / V, e % V); }
};

// Chunk pipeline of one work item, shared by the contraction kernels.  LDS holds two chunk
// buffers and there is one barrier per chunk: while compute(buf, ...) runs the MFMAs of chunk c
// from buffer `buf`, the stage() callback it calls after its first k-step stores chunk c+1 (in
// registers since the previous chunk) into the other buffer and issues the global loads of
// chunk c+2 into the same registers.  stage() has no branch, so the compiler can interleave its
// LDS stores and global loads with the MFMAs; past the last chunk it moves data nobody reads.
// The bookkeeping that does branch (the next chunk's pair, its table entries) runs in the
// post() callback, which compute calls once its last MFMA is issued.  `flush` tells compute that chunk c ends a promotion window of W
// summed indices or a pair (W = 0: pairs only); the flags travel with the chunks in a FIFO.
// Chunks run over pairs [pb, pe) and KT-long pieces of each.
template <int KT, int W, typename G, typename T, typename StoreF, typename ComputeF>
__device__ __forceinline__ void chunk_pipeline(G& g, const PairDesc* pairs, int pb, int pe, const int32_t* pool,
                                               const T* A, const T* B, int m0, int n0, int mext, int next,
                                               StoreF&& store, ComputeF&& compute) {
  PairDesc d1 = wave_uniform(sload(pairs + pb));  // pair of the chunk whose tables were fetched last
  int p1 = pb, k1 = 0;
  uint32_t fifo = 0;  // flush flags of fetched chunks not yet computed, oldest in bit 0
  int nf = 0;
  auto push = [&]() {
    const int kend = k1 + KT;
    const bool f = kend >= d1.kext || (W > 0 && kend % (W > 0 ? W : 1) == 0);
    fifo |= (f ? 1u : 0u) << nf;
    ++nf;
  };
  auto advance = [&]() {  // table entries of the next chunk; false past the last one
    k1 += KT;
    if (k1 >= d1.kext) {
      ++p1;
      k1 = 0;
      if (p1 >= pe) return false;
      d1 = wave_uniform(sload(pairs + p1));
      g.setup_pair(d1, pool, A, B, m0, n0, mext, next);
    }
    g.load_tables(d1, pool, k1);
    push();
    return true;
  };
  // prologue: chunk 0 into buffer 0, chunk 1 in flight, table entries of chunk 2 in flight
  g.setup_pair(d1, pool, A, B, m0, n0, mext, next);
  g.load_tables(d1, pool, 0);
  push();
  g.load_data();
  bool inflight = advance();  // the next chunk's data is in registers (or on its way)
  store(0);
  bool tabs = false;          // the table entries of the chunk after it are
  if (inflight) {
    g.load_data();
    tabs = advance();
  }
  __syncthreads();
  int buf = 0;
  while (true) {
    const bool flush = (fifo & 1u) != 0;
    fifo >>= 1;
    --nf;
    bool tabs_next = false;
    compute(
        buf, flush,
        [&]() {  // after the first k-step: the next chunk to LDS, the loads of the one after it
          store(buf ^ 1);
          g.load_data();
        },
        [&]() {  // after the last MFMA is issued: the bookkeeping runs while the MFMAs drain
          tabs_next = tabs && advance();
        });
    __syncthreads();  // buffer `buf` is free again; the other one holds the next chunk
    if (!inflight) break;
    inflight = tabs;  // the loads issued in this chunk carried a real chunk
    tabs = tabs_next;
    buf ^= 1;
  }
}

}  // namespace tamm
