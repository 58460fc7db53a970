// HIP kernels for gfx950: the element-wise operations of the operation grammar -- SetOp (every
// stored element takes one value), AddOp (out = beta*out + alpha*in, in read through a label
// permutation) and AddOp chains (several AddOps into one out in one pass, built by the
// scheduler).  All are bound by HBM bandwidth: each element is read and written once, with
// coalesced accesses on both sides.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace tamm {

// ---------------------------------------------------------------------------------------------
// SetOp.  Two elements per lane and step (16-byte stores), grid-stride.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill(double* __restrict__ p, int64_t n, double v) {
  typedef double d2_t __attribute__((ext_vector_type(2)));
  const int64_t pairs = n / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs; i += stride)
    reinterpret_cast<d2_t*>(p)[i] = (d2_t){v, v};
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) p[n - 1] = v;
}

hipError_t launch_fill(double* p, int64_t n, double value, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (((uintptr_t)p) % 16) {  // 8-byte aligned storage: first element alone, then pairs
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, p, (int64_t)1, value);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ++p;
    --n;
    if (n == 0) return hipSuccess;
  }
  const int64_t blocks = std::min<int64_t>((n / 2 + 255) / 256 + 1, 8192);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// AddOp, direct mode: out and in share their last (stride-1) label, so consecutive lanes read
// and write consecutive elements.  An item is `chunk` consecutive elements of one out block;
// every element's in offset comes from its out index split into the block's mixed radix.
// ---------------------------------------------------------------------------------------------
constexpr int kAddUnroll = 4;

__global__ __launch_bounds__(256) void k_add_direct(AddParams P) {
  const int64_t it = blockIdx.x;
  if (it >= P.n_items) return;
  const AddItem item = P.items[it];
  const AddBlock& B = P.blocks[item.block];
  int n = 1;
  for (int d = 0; d < P.rank; ++d) n *= B.ext[d];
  const int e1 = min(n, item.a + P.chunk);
  const bool has_in = B.in_off >= 0;
  const double* __restrict__ in = P.in + (has_in ? B.in_off : 0);
  double* __restrict__ out = P.out + B.out_off;
  for (int e0 = item.a + (int)threadIdx.x; e0 < e1; e0 += kAddUnroll * (int)blockDim.x) {
    // all loads of the batch first, then the arithmetic and stores
    double x[kAddUnroll], o[kAddUnroll];
#pragma unroll
    for (int u = 0; u < kAddUnroll; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      x[u] = 0.0;
      o[u] = 0.0;
      if (e >= e1) continue;
      if (has_in) {
        int rem = e, off = 0;
        for (int d = P.rank - 1; d >= 0; --d) {
          const int i = rem % B.ext[d];
          rem /= B.ext[d];
          off += i * B.istr[d];
        }
        x[u] = in[off];
      }
      if (P.beta != 0.0) o[u] = out[e];
    }
#pragma unroll
    for (int u = 0; u < kAddUnroll; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      if (e < e1) out[e] = P.beta == 0.0 ? P.alpha * x[u] : P.beta * o[u] + P.alpha * x[u];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// AddOp, transpose mode: in's last label is out dimension ydim, not out's last.  A workgroup
// takes a 32 x 32 tile of the (ydim, last) plane at one value of the other dimensions: lanes
// read in along ydim (in's stride-1 label) into LDS, then write out along its last dimension.
// The LDS tile has a row stride of 33 doubles, so both the column writes and the row reads of a
// wave touch distinct banks.
// ---------------------------------------------------------------------------------------------
constexpr int kAddTile = 32;

__global__ __launch_bounds__(256) void k_add_transpose(AddParams P) {
  __shared__ double tile[kAddTile][kAddTile + 1];
  const int64_t it = blockIdx.x;
  if (it >= P.n_items) return;
  const AddItem item = P.items[it];
  const AddBlock& B = P.blocks[item.block];
  const int r = P.rank, yd = P.ydim, xd = r - 1;
  // out strides (row-major in out's order) and the batch index split over the other dimensions
  int ostr[kMaxRank];
  int s = 1;
  for (int d = r - 1; d >= 0; --d) {
    ostr[d] = s;
    s *= B.ext[d];
  }
  int rem = item.a;
  int64_t obase = B.out_off, ibase = B.in_off;
  for (int d = r - 1; d >= 0; --d) {
    if (d == yd || d == xd) continue;
    const int i = rem % B.ext[d];
    rem /= B.ext[d];
    obase += (int64_t)i * ostr[d];
    ibase += (int64_t)i * B.istr[d];
  }
  const bool has_in = B.in_off >= 0;
  const int ey = B.ext[yd], ex = B.ext[xd];
  const int l = threadIdx.x % kAddTile, k0 = threadIdx.x / kAddTile;  // 8 rows per pass
  constexpr int kPasses = kAddTile / 8;
  // read: lanes along y (in's stride-1 label), rows of the tile along x
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int k = k0 + 8 * q;
    const int y = item.b + l, x = item.c + k;
    double v = 0.0;
    if (has_in && y < ey && x < ex) v = P.in[ibase + y + (int64_t)x * B.istr[xd]];
    tile[k][l] = v;
  }
  __syncthreads();
  // write: lanes along x (out's stride-1 label)
  double o[kPasses];
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int y = item.b + k0 + 8 * q, x = item.c + l;
    o[q] = (P.beta != 0.0 && y < ey && x < ex) ? P.out[obase + (int64_t)y * ostr[yd] + x] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int k = k0 + 8 * q;
    const int y = item.b + k, x = item.c + l;
    if (y < ey && x < ex) {
      const double v = tile[l][k];
      P.out[obase + (int64_t)y * ostr[yd] + x] = P.beta == 0.0 ? P.alpha * v : P.beta * o[q] + P.alpha * v;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// AddOp chain (several AddOps into one out, fused by the scheduler): one 32 x 32 tile of the
// (ydim, last) plane per workgroup, as in k_add_transpose.  Every term's loads are issued before
// any is used; a term whose in ends in out's last label is read along it, one whose in ends in
// label ydim goes through the LDS tile.  The terms are added to beta*out in queue order, each
// product alpha*in and each sum rounded on its own (no fused multiply-add), which is the
// arithmetic of the AddOps applied one after another.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_add_multi(AddMultiParams P) {
#pragma clang fp contract(off)  // every product and every sum rounded once, as AddOps one by one
  __shared__ double tile[kAddTile][kAddTile + 1];
  const int64_t it = blockIdx.x;
  if (it >= P.n_items) return;
  const AddItem item = P.items[it];
  const int r = P.rank, yd = P.ydim, xd = r - 1;
  const AddBlock& B0 = P.blocks[0][item.block];  // out geometry, the same for every term
  int ostr[kMaxRank], idx[kMaxRank];
  int s = 1;
  for (int d = r - 1; d >= 0; --d) {
    ostr[d] = s;
    s *= B0.ext[d];
  }
  int rem = item.a;
  int64_t obase = B0.out_off;
  for (int d = r - 1; d >= 0; --d) {
    idx[d] = 0;
    if (d == yd || d == xd) continue;
    idx[d] = rem % B0.ext[d];
    rem /= B0.ext[d];
    obase += (int64_t)idx[d] * ostr[d];
  }
  const int ey = B0.ext[yd], ex = B0.ext[xd];
  const int l = threadIdx.x % kAddTile, k0 = threadIdx.x / kAddTile;  // 8 rows per pass
  constexpr int kPasses = kAddTile / 8;
  // loads of every term: direct terms at the out element (y0 + k0 + 8q, x0 + l), lanes along x;
  // transposed terms at (y0 + l, x0 + k0 + 8q), lanes along y (in's stride-1 label)
  double v[kMaxAddTerms][kPasses];
#pragma unroll
  for (int t = 0; t < kMaxAddTerms; ++t) {
#pragma unroll
    for (int q = 0; q < kPasses; ++q) v[t][q] = 0.0;
    if (t >= P.nterms) continue;
    const AddBlock& B = P.blocks[t][item.block];
    if (B.in_off < 0) continue;  // block not stored in this term's input: adds zero
    int64_t ibase = B.in_off;
    for (int d = 0; d < r; ++d)
      if (d != yd && d != xd) ibase += (int64_t)idx[d] * B.istr[d];
    const double* __restrict__ in = P.in[t] + ibase;
#pragma unroll
    for (int q = 0; q < kPasses; ++q) {
      const int k = k0 + 8 * q;
      if (P.trans[t]) {
        const int y = item.b + l, x = item.c + k;
        if (y < ey && x < ex) v[t][q] = in[y + (int64_t)x * B.istr[xd]];
      } else {
        const int y = item.b + k, x = item.c + l;
        if (y < ey && x < ex) v[t][q] = in[(int64_t)y * B.istr[yd] + x];
      }
    }
  }
  double acc[kPasses];
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int y = item.b + k0 + 8 * q, x = item.c + l;
    acc[q] = (P.beta != 0.0 && y < ey && x < ex) ? P.beta * P.out[obase + (int64_t)y * ostr[yd] + x] : 0.0;
  }
  // transposed terms through the tile, one after another; then every term into the sum
#pragma unroll
  for (int t = 0; t < kMaxAddTerms; ++t) {
    if (t >= P.nterms) continue;
    if (P.trans[t]) {
      __syncthreads();  // the previous term's reads of the tile are done
#pragma unroll
      for (int q = 0; q < kPasses; ++q) tile[k0 + 8 * q][l] = v[t][q];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPasses; ++q) v[t][q] = tile[l][k0 + 8 * q];
    }
#pragma unroll
    for (int q = 0; q < kPasses; ++q) acc[q] += P.alpha[t] * v[t][q];
  }
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int y = item.b + k0 + 8 * q, x = item.c + l;
    if (y < ey && x < ex) P.out[obase + (int64_t)y * ostr[yd] + x] = acc[q];
  }
}

// Plane mode of the AddOp chain (small planes, contiguous in every input): one workgroup per
// plane, lanes along the flattened plane, so a direct term is one contiguous run of loads; a
// transposed term (its plane stored [x][y]) is read contiguously too and turned through LDS,
// stored with a row stride of ey + 1 doubles so that the transposed reads spread over the banks.
__global__ __launch_bounds__(256) void k_add_multi_plane(AddMultiParams P) {
#pragma clang fp contract(off)  // every product and every sum rounded once, as AddOps one by one
  __shared__ double tile[2 * kAddPlaneMax];
  const int64_t it = blockIdx.x;
  if (it >= P.n_items) return;
  const AddItem item = P.items[it];
  const int r = P.rank, yd = r - 2, xd = r - 1;
  const AddBlock& B0 = P.blocks[0][item.block];
  const int ey = B0.ext[yd], ex = B0.ext[xd], n = ey * ex;
  int idx[kMaxRank];
  int rem = item.a;
  for (int d = r - 3; d >= 0; --d) {
    idx[d] = rem % B0.ext[d];
    rem /= B0.ext[d];
  }
  const int64_t obase = B0.out_off + (int64_t)item.a * n;  // the plane is out's last two dimensions
  constexpr int kPasses = kAddPlaneMax / 256;
  double v[kMaxAddTerms][kPasses];
#pragma unroll
  for (int t = 0; t < kMaxAddTerms; ++t) {
#pragma unroll
    for (int q = 0; q < kPasses; ++q) v[t][q] = 0.0;
    if (t >= P.nterms) continue;
    const AddBlock& B = P.blocks[t][item.block];
    if (B.in_off < 0) continue;  // block not stored in this term's input: adds zero
    int64_t ibase = B.in_off;
    for (int d = 0; d < r - 2; ++d) ibase += (int64_t)idx[d] * B.istr[d];
    const double* __restrict__ in = P.in[t] + ibase;
#pragma unroll
    for (int q = 0; q < kPasses; ++q) {
      const int f = (int)threadIdx.x + 256 * q;
      if (f < n) v[t][q] = in[f];
    }
  }
  double acc[kPasses];
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int f = (int)threadIdx.x + 256 * q;
    acc[q] = (P.beta != 0.0 && f < n) ? P.beta * P.out[obase + f] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < kMaxAddTerms; ++t) {
    if (t >= P.nterms) continue;
    if (P.trans[t]) {
      __syncthreads();  // the previous term's reads of the tile are done
#pragma unroll
      for (int q = 0; q < kPasses; ++q) {
        const int f = (int)threadIdx.x + 256 * q;  // in's plane index: f = x*ey + y
        if (f < n) {
          const int x = f / ey, y = f - x * ey;
          tile[x * (ey + 1) + y] = v[t][q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPasses; ++q) {
        const int f = (int)threadIdx.x + 256 * q;  // out's plane index: f = y*ex + x
        if (f < n) {
          const int y = f / ex, x = f - y * ex;
          v[t][q] = tile[x * (ey + 1) + y];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kPasses; ++q) acc[q] += P.alpha[t] * v[t][q];
  }
#pragma unroll
  for (int q = 0; q < kPasses; ++q) {
    const int f = (int)threadIdx.x + 256 * q;
    if (f < n) P.out[obase + f] = acc[q];
  }
}

hipError_t launch_add_multi(const AddMultiParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  if (p.plane) hipLaunchKernelGGL(k_add_multi_plane, dim3((unsigned)p.n_items), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(k_add_multi, dim3((unsigned)p.n_items), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_add(const AddParams& p, hipStream_t s) {
  if (p.n_items <= 0) return hipSuccess;
  const dim3 g((unsigned)p.n_items), b(256);
  if (p.ydim < 0) hipLaunchKernelGGL(k_add_direct, g, b, 0, s, p);
  else hipLaunchKernelGGL(k_add_transpose, g, b, 0, s, p);
  return hipGetLastError();
}

}  // namespace tamm
