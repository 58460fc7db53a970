// Host side of the C ABI, part 3: the orbital-energy denominator update (the Jacobi step that
// turns a residual into amplitudes), prepared once and executed many times.
#include <algorithm>
#include <cstring>
#include <vector>

#include "host.h"

using namespace tamm;

struct tamm_denominator {
  tamm_tensor* out = nullptr;
  const tamm_tensor* in = nullptr;
  int8_t sign[kMaxRank] = {0};
  int32_t chunk = 1024;  // elements per workgroup: one batch of 4 per thread
  std::vector<int32_t> item_block, item_start;
  size_t off_boff = 0, off_btiles = 0, off_toff = 0, off_tsz = 0, off_iblock = 0, off_istart = 0, ws_size = 0;
  char* ws = nullptr;
  bool bound = false;
};

extern "C" int tamm_denominator_create(tamm_tensor* out, const tamm_tensor* in, const int8_t* sign, tamm_denominator** dp) {
  if (!dp) return fail(TAMM_ERR_ARG, "null output pointer");
  *dp = nullptr;
  if (!out || !in || !sign) return fail(TAMM_ERR_ARG, "null argument");
  if (out->rank != in->rank || out->block_off != in->block_off || out->block_tiles != in->block_tiles)
    return fail(TAMM_ERR_SPARSITY, "out and in must have identical block structure");
  for (int d = 0; d < out->rank; ++d)
    if (!out->dims[d]->same(*in->dims[d])) return fail(TAMM_ERR_SPARSITY, "out and in differ in dimension %d", d);
  bool any = false;
  for (int d = 0; d < out->rank; ++d) {
    if (sign[d] < -1 || sign[d] > 1) return fail(TAMM_ERR_ARG, "sign[%d] must be -1, 0 or +1", d);
    any = any || sign[d] != 0;
  }
  if (!any) return fail(TAMM_ERR_ARG, "at least one dimension must carry an energy");
  auto p = std::make_unique<tamm_denominator>();
  p->out = out;
  p->in = in;
  for (int d = 0; d < out->rank; ++d) p->sign[d] = sign[d];
  for (size_t b = 0; b < out->block_off.size(); ++b) {
    int64_t n = 1;
    for (int d = 0; d < out->rank; ++d) n *= out->dims[d]->size[out->block_tiles[b * out->rank + d]];
    if (n > INT32_MAX) return fail(TAMM_ERR_UNSUPPORTED, "block %zu has more than 2^31 elements", b);
    for (int64_t s = 0; s < n; s += p->chunk) {
      p->item_block.push_back((int32_t)b);
      p->item_start.push_back((int32_t)s);
    }
  }
  size_t off = 0;
  p->off_boff = off;
  off = align256(off + out->block_off.size() * 8);
  p->off_btiles = off;
  off = align256(off + out->block_tiles.size() * 4);
  p->off_toff = off;
  off = align256(off + out->tile_offset_cat.size() * 8);
  p->off_tsz = off;
  off = align256(off + out->tile_size_cat.size() * 8);
  p->off_iblock = off;
  off = align256(off + p->item_block.size() * 4);
  p->off_istart = off;
  off = align256(off + p->item_start.size() * 4);
  p->ws_size = std::max<size_t>(off, 256);
  *dp = p.release();
  return ok();
}

extern "C" int tamm_denominator_workspace_size(const tamm_denominator* d, size_t* bytes) {
  if (!d || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = d->ws_size;
  return ok();
}

extern "C" int tamm_denominator_bind_workspace(tamm_denominator* d, void* workspace, size_t bytes) {
  if (!d) return fail(TAMM_ERR_ARG, "null argument");
  if (!workspace || ((uintptr_t)workspace) % 256 || bytes < d->ws_size)
    return fail(TAMM_ERR_WORKSPACE, "workspace must be 256-byte aligned and at least %zu bytes", d->ws_size);
  char* ws = (char*)workspace;
  const tamm_tensor* t = d->out;
  if (!t->block_off.empty()) {
    HIP_TRY(hipMemcpy(ws + d->off_boff, t->block_off.data(), t->block_off.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ws + d->off_btiles, t->block_tiles.data(), t->block_tiles.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ws + d->off_iblock, d->item_block.data(), d->item_block.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ws + d->off_istart, d->item_start.data(), d->item_start.size() * 4, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(ws + d->off_toff, t->tile_offset_cat.data(), t->tile_offset_cat.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws + d->off_tsz, t->tile_size_cat.data(), t->tile_size_cat.size() * 8, hipMemcpyHostToDevice));
  d->ws = ws;
  d->bound = true;
  return ok();
}

void tamm::denominator_io(const tamm_denominator* d, tamm_tensor** out, const tamm_tensor** in) {
  *out = d->out;
  *in = d->in;
}

int tamm::denominator_enqueue(tamm_denominator* d, const double* const* energy, hipStream_t stream) {
  if (!d || !energy) return fail(TAMM_ERR_ARG, "null argument");
  if (!d->bound) return fail(TAMM_ERR_UNBOUND, "denominator workspace is not bound");
  if (!d->out->bound || !d->in->bound) return fail(TAMM_ERR_UNBOUND, "tensor storage not bound");
  const tamm_tensor* t = d->out;
  DenomParams dp{};
  for (int k = 0; k < t->rank; ++k) {
    if (d->sign[k] != 0 && !energy[k]) return fail(TAMM_ERR_ARG, "dimension %d has a sign but no energies", k);
    dp.dim_tile_base[k] = t->dim_tile_base[k];
    dp.energy[k] = energy[k];
    dp.sign[k] = d->sign[k];
  }
  if (d->item_block.empty()) return TAMM_OK;
  dp.out = d->out->dev;
  dp.in = d->in->dev;
  dp.block_off = (const int64_t*)(d->ws + d->off_boff);
  dp.block_tiles = (const int32_t*)(d->ws + d->off_btiles);
  dp.tile_offset = (const int64_t*)(d->ws + d->off_toff);
  dp.tile_size = (const int64_t*)(d->ws + d->off_tsz);
  dp.item_block = (const int32_t*)(d->ws + d->off_iblock);
  dp.item_start = (const int32_t*)(d->ws + d->off_istart);
  dp.rank = t->rank;
  dp.chunk = d->chunk;
  dp.n_items = (int64_t)d->item_block.size();
  HIP_TRY(launch_denominator(dp, stream));
  return TAMM_OK;
}

extern "C" int tamm_denominator_execute(tamm_denominator* d, const double* const* energy, void* stream) {
  const int rc = denominator_enqueue(d, energy, (hipStream_t)stream);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_denominator_destroy(tamm_denominator* d) {
  delete d;
  return ok();
}
