// Host side of the C ABI, part 1: error reporting, tiled index spaces and block-sparse tensors.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "host.h"

using namespace tamm;

// ---------------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_err;

int tamm::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int tamm::ok() {
  g_err.clear();
  return TAMM_OK;
}

extern "C" const char* tamm_last_error(void) { return g_err.c_str(); }
extern "C" int32_t tamm_version(void) { return 100; }

// ---------------------------------------------------------------------------------------------
// spaces
// ---------------------------------------------------------------------------------------------

static int make_space(std::vector<int64_t> sizes, std::vector<int8_t> spins, tamm_space** out) {
  if (!out) return fail(TAMM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (sizes.empty()) return fail(TAMM_ERR_ARG, "a tiled space needs at least one tile");
  if (sizes.size() > (1u << 20)) return fail(TAMM_ERR_ARG, "too many tiles");
  auto d = std::make_shared<SpaceData>();
  int64_t off = 0;
  for (size_t i = 0; i < sizes.size(); ++i) {
    if (sizes[i] <= 0) return fail(TAMM_ERR_ARG, "tile %zu has non-positive size %lld", i, (long long)sizes[i]);
    if (spins[i] != 0 && spins[i] != 1) return fail(TAMM_ERR_ARG, "tile %zu has spin %d (0 or 1 expected)", i, spins[i]);
    d->offset.push_back(off);
    off += sizes[i];
    if (off > (int64_t)1 << 31) return fail(TAMM_ERR_ARG, "space extent exceeds 2^31");
  }
  d->size = std::move(sizes);
  d->spin = std::move(spins);
  d->extent = off;
  *out = new tamm_space{d};
  return ok();
}

extern "C" int tamm_space_create(const int64_t* tile_sizes, const int8_t* tile_spin, int32_t ntiles, tamm_space** out) {
  if (!tile_sizes || ntiles <= 0) return fail(TAMM_ERR_ARG, "tile_sizes must be non-null and ntiles positive");
  std::vector<int64_t> s(tile_sizes, tile_sizes + ntiles);
  std::vector<int8_t> sp(ntiles, 0);
  if (tile_spin) sp.assign(tile_spin, tile_spin + ntiles);
  return make_space(std::move(s), std::move(sp), out);
}

static void fixed_tiles(int64_t extent, int64_t tile, int8_t spin, std::vector<int64_t>& s, std::vector<int8_t>& sp) {
  for (int64_t i = 0; i + tile <= extent; i += tile) {
    s.push_back(tile);
    sp.push_back(spin);
  }
  if (extent % tile) {
    s.push_back(extent % tile);
    sp.push_back(spin);
  }
}

extern "C" int tamm_space_create_fixed(int64_t extent, int64_t tile, tamm_space** out) {
  if (extent <= 0 || tile <= 0) return fail(TAMM_ERR_ARG, "extent and tile must be positive");
  std::vector<int64_t> s;
  std::vector<int8_t> sp;
  fixed_tiles(extent, tile, 0, s, sp);
  return make_space(std::move(s), std::move(sp), out);
}

extern "C" int tamm_space_create_spin(int64_t n_alpha, int64_t n_beta, int64_t tile, tamm_space** out) {
  if (n_alpha < 0 || n_beta < 0 || tile <= 0 || n_alpha + n_beta <= 0)
    return fail(TAMM_ERR_ARG, "need n_alpha, n_beta >= 0 with a positive sum and a positive tile");
  std::vector<int64_t> s;
  std::vector<int8_t> sp;
  if (n_alpha > 0) fixed_tiles(n_alpha, std::min(tile, n_alpha), 0, s, sp);
  if (n_beta > 0) fixed_tiles(n_beta, std::min(tile, n_beta), 1, s, sp);
  return make_space(std::move(s), std::move(sp), out);
}

extern "C" int tamm_space_info(const tamm_space* s, int32_t* ntiles, int64_t* extent) {
  if (!s) return fail(TAMM_ERR_ARG, "null space");
  if (ntiles) *ntiles = s->d->ntiles();
  if (extent) *extent = s->d->extent;
  return ok();
}

extern "C" int tamm_space_tiles(const tamm_space* s, int64_t* sizes, int64_t* offsets, int8_t* spins) {
  if (!s) return fail(TAMM_ERR_ARG, "null space");
  const SpaceData& d = *s->d;
  for (int t = 0; t < d.ntiles(); ++t) {
    if (sizes) sizes[t] = d.size[t];
    if (offsets) offsets[t] = d.offset[t];
    if (spins) spins[t] = d.spin[t];
  }
  return ok();
}

extern "C" int tamm_space_destroy(tamm_space* s) {
  delete s;
  return ok();
}

// ---------------------------------------------------------------------------------------------
// tensors
// ---------------------------------------------------------------------------------------------

static bool spin_rule(const int8_t* spins, int rank) {
  if (rank % 2) return true;
  int a = 0, b = 0;
  for (int d = 0; d < rank / 2; ++d) a += spins[d];
  for (int d = rank / 2; d < rank; ++d) b += spins[d];
  return a == b;
}

extern "C" int tamm_tensor_create(tamm_space* const* dims, int32_t rank, tamm_nonzero_fn nonzero, void* user, tamm_tensor** out) {
  if (!out) return fail(TAMM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!dims || rank < 1 || rank > kMaxRank) return fail(TAMM_ERR_ARG, "rank must be in [1, %d] and dims non-null", kMaxRank);
  for (int d = 0; d < rank; ++d)
    if (!dims[d]) return fail(TAMM_ERR_ARG, "dimension %d has a null space", d);
  auto t = std::make_unique<tamm_tensor>();
  t->rank = rank;
  int64_t ntup = 1;
  for (int d = 0; d < rank; ++d) {
    t->dims.push_back(dims[d]->d);
    ntup *= dims[d]->d->ntiles();
    if (ntup > (int64_t)1 << 26) return fail(TAMM_ERR_ARG, "too many tile tuples (%lld)", (long long)ntup);
  }
  t->tstride.assign(rank, 1);
  for (int d = rank - 2; d >= 0; --d) t->tstride[d] = t->tstride[d + 1] * t->dims[d + 1]->ntiles();
  t->tile_off.assign(ntup, -1);
  std::vector<int32_t> tile(rank, 0);
  std::vector<int8_t> spin(rank, 0);
  int64_t off = 0;
  for (int64_t lin = 0; lin < ntup; ++lin) {
    int64_t rem = lin, elems = 1;
    for (int d = rank - 1; d >= 0; --d) {
      tile[d] = (int32_t)(rem % t->dims[d]->ntiles());
      rem /= t->dims[d]->ntiles();
      spin[d] = t->dims[d]->spin[tile[d]];
      elems *= t->dims[d]->size[tile[d]];
    }
    const bool keep = nonzero ? nonzero(tile.data(), spin.data(), rank, user) != 0 : spin_rule(spin.data(), rank);
    if (!keep) continue;
    t->tile_off[lin] = off;
    t->block_off.push_back(off);
    t->block_tiles.insert(t->block_tiles.end(), tile.begin(), tile.end());
    t->max_block = std::max(t->max_block, elems);
    off += elems;
  }
  t->numel = off;
  for (int d = 0; d < rank; ++d) {
    t->dim_tile_base.push_back((int32_t)t->tile_offset_cat.size());
    t->tile_offset_cat.insert(t->tile_offset_cat.end(), t->dims[d]->offset.begin(), t->dims[d]->offset.end());
    t->tile_size_cat.insert(t->tile_size_cat.end(), t->dims[d]->size.begin(), t->dims[d]->size.end());
  }
  *out = t.release();
  return ok();
}

extern "C" int tamm_tensor_numel(const tamm_tensor* t, int64_t* numel) {
  if (!t || !numel) return fail(TAMM_ERR_ARG, "null argument");
  *numel = t->numel;
  return ok();
}

extern "C" int tamm_tensor_nbytes(const tamm_tensor* t, size_t* bytes) {
  if (!t || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = (size_t)t->numel * sizeof(double);
  return ok();
}

extern "C" int tamm_tensor_blocks(const tamm_tensor* t, int64_t* nblocks, int32_t* tile_idx, int64_t* elem_off) {
  if (!t || !nblocks) return fail(TAMM_ERR_ARG, "null argument");
  *nblocks = (int64_t)t->block_off.size();
  if (tile_idx) std::copy(t->block_tiles.begin(), t->block_tiles.end(), tile_idx);
  if (elem_off) std::copy(t->block_off.begin(), t->block_off.end(), elem_off);
  return ok();
}

extern "C" int tamm_tensor_bind(tamm_tensor* t, void* dev_ptr, size_t bytes) {
  if (!t) return fail(TAMM_ERR_ARG, "null tensor");
  const size_t need = (size_t)t->numel * sizeof(double);
  if (need > 0 && !dev_ptr) return fail(TAMM_ERR_ARG, "null storage for a tensor with %lld stored elements", (long long)t->numel);
  if (((uintptr_t)dev_ptr) % 8) return fail(TAMM_ERR_ARG, "storage must be 8-byte aligned");
  if (bytes < need) return fail(TAMM_ERR_UNBOUND, "storage of %zu bytes is smaller than the %zu bytes needed", bytes, need);
  t->dev = (double*)dev_ptr;
  t->dev_bytes = bytes;
  t->bound = true;
  return ok();
}

extern "C" int tamm_tensor_destroy(tamm_tensor* t) {
  if (t) tamm::contract_cache_evict(t);
  delete t;
  return ok();
}

