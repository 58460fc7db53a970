// Host side of the C ABI: tiled spaces, block-sparse tensors, label analysis, contraction plans
// (offset tables, screening setup, work decomposition), groups and the denominator update.
#include "../../include/tamm_mi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

using namespace tamm;

// ---------------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int ok() {
  g_err.clear();
  return TAMM_OK;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(TAMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* tamm_last_error(void) { return g_err.c_str(); }
extern "C" int32_t tamm_version(void) { return 100; }

// ---------------------------------------------------------------------------------------------
// spaces
// ---------------------------------------------------------------------------------------------
struct SpaceData {
  std::vector<int64_t> size, offset;
  std::vector<int8_t> spin;
  int64_t extent = 0;
  bool same(const SpaceData& o) const { return size == o.size && spin == o.spin; }
  int ntiles() const { return (int)size.size(); }
};

struct tamm_space {
  std::shared_ptr<SpaceData> d;
};

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
struct tamm_tensor {
  int rank = 0;
  std::vector<std::shared_ptr<SpaceData>> dims;
  std::vector<int64_t> tstride;   // tile-linear strides per dim
  std::vector<int64_t> tile_off;  // per tile-linear index: element offset, -1 = not stored
  std::vector<int32_t> block_tiles;  // stored blocks, rank entries each, lexicographic
  std::vector<int64_t> block_off;
  std::vector<int64_t> tile_offset_cat, tile_size_cat;  // per dim, concatenated
  std::vector<int32_t> dim_tile_base;
  int64_t numel = 0;
  int64_t max_block = 0;
  double* dev = nullptr;
  size_t dev_bytes = 0;
  bool bound = false;
};

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
  delete t;
  return ok();
}

// ---------------------------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------------------------
namespace {

struct Label {
  char c;
  int od = -1, ad = -1, bd = -1;  // dimension in out, A, B (-1 if absent)
  std::shared_ptr<SpaceData> sp;
  std::vector<int32_t> cls;      // size class per tile
  std::vector<int64_t> cls_size; // tile size of each class
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct tamm_plan {
  tamm_tensor* out = nullptr;
  const tamm_tensor* lhs = nullptr;
  const tamm_tensor* rhs = nullptr;
  const tamm_tensor* A = nullptr;  // the operand whose labels are M + K
  const tamm_tensor* B = nullptr;
  bool swapped = false;
  tamm_precision prec = TAMM_PREC_F64;
  std::vector<Label> labels;
  std::vector<int> M, N, K;  // label indices in flattening order (last fastest)
  std::vector<int> k_lhs_order;  // for each K label in lhs order: its position in K
  bool a_kc = true, b_kc = true;
  std::vector<int32_t> pool;
  ScreenParams sp{};
  int64_t n_kt = 1;
  std::vector<OutBlockDesc> blocks;
  std::vector<double> block_cost;
  std::vector<WorkItem> work;
  int config = -1;
  int k_splits = 1;
  int64_t n_tiles = 0;
  tamm_plan_stats stats{};
  // workspace layout
  size_t off_pool = 0, off_atile = 0, off_btile = 0, off_blocks = 0, off_work = 0, off_pairs = 0, off_counts = 0,
         off_partial = 0, ws_size = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_bound = false;
  bool screened = false;
  bool executed = false;
};

static int32_t pool_push(std::vector<int32_t>& pool, const std::vector<int64_t>& v) {
  int32_t start = (int32_t)pool.size();
  for (int64_t x : v) pool.push_back((int32_t)x);
  return start;
}

// Offset table of one label group inside blocks of one operand shape: flattened index (mixed
// radix over `group`, last fastest) -> element offset in the row-major block.
static std::vector<int64_t> group_table(const std::vector<int>& group, const std::vector<int64_t>& lab_ext,
                                        const std::vector<int64_t>& lab_stride) {
  int64_t n = 1;
  for (int l : group) n *= lab_ext[l];
  std::vector<int64_t> tab(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t rem = i, off = 0;
    for (int q = (int)group.size() - 1; q >= 0; --q) {
      const int l = group[q];
      off += (rem % lab_ext[l]) * lab_stride[l];
      rem /= lab_ext[l];
    }
    tab[i] = off;
  }
  return tab;
}

static int configure_work(tamm_plan* p, int config, int k_splits);

extern "C" int tamm_plan_create(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                                const tamm_tensor* rhs, const char* rhs_lbl, tamm_precision precision, tamm_plan** plan) {
  if (!plan) return fail(TAMM_ERR_ARG, "null output pointer");
  *plan = nullptr;
  if (!out || !lhs || !rhs || !out_lbl || !lhs_lbl || !rhs_lbl) return fail(TAMM_ERR_ARG, "null tensor or label string");
  if (precision != TAMM_PREC_F64)
    return fail(TAMM_ERR_UNSUPPORTED, "precision %d is not available in this build", (int)precision);
  const tamm_tensor* ts[3] = {out, lhs, rhs};
  const char* ls[3] = {out_lbl, lhs_lbl, rhs_lbl};
  for (int x = 0; x < 3; ++x) {
    const size_t n = strlen(ls[x]);
    if ((int)n != ts[x]->rank)
      return fail(TAMM_ERR_SHAPE, "label string '%s' has %zu letters for a rank-%d tensor", ls[x], n, ts[x]->rank);
    for (size_t i = 0; i < n; ++i) {
      const char c = ls[x][i];
      if (!((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'))) return fail(TAMM_ERR_LABEL, "label '%c' is not a letter", c);
      for (size_t j = 0; j < i; ++j)
        if (ls[x][j] == c) return fail(TAMM_ERR_LABEL, "label '%c' repeats inside '%s'", c, ls[x]);
    }
  }
  auto p = std::make_unique<tamm_plan>();
  p->out = out;
  p->lhs = lhs;
  p->rhs = rhs;
  p->prec = precision;
  // orientation: the operand holding out's last label becomes B, so output stores run along N
  const char last = out_lbl[out->rank - 1];
  p->swapped = strchr(lhs_lbl, last) != nullptr;
  p->A = p->swapped ? rhs : lhs;
  p->B = p->swapped ? lhs : rhs;
  const char* a_lbl = p->swapped ? rhs_lbl : lhs_lbl;
  const char* b_lbl = p->swapped ? lhs_lbl : rhs_lbl;
  std::map<char, int> idx;
  auto touch = [&](char c) -> Label& {
    auto it = idx.find(c);
    if (it == idx.end()) {
      idx[c] = (int)p->labels.size();
      p->labels.push_back(Label{c});
      return p->labels.back();
    }
    return p->labels[it->second];
  };
  for (int d = 0; d < out->rank; ++d) touch(out_lbl[d]).od = d;
  for (int d = 0; d < p->A->rank; ++d) touch(a_lbl[d]).ad = d;
  for (int d = 0; d < p->B->rank; ++d) touch(b_lbl[d]).bd = d;
  for (auto& L : p->labels) {
    const int n = (L.od >= 0) + (L.ad >= 0) + (L.bd >= 0);
    if (n != 2) return fail(TAMM_ERR_LABEL, "label '%c' appears in %d tensors; each label must appear in exactly two", L.c, n);
    std::shared_ptr<SpaceData> s[3] = {L.od >= 0 ? out->dims[L.od] : nullptr, L.ad >= 0 ? p->A->dims[L.ad] : nullptr,
                                       L.bd >= 0 ? p->B->dims[L.bd] : nullptr};
    for (int x = 0; x < 3; ++x)
      if (s[x]) {
        if (!L.sp) L.sp = s[x];
        else if (!L.sp->same(*s[x])) return fail(TAMM_ERR_LABEL, "label '%c' binds two different tiled spaces", L.c);
      }
    // size classes: distinct tile sizes in order of first appearance
    for (int t = 0; t < L.sp->ntiles(); ++t) {
      auto it = std::find(L.cls_size.begin(), L.cls_size.end(), L.sp->size[t]);
      if (it == L.cls_size.end()) {
        L.cls.push_back((int32_t)L.cls_size.size());
        L.cls_size.push_back(L.sp->size[t]);
      } else {
        L.cls.push_back((int32_t)(it - L.cls_size.begin()));
      }
    }
  }
  const int nl = (int)p->labels.size();
  // flattening orders: M and N follow the operand's own dimension order; K follows the operand
  // whose stride-1 label is a K label (A first), so that gathers run along memory.
  std::vector<int> a_dim_label(p->A->rank), b_dim_label(p->B->rank), o_dim_label(out->rank);
  for (int l = 0; l < nl; ++l) {
    if (p->labels[l].ad >= 0) a_dim_label[p->labels[l].ad] = l;
    if (p->labels[l].bd >= 0) b_dim_label[p->labels[l].bd] = l;
    if (p->labels[l].od >= 0) o_dim_label[p->labels[l].od] = l;
  }
  for (int d = 0; d < p->A->rank; ++d)
    if (p->labels[a_dim_label[d]].od >= 0) p->M.push_back(a_dim_label[d]);
  for (int d = 0; d < p->B->rank; ++d)
    if (p->labels[b_dim_label[d]].od >= 0) p->N.push_back(b_dim_label[d]);
  const int a_last = a_dim_label[p->A->rank - 1], b_last = b_dim_label[p->B->rank - 1];
  p->a_kc = p->labels[a_last].od < 0;
  p->b_kc = p->labels[b_last].od < 0;
  if (p->a_kc || !p->b_kc) {
    for (int d = 0; d < p->A->rank; ++d)
      if (p->labels[a_dim_label[d]].od < 0) p->K.push_back(a_dim_label[d]);
  } else {
    for (int d = 0; d < p->B->rank; ++d)
      if (p->labels[b_dim_label[d]].od < 0) p->K.push_back(b_dim_label[d]);
  }
  if (p->K.size() > (size_t)kMaxRank) return fail(TAMM_ERR_UNSUPPORTED, "too many contracted labels");
  for (int i = 0; lhs_lbl[i]; ++i) {
    const int l = idx[lhs_lbl[i]];
    if (p->labels[l].od < 0) p->k_lhs_order.push_back((int)(std::find(p->K.begin(), p->K.end(), l) - p->K.begin()));
  }

  // ---- offset tables per operand shape class --------------------------------------------------
  auto& pool = p->pool;
  struct OpInfo {
    const tamm_tensor* t;
    std::vector<int> dim_label;
    std::vector<int64_t> cstride;  // class-id stride per dim
    int64_t ncls = 1;
  };
  auto op_info = [&](const tamm_tensor* t, const std::vector<int>& dl) {
    OpInfo o{t, dl, std::vector<int64_t>(t->rank, 1), 1};
    for (int d = t->rank - 1; d >= 0; --d) {
      o.cstride[d] = o.ncls;
      o.ncls *= (int64_t)p->labels[dl[d]].cls_size.size();
    }
    return o;
  };
  OpInfo ai = op_info(p->A, a_dim_label), bi = op_info(p->B, b_dim_label), oi = op_info(out, o_dim_label);
  if (ai.ncls + bi.ncls + oi.ncls > 100000) return fail(TAMM_ERR_UNSUPPORTED, "too many distinct block shapes");
  // for every class of an operand: per-label extents and element strides, then the two tables
  auto build_tables = [&](const OpInfo& o, const std::vector<int>& g1, const std::vector<int>& g2,
                          std::vector<int64_t>& start1, std::vector<int64_t>& start2) {
    start1.assign(o.ncls, 0);
    start2.assign(o.ncls, 0);
    std::vector<int64_t> lab_ext(nl, 1), lab_stride(nl, 0);
    for (int64_t c = 0; c < o.ncls; ++c) {
      int64_t stride = 1;
      for (int d = o.t->rank - 1; d >= 0; --d) {
        const Label& L = p->labels[o.dim_label[d]];
        const int64_t cl = (c / o.cstride[d]) % (int64_t)L.cls_size.size();
        lab_ext[o.dim_label[d]] = L.cls_size[cl];
        lab_stride[o.dim_label[d]] = stride;
        stride *= L.cls_size[cl];
      }
      if (stride > INT32_MAX) return false;
      start1[c] = pool_push(pool, group_table(g1, lab_ext, lab_stride));
      start2[c] = pool_push(pool, group_table(g2, lab_ext, lab_stride));
    }
    return true;
  };
  std::vector<int64_t> aM, aK, bK, bN, oM, oN;
  if (!build_tables(ai, p->M, p->K, aM, aK) || !build_tables(bi, p->K, p->N, bK, bN) || !build_tables(oi, p->M, p->N, oM, oN))
    return fail(TAMM_ERR_UNSUPPORTED, "a block has more than 2^31 elements");
  if (pool.size() > (size_t)INT32_MAX / 2) return fail(TAMM_ERR_UNSUPPORTED, "offset tables too large");
  ScreenParams& sp = p->sp;
  sp.a_cls_tabM = pool_push(pool, aM);
  sp.a_cls_tabK = pool_push(pool, aK);
  sp.b_cls_tabK = pool_push(pool, bK);
  sp.b_cls_tabN = pool_push(pool, bN);
  sp.nk = (int)p->K.size();
  p->n_kt = 1;
  for (int q = 0; q < sp.nk; ++q) {
    const Label& L = p->labels[p->K[q]];
    sp.k_ntiles[q] = L.sp->ntiles();
    p->n_kt *= L.sp->ntiles();
    sp.a_tstride[q] = (int32_t)p->A->tstride[L.ad];
    sp.b_tstride[q] = (int32_t)p->B->tstride[L.bd];
    sp.a_cstride[q] = (int32_t)ai.cstride[L.ad];
    sp.b_cstride[q] = (int32_t)bi.cstride[L.bd];
    sp.k_size_tab[q] = pool_push(pool, L.sp->size);
    std::vector<int64_t> cls(L.cls.begin(), L.cls.end());
    sp.k_cls_tab[q] = pool_push(pool, cls);
  }
  if (p->n_kt > (1 << 20)) return fail(TAMM_ERR_UNSUPPORTED, "too many contracted tile tuples");
  sp.n_kt = (int32_t)p->n_kt;

  // ---- output blocks, host structural screening statistics ------------------------------------
  const int64_t nob = (int64_t)out->block_off.size();
  if (nob * p->n_kt > (int64_t)1 << 28) return fail(TAMM_ERR_UNSUPPORTED, "pair capacity too large");
  p->blocks.resize(nob);
  p->block_cost.assign(nob, 0.0);
  std::vector<int32_t> kt_tiles(sp.nk);
  double flops = 0;
  int64_t tasks = 0;
  for (int64_t b = 0; b < nob; ++b) {
    const int32_t* ot = &out->block_tiles[b * out->rank];
    OutBlockDesc& d = p->blocks[b];
    memset(&d, 0, sizeof(d));
    d.c_off = out->block_off[b];
    int64_t mext = 1, next = 1, ocls = 0;
    for (int l : p->M) mext *= p->labels[l].sp->size[ot[p->labels[l].od]];
    for (int l : p->N) next *= p->labels[l].sp->size[ot[p->labels[l].od]];
    for (int dd = 0; dd < out->rank; ++dd) ocls += p->labels[o_dim_label[dd]].cls[ot[dd]] * oi.cstride[dd];
    d.mext = (int32_t)mext;
    d.next = (int32_t)next;
    d.c_tabM = (int32_t)oM[ocls];
    d.c_tabN = (int32_t)oN[ocls];
    int64_t atb = 0, btb = 0, acb = 0, bcb = 0;
    for (int l : p->M) {
      const Label& L = p->labels[l];
      atb += ot[L.od] * p->A->tstride[L.ad];
      acb += L.cls[ot[L.od]] * ai.cstride[L.ad];
    }
    for (int l : p->N) {
      const Label& L = p->labels[l];
      btb += ot[L.od] * p->B->tstride[L.bd];
      bcb += L.cls[ot[L.od]] * bi.cstride[L.bd];
    }
    d.a_tbase = (int32_t)atb;
    d.b_tbase = (int32_t)btb;
    d.a_cbase = (int32_t)acb;
    d.b_cbase = (int32_t)bcb;
    d.pair_base = (int32_t)(b * p->n_kt);
    // host count of surviving pairs (statistics and scheduling cost only; the kernel's pair list
    // comes from the GPU screen)
    for (int64_t kt = 0; kt < p->n_kt; ++kt) {
      int64_t rem = kt, alin = atb, blin = btb, kext = 1;
      for (int q = sp.nk - 1; q >= 0; --q) {
        const int t = (int)(rem % sp.k_ntiles[q]);
        rem /= sp.k_ntiles[q];
        alin += (int64_t)t * sp.a_tstride[q];
        blin += (int64_t)t * sp.b_tstride[q];
        kext *= p->labels[p->K[q]].sp->size[t];
      }
      if (p->A->tile_off[alin] >= 0 && p->B->tile_off[blin] >= 0) {
        ++tasks;
        flops += 2.0 * (double)mext * (double)next * (double)kext;
        p->block_cost[b] += (double)kext;
      }
    }
  }
  // dropped pairs: surviving pairs whose output block is not stored (user predicates only)
  int64_t dropped = 0;
  {
    std::vector<int32_t> ot(out->rank);
    const int64_t ntup = (int64_t)out->tile_off.size();
    for (int64_t lin = 0; lin < ntup; ++lin) {
      if (out->tile_off[lin] >= 0) continue;
      int64_t rem = lin;
      for (int dd = out->rank - 1; dd >= 0; --dd) {
        ot[dd] = (int32_t)(rem % out->dims[dd]->ntiles());
        rem /= out->dims[dd]->ntiles();
      }
      int64_t atb = 0, btb = 0;
      for (int l : p->M) atb += ot[p->labels[l].od] * p->A->tstride[p->labels[l].ad];
      for (int l : p->N) btb += ot[p->labels[l].od] * p->B->tstride[p->labels[l].bd];
      for (int64_t kt = 0; kt < p->n_kt; ++kt) {
        int64_t r2 = kt, alin = atb, blin = btb;
        for (int q = sp.nk - 1; q >= 0; --q) {
          const int t = (int)(r2 % sp.k_ntiles[q]);
          r2 /= sp.k_ntiles[q];
          alin += (int64_t)t * sp.a_tstride[q];
          blin += (int64_t)t * sp.b_tstride[q];
        }
        if (p->A->tile_off[alin] >= 0 && p->B->tile_off[blin] >= 0) ++dropped;
      }
    }
  }
  tamm_plan_stats& st = p->stats;
  st.out_blocks = nob;
  st.candidates = nob * p->n_kt;
  st.tasks = tasks;
  st.dropped = dropped;
  st.useful_flops = flops;
  st.algorithmic_bytes = 8.0 * ((double)lhs->numel + (double)rhs->numel + 2.0 * (double)out->numel);
  int rc = configure_work(p.get(), -1, 0);
  if (rc != TAMM_OK) return rc;
  *plan = p.release();
  return ok();
}

// Work decomposition for one kernel configuration: macro-tiles of every stored output block,
// heaviest first (longest-processing-time order), with the K splits of a tile adjacent.
static int configure_work(tamm_plan* p, int config, int k_splits) {
  const int ncfg = f64_config_count();
  const int64_t nob = (int64_t)p->blocks.size();
  auto tiles_for = [&](int c) {
    const F64Config& f = f64_config(c);
    int64_t n = 0;
    double area = 0, useful = 0;
    for (const auto& b : p->blocks) {
      const int64_t tm = (b.mext + f.mt - 1) / f.mt, tn = (b.next + f.nt - 1) / f.nt;
      n += tm * tn;
      area += (double)tm * f.mt * tn * f.nt;
      useful += (double)b.mext * b.next;
    }
    return std::make_pair(n, useful > 0 ? area / useful : 1.0);
  };
  if (config < 0) {
    // default: the largest tile that still gives every compute unit two tiles and wastes at most
    // 15% to padding; otherwise the smallest-waste configuration.  The autotuner overrides this.
    int best = 0;
    double best_score = -1;
    for (int c = 0; c < ncfg; ++c) {
      auto [n, waste] = tiles_for(c);
      const F64Config& f = f64_config(c);
      double score = (double)f.mt * f.nt / waste;
      if (n < 512) score *= (double)n / 512.0;
      if (score > best_score) {
        best_score = score;
        best = c;
      }
    }
    config = best;
  }
  if (config >= ncfg) return fail(TAMM_ERR_ARG, "kernel configuration %d does not exist (%d available)", config, ncfg);
  const F64Config& f = f64_config(config);
  auto [ntiles, waste] = tiles_for(config);
  (void)waste;
  if (k_splits <= 0) {
    k_splits = 1;
    // output-starved operations: split K so that there are about two tiles per compute unit
    if (ntiles > 0 && ntiles < 512) {
      double maxk = 0;
      for (double c : p->block_cost) maxk = std::max(maxk, c);
      const int want = (int)((512 + ntiles - 1) / ntiles);
      const int kmax = (int)std::max(1.0, maxk / (4.0 * f.kt));
      k_splits = std::max(1, std::min({want, 16, kmax}));
    }
  }
  if (k_splits > 64) return fail(TAMM_ERR_ARG, "k_splits must be in [1, 64]");
  struct Tile {
    double cost;
    int32_t ob, m0, n0;
  };
  std::vector<Tile> tiles;
  tiles.reserve(ntiles);
  for (int64_t b = 0; b < nob; ++b) {
    const auto& d = p->blocks[b];
    for (int32_t m0 = 0; m0 < d.mext; m0 += f.mt)
      for (int32_t n0 = 0; n0 < d.next; n0 += f.nt)
        tiles.push_back(Tile{p->block_cost[b] * std::min(f.mt, d.mext - m0) * std::min(f.nt, d.next - n0), (int32_t)b, m0, n0});
  }
  std::stable_sort(tiles.begin(), tiles.end(), [](const Tile& x, const Tile& y) { return x.cost > y.cost; });
  p->work.clear();
  for (const Tile& t : tiles)
    for (int s = 0; s < k_splits; ++s) p->work.push_back(WorkItem{t.ob, t.m0, t.n0, s});
  if (p->work.size() > (size_t)INT32_MAX / 2) return fail(TAMM_ERR_UNSUPPORTED, "too many work items");
  p->config = config;
  p->k_splits = k_splits;
  p->n_tiles = (int64_t)tiles.size();
  p->stats.work_items = (int64_t)p->work.size();
  p->stats.kernel_config = config;
  p->stats.k_splits = k_splits;
  // workspace layout
  size_t off = 0;
  p->off_pool = off;
  off = align256(off + p->pool.size() * sizeof(int32_t));
  p->off_atile = off;
  off = align256(off + p->A->tile_off.size() * sizeof(int64_t));
  p->off_btile = off;
  off = align256(off + p->B->tile_off.size() * sizeof(int64_t));
  p->off_blocks = off;
  off = align256(off + p->blocks.size() * sizeof(OutBlockDesc));
  p->off_work = off;
  off = align256(off + p->work.size() * sizeof(WorkItem));
  p->off_pairs = off;
  off = align256(off + (size_t)nob * (size_t)p->n_kt * sizeof(PairDesc));
  p->off_counts = off;
  off = align256(off + (size_t)nob * sizeof(int32_t));
  p->off_partial = off;
  if (k_splits > 1) off = align256(off + p->work.size() * (size_t)f.mt * f.nt * sizeof(double));
  p->ws_size = std::max<size_t>(off, 256);
  p->ws_bound = false;
  p->screened = false;
  p->executed = false;
  return TAMM_OK;
}

extern "C" int tamm_plan_workspace_size(const tamm_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = p->ws_size;
  return ok();
}

extern "C" int tamm_plan_bind_workspace(tamm_plan* p, void* dev_ptr, size_t bytes) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  if (!dev_ptr || ((uintptr_t)dev_ptr) % 256) return fail(TAMM_ERR_WORKSPACE, "workspace must be non-null and 256-byte aligned");
  if (bytes < p->ws_size) return fail(TAMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, p->ws_size);
  char* ws = (char*)dev_ptr;
  HIP_TRY(hipMemcpy(ws + p->off_pool, p->pool.data(), p->pool.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws + p->off_atile, p->A->tile_off.data(), p->A->tile_off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws + p->off_btile, p->B->tile_off.data(), p->B->tile_off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  if (!p->blocks.empty())
    HIP_TRY(hipMemcpy(ws + p->off_blocks, p->blocks.data(), p->blocks.size() * sizeof(OutBlockDesc), hipMemcpyHostToDevice));
  if (!p->work.empty())
    HIP_TRY(hipMemcpy(ws + p->off_work, p->work.data(), p->work.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  p->ws = ws;
  p->ws_bytes = bytes;
  p->ws_bound = true;
  p->screened = false;
  p->executed = false;
  return ok();
}

extern "C" int tamm_plan_stats_get(const tamm_plan* p, tamm_plan_stats* s) {
  if (!p || !s) return fail(TAMM_ERR_ARG, "null argument");
  *s = p->stats;
  return ok();
}

extern "C" int tamm_plan_config_count(const tamm_plan* p, int32_t* count) {
  if (!p || !count) return fail(TAMM_ERR_ARG, "null argument");
  *count = f64_config_count();
  return ok();
}

extern "C" int tamm_plan_set_config(tamm_plan* p, int32_t config, int32_t k_splits) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  if (config < 0 || config >= f64_config_count()) return fail(TAMM_ERR_ARG, "configuration %d does not exist", config);
  if (k_splits < 0 || k_splits > 64) return fail(TAMM_ERR_ARG, "k_splits must be in [0, 64]");
  const int rc = configure_work(p, config, k_splits);
  if (rc != TAMM_OK) return rc;
  return ok();
}

extern "C" const char* tamm_config_name(int32_t precision, int32_t config) {
  if (precision != TAMM_PREC_F64 || config < 0 || config >= f64_config_count()) return "";
  return f64_config(config).name;
}

static bool overlaps(const tamm_tensor* a, const tamm_tensor* b) {
  if (a->numel == 0 || b->numel == 0) return false;
  const char* a0 = (const char*)a->dev;
  const char* b0 = (const char*)b->dev;
  return a0 < b0 + b->numel * 8 && b0 < a0 + a->numel * 8;
}

static int check_bound(const tamm_plan* p) {
  if (!p->ws_bound) return fail(TAMM_ERR_UNBOUND, "plan workspace is not bound (or the configuration changed since binding)");
  const tamm_tensor* ts[3] = {p->out, p->lhs, p->rhs};
  const char* nm[3] = {"out", "lhs", "rhs"};
  for (int x = 0; x < 3; ++x)
    if (!ts[x]->bound) return fail(TAMM_ERR_UNBOUND, "%s tensor has no bound storage", nm[x]);
  if (overlaps(p->out, p->lhs) || overlaps(p->out, p->rhs)) return fail(TAMM_ERR_ARG, "out storage overlaps an operand");
  return TAMM_OK;
}

static void fill_screen_ptrs(tamm_plan* p, ScreenParams& s) {
  s = p->sp;
  s.a_tile_off = (const int64_t*)(p->ws + p->off_atile);
  s.b_tile_off = (const int64_t*)(p->ws + p->off_btile);
  s.blocks = (const OutBlockDesc*)(p->ws + p->off_blocks);
  s.pairs = (PairDesc*)(p->ws + p->off_pairs);
  s.counts = (int32_t*)(p->ws + p->off_counts);
  s.pool = (const int32_t*)(p->ws + p->off_pool);
  s.n_blocks = (int32_t)p->blocks.size();
}

static void fill_contract_params(tamm_plan* p, ContractParams& c, double alpha, double beta) {
  c.A = p->A->dev;
  c.B = p->B->dev;
  c.C = p->out->dev;
  c.blocks = (const OutBlockDesc*)(p->ws + p->off_blocks);
  c.pairs = (const PairDesc*)(p->ws + p->off_pairs);
  c.counts = (const int32_t*)(p->ws + p->off_counts);
  c.pool = (const int32_t*)(p->ws + p->off_pool);
  c.work = (const WorkItem*)(p->ws + p->off_work);
  c.partial = p->k_splits > 1 ? (double*)(p->ws + p->off_partial) : nullptr;
  c.n_work = (int32_t)p->work.size();
  c.k_splits = p->k_splits;
  c.alpha = alpha;
  c.beta = beta;
}

extern "C" int tamm_plan_screen(tamm_plan* p, void* stream) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  int rc = check_bound(p);
  if (rc != TAMM_OK) return rc;
  ScreenParams sp;
  fill_screen_ptrs(p, sp);
  HIP_TRY(launch_screen(sp, (hipStream_t)stream));
  p->screened = true;
  return ok();
}

extern "C" int tamm_plan_contract(tamm_plan* p, double alpha, double beta, void* stream) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  int rc = check_bound(p);
  if (rc != TAMM_OK) return rc;
  if (!p->screened) return fail(TAMM_ERR_UNBOUND, "the plan has not been screened on its bound workspace");
  hipStream_t s = (hipStream_t)stream;
  ContractParams cp;
  fill_contract_params(p, cp, alpha, beta);
  HIP_TRY(launch_contract_f64(p->config, p->a_kc, p->b_kc, cp, s));
  if (p->k_splits > 1) {
    const F64Config& f = f64_config(p->config);
    ReduceParams r;
    r.C = p->out->dev;
    r.blocks = cp.blocks;
    r.pool = cp.pool;
    r.work = cp.work;
    r.partial = cp.partial;
    r.n_tiles = (int32_t)p->n_tiles;
    r.k_splits = p->k_splits;
    r.tile_m = f.mt;
    r.tile_n = f.nt;
    r.alpha = alpha;
    r.beta = beta;
    HIP_TRY(launch_reduce(r, s));
  }
  p->executed = true;
  return ok();
}

extern "C" int tamm_plan_execute(tamm_plan* p, double alpha, double beta, void* stream) {
  int rc = tamm_plan_screen(p, stream);
  if (rc != TAMM_OK) return rc;
  return tamm_plan_contract(p, alpha, beta, stream);
}

extern "C" int tamm_plan_screen_result(tamm_plan* p, void* stream, int32_t* counts, int32_t* k_tiles) {
  if (!p || !counts) return fail(TAMM_ERR_ARG, "null argument");
  if (!p->ws_bound || !p->executed) return fail(TAMM_ERR_UNBOUND, "plan has not been executed on a bound workspace");
  const size_t nob = p->blocks.size();
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(counts, p->ws + p->off_counts, nob * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (k_tiles) {
    std::vector<PairDesc> pairs((size_t)nob * p->n_kt);
    HIP_TRY(hipMemcpy(pairs.data(), p->ws + p->off_pairs, pairs.size() * sizeof(PairDesc), hipMemcpyDeviceToHost));
    const int nk = p->sp.nk;
    std::vector<int> t(nk);
    size_t w = 0;
    for (size_t b = 0; b < nob; ++b)
      for (int i = 0; i < counts[b]; ++i) {
        int rem = pairs[b * p->n_kt + i].kt;
        for (int q = nk - 1; q >= 0; --q) {
          t[q] = rem % p->sp.k_ntiles[q];
          rem /= p->sp.k_ntiles[q];
        }
        for (int j = 0; j < nk; ++j) k_tiles[w++] = t[p->k_lhs_order[j]];
      }
  }
  return ok();
}

extern "C" int tamm_plan_destroy(tamm_plan* p) {
  delete p;
  return ok();
}

// ---------------------------------------------------------------------------------------------
// groups (not yet available)
// ---------------------------------------------------------------------------------------------
struct tamm_group {
  int dummy;
};

extern "C" int tamm_group_create(tamm_plan* const*, int32_t, tamm_group** g) {
  if (g) *g = nullptr;
  return fail(TAMM_ERR_UNSUPPORTED, "groups are not available in this build");
}
extern "C" int tamm_group_workspace_size(const tamm_group*, size_t*) { return fail(TAMM_ERR_UNSUPPORTED, "groups are not available"); }
extern "C" int tamm_group_bind_workspace(tamm_group*, void*, size_t) { return fail(TAMM_ERR_UNSUPPORTED, "groups are not available"); }
extern "C" int tamm_group_set_config(tamm_group*, int32_t, int32_t) { return fail(TAMM_ERR_UNSUPPORTED, "groups are not available"); }
extern "C" int tamm_group_execute(tamm_group*, const double*, const double*, void*) {
  return fail(TAMM_ERR_UNSUPPORTED, "groups are not available");
}
extern "C" int tamm_group_destroy(tamm_group* g) {
  delete g;
  return ok();
}

// ---------------------------------------------------------------------------------------------
// denominator update
// ---------------------------------------------------------------------------------------------
extern "C" int tamm_denominator_workspace_size(const tamm_tensor* t, size_t* bytes) {
  if (!t || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = align256(t->block_off.size() * 8) + align256(t->block_tiles.size() * 4) + 2 * align256(t->tile_offset_cat.size() * 8);
  return ok();
}

extern "C" int tamm_denominator_update(tamm_tensor* out, const tamm_tensor* in, const double* const* energy, const int8_t* sign,
                                       void* workspace, size_t ws_bytes, void* stream) {
  if (!out || !in || !energy || !sign) return fail(TAMM_ERR_ARG, "null argument");
  if (out->rank != in->rank || out->block_off != in->block_off || out->block_tiles != in->block_tiles)
    return fail(TAMM_ERR_SPARSITY, "out and in must have identical block structure");
  for (int d = 0; d < out->rank; ++d)
    if (!out->dims[d]->same(*in->dims[d])) return fail(TAMM_ERR_SPARSITY, "out and in differ in dimension %d", d);
  if (!out->bound || !in->bound) return fail(TAMM_ERR_UNBOUND, "tensor storage not bound");
  for (int d = 0; d < out->rank; ++d)
    if (!energy[d] && sign[d] != 0) return fail(TAMM_ERR_ARG, "dimension %d has a sign but no energies", d);
  size_t need = 0;
  tamm_denominator_workspace_size(out, &need);
  if (!workspace || ((uintptr_t)workspace) % 256 || ws_bytes < need)
    return fail(TAMM_ERR_WORKSPACE, "denominator workspace must be 256-byte aligned and at least %zu bytes", need);
  if (out->block_off.empty()) return ok();
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  DenomParams dp{};
  for (int d = 0; d < out->rank; ++d) {
    dp.dim_tile_base[d] = out->dim_tile_base[d];
    dp.energy[d] = energy[d];
    dp.sign[d] = sign[d];
  }
  const size_t o1 = align256(out->block_off.size() * 8), o2 = o1 + align256(out->block_tiles.size() * 4),
               o3 = o2 + align256(out->tile_offset_cat.size() * 8);
  // the sources are host vectors owned by the tensor, alive as long as the tensor
  HIP_TRY(hipMemcpyAsync(ws, out->block_off.data(), out->block_off.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + o1, out->block_tiles.data(), out->block_tiles.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + o2, out->tile_offset_cat.data(), out->tile_offset_cat.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + o3, out->tile_size_cat.data(), out->tile_size_cat.size() * 8, hipMemcpyHostToDevice, s));
  dp.out = out->dev;
  dp.in = in->dev;
  dp.block_off = (const int64_t*)ws;
  dp.block_tiles = (const int32_t*)(ws + o1);
  dp.tile_offset = (const int64_t*)(ws + o2);
  dp.tile_size = (const int64_t*)(ws + o3);
  dp.rank = out->rank;
  dp.n_blocks = (int64_t)out->block_off.size();
  HIP_TRY(launch_denominator(dp, out->max_block, s));
  return ok();
}
