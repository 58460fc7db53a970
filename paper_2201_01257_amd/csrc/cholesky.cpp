// Host side of the C ABI, part 6: row views of block-sparse tensors (the view tensors of Sec. III-A)
// and the particle-particle ladder over integrals rebuilt from Cholesky vectors (Sec. IV-A-1,
// Eq. (cc12)).
//
// The ladder R[a,b,i,j] = beta R + alpha sum_cd V[a,b,c,d] T[c,d,i,j] with
// V[a,b,c,d] = sum_L B[a,c,L] B[b,d,L] - B[a,d,L] B[b,c,L] never forms V.  Renaming c <-> d in the
// second term gives
//     R[a,b,i,j] = beta R + alpha sum_cd G[a,c,b,d] Tm[c,d,i,j],
//     G[a,c,b,d] = sum_L B[a,c,L] B[b,d,L],      Tm[c,d,i,j] = T[c,d,i,j] - T[d,c,i,j],
// so the operation is one AddOp pair (Tm, quadratic in the orbital count) and, per strip of
// a-tiles, two block-sparse contractions on the matrix cores: the pair product G of the strip
// (a GEMM over the auxiliary index, rows (a,c), columns (b,d)) into a workspace buffer reused by
// every strip, and the ladder of the strip's rows of R against Tm.  G has the sparsity of B's
// pairs (spin-diagonal B: s_a = s_c and s_b = s_d), stricter than V's spin conservation, so the
// ladder half does fewer products than a ladder over stored V.  Memory: Tm plus one strip of G
// (the strip's share of a tensor of the fourth power of the virtual count) instead of all of V.
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "host.h"

using namespace tamm;

namespace {

// A tensor whose first dimension is restricted to tiles [lo, hi) of parent's, sharing parent's
// storage: parent's stored blocks with first tile in the range are contiguous (lexicographic
// order, first tile most significant), so the view's storage starts at the element offset *base
// of parent's storage and its blocks sit at parent's offsets minus *base.
std::unique_ptr<tamm_tensor> row_view(const tamm_tensor* P, int lo, int hi, int64_t* base) {
  auto v = std::make_unique<tamm_tensor>();
  auto sd = std::make_shared<SpaceData>();
  int64_t off = 0;
  for (int t = lo; t < hi; ++t) {
    sd->size.push_back(P->dims[0]->size[t]);
    sd->spin.push_back(P->dims[0]->spin[t]);
    sd->offset.push_back(off);
    off += P->dims[0]->size[t];
  }
  sd->extent = off;
  v->rank = P->rank;
  v->dims = P->dims;
  v->dims[0] = sd;
  v->tstride = P->tstride;
  const int64_t s0 = P->tstride[0];
  const size_t nb = P->block_off.size();
  int64_t b0 = -1, end = 0;
  for (size_t b = 0; b < nb; ++b) {
    const int t0 = P->block_tiles[b * P->rank];
    if (t0 < lo || t0 >= hi) continue;
    int64_t elems = 1;
    for (int d = 0; d < P->rank; ++d) elems *= P->dims[d]->size[P->block_tiles[b * P->rank + d]];
    if (b0 < 0) b0 = P->block_off[b];
    v->block_off.push_back(P->block_off[b] - b0);
    for (int d = 0; d < P->rank; ++d) v->block_tiles.push_back(P->block_tiles[b * P->rank + d] - (d == 0 ? lo : 0));
    v->max_block = std::max(v->max_block, elems);
    end = P->block_off[b] + elems;
  }
  if (b0 < 0) b0 = 0;
  v->tile_off.assign((size_t)((hi - lo) * s0), -1);
  for (int64_t lin = 0; lin < (hi - lo) * s0; ++lin) {
    const int64_t o = P->tile_off[(size_t)(lo * s0 + lin)];
    v->tile_off[(size_t)lin] = o < 0 ? -1 : o - b0;
  }
  v->numel = v->block_off.empty() ? 0 : end - b0;
  for (int d = 0; d < v->rank; ++d) {
    v->dim_tile_base.push_back((int32_t)v->tile_offset_cat.size());
    v->tile_offset_cat.insert(v->tile_offset_cat.end(), v->dims[d]->offset.begin(), v->dims[d]->offset.end());
    v->tile_size_cat.insert(v->tile_size_cat.end(), v->dims[d]->size.begin(), v->dims[d]->size.end());
  }
  *base = b0;
  return v;
}

// A tensor with t's spaces and block structure (no storage).
std::unique_ptr<tamm_tensor> clone_structure(const tamm_tensor* t) {
  auto c = std::make_unique<tamm_tensor>(*t);
  c->dev = nullptr;
  c->dev_bytes = 0;
  c->bound = false;
  return c;
}

bool stored(const tamm_tensor* t, int t0, int t1, int t2) {
  const int64_t lin = t0 * t->tstride[0] + t1 * t->tstride[1] + t2 * t->tstride[2];
  return t->tile_off[(size_t)lin] >= 0;
}

// Storage rule of the pair product G[a,c,b,d] of a strip: some auxiliary tile has both B[a,c,L]
// and B[b,d,L] stored.  The first tile index is relative to the strip.
struct PairRule {
  const tamm_tensor* b;
  int lo;
};

int pair_nonzero(const int32_t* t, const int8_t*, int32_t, void* user) {
  const PairRule* u = static_cast<const PairRule*>(user);
  const int nl = u->b->dims[2]->ntiles();
  for (int l = 0; l < nl; ++l)
    if (stored(u->b, u->lo + t[0], t[1], l) && stored(u->b, t[2], t[3], l)) return 1;
  return 0;
}

// Workspace slot of a plan: the largest workspace of any configuration with at most max_splits
// K splits (the autotuner tries only candidates that fit the slot it is given).  The plan is left
// in its default configuration.
int plan_slot(tamm_plan* p, int max_splits, size_t* bytes) {
  tamm_plan_stats st{};
  int rc = tamm_plan_stats_get(p, &st);
  if (rc != TAMM_OK) return rc;
  size_t mx = 0, n = 0;
  if ((rc = tamm_plan_workspace_size(p, &mx)) != TAMM_OK) return rc;
  int32_t nc = 0;
  tamm_plan_config_count(p, &nc);
  for (int c = 0; c < nc; ++c)
    for (int ks = 1; ks <= max_splits; ks *= 2) {
      if (tamm_plan_set_config(p, c, ks) != TAMM_OK) continue;
      tamm_plan_workspace_size(p, &n);
      mx = std::max(mx, n);
    }
  if ((rc = tamm_plan_set_config(p, st.kernel_config, st.k_splits)) != TAMM_OK) return rc;
  *bytes = align256(mx);
  return TAMM_OK;
}

}  // namespace

extern "C" int tamm_tensor_view_rows(const tamm_tensor* parent, int32_t tile_lo, int32_t tile_hi, tamm_tensor** out,
                                     int64_t* elem_offset) {
  if (!out) return fail(TAMM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!parent || !elem_offset) return fail(TAMM_ERR_ARG, "null argument");
  if (tile_lo < 0 || tile_hi <= tile_lo || tile_hi > parent->dims[0]->ntiles())
    return fail(TAMM_ERR_ARG, "tile range [%d, %d) is not inside the %d tiles of the first dimension", tile_lo, tile_hi,
                parent->dims[0]->ntiles());
  int64_t base = 0;
  *out = row_view(parent, tile_lo, tile_hi, &base).release();
  *elem_offset = base;
  return ok();
}

struct CholStrip {
  int lo = 0, hi = 0;
  std::unique_ptr<tamm_tensor> bv, rv, g;
  int64_t b_base = 0, r_base = 0;
  PairRule rule{};
  tamm_plan* build = nullptr;
  tamm_plan* ladder = nullptr;
  size_t off_build = 0, off_ladder = 0, sz_build = 0, sz_ladder = 0;
};

struct tamm_chol {
  tamm_tensor* r = nullptr;
  const tamm_tensor* t = nullptr;
  const tamm_tensor* b = nullptr;
  std::unique_ptr<tamm_tensor> tm;
  tamm_add* copy = nullptr;
  tamm_add* swap = nullptr;
  std::vector<std::unique_ptr<CholStrip>> strips;
  size_t off_tm = 0, off_g = 0, off_copy = 0, off_swap = 0, ws_size = 0;
  int64_t g_max = 0;
  char* ws = nullptr;
  bool bound = false;
  ~tamm_chol() {
    for (auto& s : strips) {
      if (s->build) tamm_plan_destroy(s->build);
      if (s->ladder) tamm_plan_destroy(s->ladder);
    }
    if (copy) tamm_add_destroy(copy);
    if (swap) tamm_add_destroy(swap);
  }
};

extern "C" int tamm_chol_ladder_create(tamm_tensor* r, const tamm_tensor* t, const tamm_tensor* b, int32_t strip_tiles,
                                       tamm_chol** out) {
  if (!out) return fail(TAMM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!r || !t || !b) return fail(TAMM_ERR_ARG, "null tensor");
  if (r->rank != 4 || t->rank != 4 || b->rank != 3) return fail(TAMM_ERR_SHAPE, "R and T must be rank 4 and B rank 3");
  const auto& v = r->dims[0];
  if (!r->dims[1]->same(*v) || !t->dims[0]->same(*v) || !t->dims[1]->same(*v) || !b->dims[0]->same(*v) ||
      !b->dims[1]->same(*v))
    return fail(TAMM_ERR_LABEL, "R[a,b,.,.], T[c,d,.,.] and B[p,q,.] must share one virtual space");
  if (!r->dims[2]->same(*t->dims[2]) || !r->dims[3]->same(*t->dims[3]))
    return fail(TAMM_ERR_LABEL, "R[.,.,i,j] and T[.,.,i,j] must share the occupied spaces");
  if (strip_tiles < 0) return fail(TAMM_ERR_ARG, "strip_tiles must be >= 0");
  const int nv = v->ntiles();
  const int per = strip_tiles == 0 ? 1 : std::min<int>(strip_tiles, nv);
  auto c = std::make_unique<tamm_chol>();
  c->r = r;
  c->t = t;
  c->b = b;
  c->tm = clone_structure(t);
  int rc = tamm_add_create(c->tm.get(), "cdij", t, "cdij", &c->copy);
  if (rc != TAMM_OK) return rc;
  rc = tamm_add_create(c->tm.get(), "cdij", t, "dcij", &c->swap);
  if (rc != TAMM_OK) return rc;
  for (int lo = 0; lo < nv; lo += per) {
    auto s = std::make_unique<CholStrip>();
    s->lo = lo;
    s->hi = std::min(nv, lo + per);
    s->bv = row_view(b, s->lo, s->hi, &s->b_base);
    s->rv = row_view(r, s->lo, s->hi, &s->r_base);
    s->rule = PairRule{b, s->lo};
    // G over (a in the strip, c, b, d): spaces of the strip view and of B's orbital dimension
    tamm_space sa{s->bv->dims[0]}, sv{v};
    tamm_space* gd[4] = {&sa, &sv, &sv, &sv};
    tamm_tensor* g = nullptr;
    rc = tamm_tensor_create(gd, 4, pair_nonzero, &s->rule, &g);
    if (rc != TAMM_OK) return rc;
    s->g.reset(g);
    c->g_max = std::max(c->g_max, s->g->numel);
    // (a strip whose G has no stored block still runs its ladder plan: its R rows become beta R)
    rc = tamm_plan_create(s->g.get(), "acbd", s->bv.get(), "acL", b, "bdL", TAMM_PREC_F64, &s->build);
    if (rc != TAMM_OK) return rc;
    rc = tamm_plan_create(s->rv.get(), "abij", s->g.get(), "acbd", c->tm.get(), "cdij", TAMM_PREC_F64, &s->ladder);
    if (rc != TAMM_OK) return rc;
    c->strips.push_back(std::move(s));
  }
  // workspace: Tm | G (largest strip) | AddOp tables | per strip: build and ladder plans, each
  // slot large enough for any configuration the autotuner may choose
  size_t off = 0;
  c->off_tm = off;
  off = align256(off + (size_t)c->tm->numel * 8);
  c->off_g = off;
  off = align256(off + (size_t)c->g_max * 8);
  size_t a = 0;
  tamm_add_workspace_size(c->copy, &a);
  c->off_copy = off;
  off = align256(off + a);
  tamm_add_workspace_size(c->swap, &a);
  c->off_swap = off;
  off = align256(off + a);
  for (auto& s : c->strips) {
    // the pair product has thousands of output tiles per strip: no K splits (their partial tiles
    // would take several times the strip of G); the strip ladders may split
    if ((rc = plan_slot(s->build, 1, &s->sz_build)) != TAMM_OK) return rc;
    if ((rc = plan_slot(s->ladder, 8, &s->sz_ladder)) != TAMM_OK) return rc;
    s->off_build = off;
    off += s->sz_build;
    s->off_ladder = off;
    off += s->sz_ladder;
  }
  c->ws_size = std::max<size_t>(off, 256);
  *out = c.release();
  return ok();
}

extern "C" int tamm_chol_ladder_workspace_size(const tamm_chol* c, size_t* bytes) {
  if (!c || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = c->ws_size;
  return ok();
}

extern "C" int tamm_chol_ladder_bind_workspace(tamm_chol* c, void* workspace, size_t bytes) {
  if (!c) return fail(TAMM_ERR_ARG, "null argument");
  if (!workspace || ((uintptr_t)workspace) % 256 || bytes < c->ws_size)
    return fail(TAMM_ERR_WORKSPACE, "workspace must be 256-byte aligned and at least %zu bytes", c->ws_size);
  char* ws = (char*)workspace;
  int rc = tamm_tensor_bind(c->tm.get(), ws + c->off_tm, (size_t)c->tm->numel * 8);
  if (rc != TAMM_OK) return rc;
  if ((rc = tamm_add_bind_workspace(c->copy, ws + c->off_copy, c->ws_size - c->off_copy)) != TAMM_OK) return rc;
  if ((rc = tamm_add_bind_workspace(c->swap, ws + c->off_swap, c->ws_size - c->off_swap)) != TAMM_OK) return rc;
  for (auto& s : c->strips) {
    if ((rc = tamm_tensor_bind(s->g.get(), ws + c->off_g, (size_t)s->g->numel * 8)) != TAMM_OK) return rc;
    if ((rc = tamm_plan_bind_workspace(s->build, ws + s->off_build, s->sz_build)) != TAMM_OK) return rc;
    if ((rc = tamm_plan_bind_workspace(s->ladder, ws + s->off_ladder, s->sz_ladder)) != TAMM_OK) return rc;
  }
  c->ws = ws;
  c->bound = true;
  return ok();
}

// Point the views at the current storage of R and B.
static int refresh_views(tamm_chol* c) {
  if (!c->bound) return fail(TAMM_ERR_UNBOUND, "workspace is not bound");
  if (!c->r->bound || !c->t->bound || !c->b->bound) return fail(TAMM_ERR_UNBOUND, "R, T and B need bound storage");
  for (auto& s : c->strips) {
    int rc = tamm_tensor_bind(s->bv.get(), c->b->dev + s->b_base, (size_t)s->bv->numel * 8);
    if (rc != TAMM_OK) return rc;
    if ((rc = tamm_tensor_bind(s->rv.get(), c->r->dev + s->r_base, (size_t)s->rv->numel * 8)) != TAMM_OK) return rc;
  }
  return TAMM_OK;
}

static int chol_enqueue(tamm_chol* c, double alpha, double beta, hipStream_t s) {
  int rc = add_enqueue(c->copy, 1.0, 0.0, s);
  if (rc != TAMM_OK) return rc;
  if ((rc = add_enqueue(c->swap, -1.0, 1.0, s)) != TAMM_OK) return rc;
  for (auto& st : c->strips) {
    if ((rc = tamm_plan_execute(st->build, 1.0, 0.0, s)) != TAMM_OK) return rc;
    if ((rc = tamm_plan_execute(st->ladder, alpha, beta, s)) != TAMM_OK) return rc;
  }
  return TAMM_OK;
}

extern "C" int tamm_chol_ladder_execute(tamm_chol* c, double alpha, double beta, void* stream) {
  if (!c) return fail(TAMM_ERR_ARG, "null argument");
  int rc = refresh_views(c);
  if (rc != TAMM_OK) return rc;
  rc = chol_enqueue(c, alpha, beta, (hipStream_t)stream);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_chol_ladder_autotune(tamm_chol* c, void* stream, const char* cache_path, int32_t reps) {
  if (!c) return fail(TAMM_ERR_ARG, "null argument");
  int rc = refresh_views(c);
  if (rc != TAMM_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  // Tm valid and G zero, so that trial runs (alpha = 0, beta = 1) leave G and R unchanged
  if ((rc = add_enqueue(c->copy, 1.0, 0.0, s)) != TAMM_OK) return rc;
  if ((rc = add_enqueue(c->swap, -1.0, 1.0, s)) != TAMM_OK) return rc;
  HIP_TRY(launch_fill((double*)(c->ws + c->off_g), c->g_max, 0.0, s));
  for (auto& st : c->strips) {
    if ((rc = tamm_plan_autotune(st->build, c->ws + st->off_build, st->sz_build, stream, cache_path, reps)) != TAMM_OK)
      return rc;
    if ((rc = tamm_plan_autotune(st->ladder, c->ws + st->off_ladder, st->sz_ladder, stream, cache_path, reps)) != TAMM_OK)
      return rc;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return ok();
}

extern "C" int tamm_chol_ladder_stats(const tamm_chol* c, double* build_flops, double* ladder_flops, int64_t* strips,
                                      int64_t* g_max_elements, int64_t* tm_elements) {
  if (!c) return fail(TAMM_ERR_ARG, "null argument");
  double bf = 0, lf = 0;
  for (auto& s : c->strips) {
    tamm_plan_stats a{}, b{};
    tamm_plan_stats_get(s->build, &a);
    tamm_plan_stats_get(s->ladder, &b);
    bf += a.useful_flops;
    lf += b.useful_flops;
  }
  if (build_flops) *build_flops = bf;
  if (ladder_flops) *ladder_flops = lf;
  if (strips) *strips = (int64_t)c->strips.size();
  if (g_max_elements) *g_max_elements = c->g_max;
  if (tm_elements) *tm_elements = c->tm->numel;
  return ok();
}

extern "C" int tamm_chol_ladder_strip_plans(const tamm_chol* c, int32_t strip, tamm_plan** build, tamm_plan** ladder) {
  if (!c || strip < 0 || strip >= (int32_t)c->strips.size()) return fail(TAMM_ERR_ARG, "no such strip");
  if (build) *build = c->strips[strip]->build;
  if (ladder) *ladder = c->strips[strip]->ladder;
  return ok();
}

extern "C" int tamm_chol_ladder_destroy(tamm_chol* c) {
  delete c;
  return ok();
}
