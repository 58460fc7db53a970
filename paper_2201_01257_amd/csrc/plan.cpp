// Host side of the C ABI, part 2: contraction plans (label analysis, offset tables, screening
// setup, work decomposition), grouped persistent execution with hipGraph replay, and the
// autotuner that picks kernel configurations by measurement.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "host.h"
#include "mixed.h"

using namespace tamm;

namespace {

struct Label {
  char c;
  int od = -1, ad = -1, bd = -1;  // dimension in out, A, B (-1 if absent)
  std::shared_ptr<SpaceData> sp;
  std::vector<int32_t> cls;       // size class per tile
  std::vector<int64_t> cls_size;  // tile size of each class
};

int32_t pool_push(std::vector<int32_t>& pool, const std::vector<int64_t>& v) {
  int32_t start = (int32_t)pool.size();
  for (int64_t x : v) pool.push_back((int32_t)x);
  return start;
}

// An offset table followed by its padding of invalid entries (read by the gathers past the end).
static int32_t pool_push_table(std::vector<int32_t>& pool, const std::vector<int64_t>& v) {
  const int32_t start = pool_push(pool, v);
  pool.insert(pool.end(), kTablePad, kTableInvalid);
  return start;
}

// True when entries 2j and 2j+1 of a table are adjacent elements for every j (even length).
static bool pairs_adjacent(const std::vector<int64_t>& t) {
  if (t.size() % 2) return false;
  for (size_t j = 0; j + 1 < t.size(); j += 2)
    if (t[j + 1] != t[j] + 1) return false;
  return true;
}

// Offset table of one label group inside blocks of one operand shape: flattened index (mixed
// radix over `group`, last fastest) -> element offset in the row-major block.
std::vector<int64_t> group_table(const std::vector<int>& group, const std::vector<int64_t>& lab_ext,
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

uint64_t fnv(uint64_t h, const void* data, size_t n) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001B3ULL;
  }
  return h;
}

// Device regions of one contraction's static tables and screened pair lists, relative to a base.
struct Layout {
  size_t pool = 0, atile = 0, btile = 0, blocks = 0, pairs = 0, counts = 0, end = 0;
};

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
  std::vector<int> M, N, K;        // label indices in flattening order (last fastest)
  std::vector<int> k_lhs_order;    // for each K label in lhs order: its position in K
  bool a_kc = true, b_kc = true;
  bool pairs = false;              // every gathered pair of table entries is adjacent (16-byte loads)
  bool planes = false;             // split-bfloat16 operands in the planes layout
  std::vector<int32_t> pool;
  ScreenDesc sd{};                 // device pointers filled when bound
  int64_t n_kt = 1;
  std::vector<OutBlockDesc> blocks;
  std::vector<double> block_cost;  // sum of K extents of the surviving pairs of each block
  uint64_t signature = 0;
  // split-bfloat16 precisions: per stored operand block, the split work description
  std::vector<PrepBlock> prepA, prepB;
  int64_t prepA_items = 0, prepB_items = 0;
  // operands the caller declared constant (tamm_plan_set_constant): their split is reused while
  // it is valid -- taken from the same storage into the current workspace
  bool const_A = false, const_B = false;
  const void* split_src_A = nullptr;  // storage the split of A in the workspace was taken from
  const void* split_src_B = nullptr;
  // kernel configuration and work decomposition
  int config = -1;
  int k_splits = 1;
  int xcd_chunk = -1;              // work items per die chunk (xcd_order); -1: the library default
  int tile_order = 0;              // 0: tiles of a block row by row; 1: grouped by B column panel
  std::vector<WorkItem> work;
  std::vector<ReduceItem> reduce;
  tamm_plan_stats stats{};
  // workspace: static layout, then work list, reduce list, partial tiles
  Layout lay;
  size_t off_work = 0, off_reduce = 0, off_partial = 0, off_prepA = 0, off_prepB = 0, off_xA = 0, off_xB = 0, ws_size = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_bound = false;
  bool screened = false;
  bool executed = false;
};

static int configure_work(tamm_plan* p, int config, int k_splits);

// Gather layout index of a plan's kernels: bit 1 = A k-contiguous, bit 0 = B k-contiguous,
// bit 2 = 16-byte (two-element) gathers.
static int gather_layout(const tamm_plan* p) {
  return 2 * (p->a_kc ? 1 : 0) + (p->b_kc ? 1 : 0) + (p->pairs ? 4 : 0) + (p->planes ? 8 : 0);
}
constexpr int kLayouts = 8;

static Layout make_layout(const tamm_plan* p, size_t base) {
  Layout L;
  size_t off = align256(base);
  L.pool = off;
  off = align256(off + p->pool.size() * sizeof(int32_t));
  L.atile = off;
  off = align256(off + p->A->tile_off.size() * sizeof(int64_t));
  L.btile = off;
  off = align256(off + p->B->tile_off.size() * sizeof(int64_t));
  L.blocks = off;
  off = align256(off + p->blocks.size() * sizeof(OutBlockDesc));
  L.pairs = off;
  off = align256(off + p->blocks.size() * (size_t)p->n_kt * sizeof(PairDesc));
  L.counts = off;
  off = align256(off + p->blocks.size() * sizeof(int32_t));
  L.end = off;
  return L;
}

static int upload_static(const tamm_plan* p, char* ws, const Layout& L) {
  HIP_TRY(hipMemcpy(ws + L.pool, p->pool.data(), p->pool.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws + L.atile, p->A->tile_off.data(), p->A->tile_off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws + L.btile, p->B->tile_off.data(), p->B->tile_off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  if (!p->blocks.empty())
    HIP_TRY(hipMemcpy(ws + L.blocks, p->blocks.data(), p->blocks.size() * sizeof(OutBlockDesc), hipMemcpyHostToDevice));
  return TAMM_OK;
}

static ScreenDesc screen_desc(const tamm_plan* p, char* ws, const Layout& L) {
  ScreenDesc s = p->sd;
  s.a_tile_off = (const int64_t*)(ws + L.atile);
  s.b_tile_off = (const int64_t*)(ws + L.btile);
  s.blocks = (const OutBlockDesc*)(ws + L.blocks);
  s.pairs = (PairDesc*)(ws + L.pairs);
  s.counts = (int32_t*)(ws + L.counts);
  s.pool = (const int32_t*)(ws + L.pool);
  s.a_base = 0;
  s.b_base = 0;
  s.pool_base = 0;
  s.pair_stride = (int32_t)p->n_kt;
  s.next_seg = -1;
  s.n_blocks = (int32_t)p->blocks.size();
  return s;
}

static ProblemDesc problem_desc(const tamm_plan* p, char* ws, const Layout& L, double* partial, int k_splits, double alpha,
                                double beta) {
  ProblemDesc d{};
  d.A = p->A->dev;
  d.B = p->B->dev;
  d.C = p->out->dev;
  d.blocks = (const OutBlockDesc*)(ws + L.blocks);
  d.pairs = (const PairDesc*)(ws + L.pairs);
  d.counts = (const int32_t*)(ws + L.counts);
  d.pool = (const int32_t*)(ws + L.pool);
  d.partial = partial;
  d.alpha = alpha;
  d.beta = beta;
  d.k_splits = k_splits;
  d.a_kc = p->a_kc ? 1 : 0;
  d.b_kc = p->b_kc ? 1 : 0;
  return d;
}

extern "C" int tamm_plan_create(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                                const tamm_tensor* rhs, const char* rhs_lbl, tamm_precision precision, tamm_plan** plan) {
  if (!plan) return fail(TAMM_ERR_ARG, "null output pointer");
  *plan = nullptr;
  if (!out || !lhs || !rhs || !out_lbl || !lhs_lbl || !rhs_lbl) return fail(TAMM_ERR_ARG, "null tensor or label string");
  if (precision != TAMM_PREC_F64 && precision != TAMM_PREC_F32 && precision != TAMM_PREC_BF16X3 &&
      precision != TAMM_PREC_BF16X4_ALIGNED)
    return fail(TAMM_ERR_ARG, "unknown precision %d", (int)precision);
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

  // ---- offset tables per operand shape class ------------------------------------------------
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
  auto build_tables = [&](const OpInfo& o, const std::vector<int>& g1, const std::vector<int>& g2,
                          std::vector<int64_t>& start1, std::vector<int64_t>& start2, bool& pairs1, bool& pairs2) {
    start1.assign(o.ncls, 0);
    start2.assign(o.ncls, 0);
    pairs1 = pairs2 = true;
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
      const std::vector<int64_t> t1 = group_table(g1, lab_ext, lab_stride), t2 = group_table(g2, lab_ext, lab_stride);
      pairs1 = pairs1 && pairs_adjacent(t1);
      pairs2 = pairs2 && pairs_adjacent(t2);
      start1[c] = pool_push_table(pool, t1);
      start2[c] = pool_push_table(pool, t2);
      if (pool.size() > (size_t)INT32_MAX / 2) return false;
    }
    return true;
  };
  if (p->A->max_block >= kTableInvalid || p->B->max_block >= kTableInvalid)
    return fail(TAMM_ERR_UNSUPPORTED, "operand blocks of 2^27 or more elements are not supported");
  std::vector<int64_t> aM, aK, bK, bN, oM, oN;
  bool aM_pairs, aK_pairs, bK_pairs, bN_pairs, oM_pairs, oN_pairs;
  if (!build_tables(ai, p->M, p->K, aM, aK, aM_pairs, aK_pairs) || !build_tables(bi, p->K, p->N, bK, bN, bK_pairs, bN_pairs) ||
      !build_tables(oi, p->M, p->N, oM, oN, oM_pairs, oN_pairs))
    return fail(TAMM_ERR_UNSUPPORTED, "a block has more than 2^31 elements or the offset tables are too large");
  // 16-byte gathers pair consecutive k of a k-contiguous operand, consecutive rows otherwise
  p->pairs = (p->a_kc ? aK_pairs : aM_pairs) && (p->b_kc ? bK_pairs : bN_pairs);
  if (precision == TAMM_PREC_BF16X3 || precision == TAMM_PREC_BF16X4_ALIGNED) {
    // split work per stored operand block: rows (M for A, N for B) x K windows
    auto prep_list = [&](const OpInfo& o, const std::vector<int64_t>& rowtab, const std::vector<int64_t>& ktab,
                         const std::vector<int>& rowgroup, bool kc, std::vector<PrepBlock>& list, int64_t& items) {
      const tamm_tensor* t = o.t;
      items = 0;
      for (size_t b = 0; b < t->block_off.size(); ++b) {
        const int32_t* tt = &t->block_tiles[b * t->rank];
        int64_t cls = 0, rows = 1, kext = 1;
        for (int d = 0; d < t->rank; ++d) {
          const Label& L = p->labels[o.dim_label[d]];
          cls += L.cls[tt[d]] * o.cstride[d];
          const bool is_row = std::find(rowgroup.begin(), rowgroup.end(), o.dim_label[d]) != rowgroup.end();
          (is_row ? rows : kext) *= L.sp->size[tt[d]];
        }
        PrepBlock pb{};
        pb.off = t->block_off[b];
        pb.item0 = items;
        pb.rows = (int32_t)rows;
        pb.kext = (int32_t)kext;
        pb.tab_row = (int32_t)rowtab[cls];
        pb.tab_k = (int32_t)ktab[cls];
        pb.nwin = (int32_t)((kext + kSplitWindow - 1) / kSplitWindow);
        items += (kc ? rows : (rows + 63) / 64) * pb.nwin;
        list.push_back(pb);
      }
    };
    prep_list(ai, aM, aK, p->M, p->a_kc, p->prepA, p->prepA_items);
    prep_list(bi, bN, bK, p->N, p->b_kc, p->prepB, p->prepB_items);
    // planes layout (16-byte gathers of 8 consecutive k) when every block's K extent is a
    // multiple of 8; otherwise the packed layout at the float64 offsets
    p->planes = true;
    for (const auto* list : {&p->prepA, &p->prepB})
      for (const PrepBlock& pb : *list) p->planes = p->planes && pb.kext % 8 == 0;
  }
  ScreenDesc& sd = p->sd;
  memset(&sd, 0, sizeof(sd));
  sd.a_cls_tabM = pool_push(pool, aM);
  sd.a_cls_tabK = pool_push(pool, aK);
  sd.b_cls_tabK = pool_push(pool, bK);
  sd.b_cls_tabN = pool_push(pool, bN);
  sd.nk = (int)p->K.size();
  p->n_kt = 1;
  for (int q = 0; q < sd.nk; ++q) {
    const Label& L = p->labels[p->K[q]];
    sd.k_ntiles[q] = L.sp->ntiles();
    p->n_kt *= L.sp->ntiles();
    sd.a_tstride[q] = (int32_t)p->A->tstride[L.ad];
    sd.b_tstride[q] = (int32_t)p->B->tstride[L.bd];
    sd.a_cstride[q] = (int32_t)ai.cstride[L.ad];
    sd.b_cstride[q] = (int32_t)bi.cstride[L.bd];
    sd.k_size_tab[q] = pool_push(pool, L.sp->size);
    std::vector<int64_t> cls(L.cls.begin(), L.cls.end());
    sd.k_cls_tab[q] = pool_push(pool, cls);
  }
  if (p->n_kt > (1 << 20)) return fail(TAMM_ERR_UNSUPPORTED, "too many contracted tile tuples");
  sd.n_kt = (int32_t)p->n_kt;

  // ---- output blocks and host structural screening statistics ------------------------------
  const int64_t nob = (int64_t)out->block_off.size();
  if (nob * p->n_kt > (int64_t)1 << 28) return fail(TAMM_ERR_UNSUPPORTED, "pair capacity too large");
  p->blocks.resize(nob);
  p->block_cost.assign(nob, 0.0);
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
    // host count of surviving pairs (statistics and scheduling cost; the kernels use the pair
    // list produced by the GPU screen)
    for (int64_t kt = 0; kt < p->n_kt; ++kt) {
      int64_t rem = kt, alin = atb, blin = btb, kext = 1;
      for (int q = sd.nk - 1; q >= 0; --q) {
        const int t = (int)(rem % sd.k_ntiles[q]);
        rem /= sd.k_ntiles[q];
        alin += (int64_t)t * sd.a_tstride[q];
        blin += (int64_t)t * sd.b_tstride[q];
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
        for (int q = sd.nk - 1; q >= 0; --q) {
          const int t = (int)(r2 % sd.k_ntiles[q]);
          r2 /= sd.k_ntiles[q];
          alin += (int64_t)t * sd.a_tstride[q];
          blin += (int64_t)t * sd.b_tstride[q];
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
  // structural signature (autotuner cache key)
  uint64_t h = 0xCBF29CE484222325ULL;
  const int32_t hdr[6] = {(int32_t)p->M.size(), (int32_t)p->N.size(), (int32_t)p->K.size(), (int32_t)p->a_kc,
                          (int32_t)p->b_kc, (int32_t)precision};
  h = fnv(h, hdr, sizeof(hdr));
  for (int l : p->M) h = fnv(h, p->labels[l].sp->size.data(), p->labels[l].sp->size.size() * 8);
  for (int l : p->N) h = fnv(h, p->labels[l].sp->size.data(), p->labels[l].sp->size.size() * 8);
  for (int l : p->K) h = fnv(h, p->labels[l].sp->size.data(), p->labels[l].sp->size.size() * 8);
  h = fnv(h, &tasks, sizeof(tasks));
  h = fnv(h, &nob, sizeof(nob));
  h = fnv(h, p->block_cost.data(), p->block_cost.size() * sizeof(double));
  p->signature = h;
  int rc = configure_work(p.get(), -1, 0);
  if (rc != TAMM_OK) return rc;
  *plan = p.release();
  return ok();
}

// Kernel configuration tables by precision.
struct TileCfg {
  int mt, nt, kt, threads;
  const char* name;
};

static int cfg_count(int prec) { return prec == TAMM_PREC_F64 ? f64_config_count() : mixed_config_count(prec); }

static TileCfg cfg_get(int prec, int c) {
  if (prec == TAMM_PREC_F64) {
    const F64Config& f = f64_config(c);
    return TileCfg{f.mt, f.nt, f.kt, 64 * f.wgm * f.wgn, f.name};
  }
  const MixedConfig& f = mixed_config(prec, c);
  return TileCfg{f.mt, f.nt, f.kt, 64 * f.wgm * f.wgn, f.name};
}

// Number of output tiles and padding factor of one configuration.
static std::pair<int64_t, double> tiles_for(const tamm_plan* p, int c) {
  const TileCfg f = cfg_get(p->prec, c);
  int64_t n = 0;
  double area = 0, useful = 0;
  for (const auto& b : p->blocks) {
    const int64_t tm = (b.mext + f.mt - 1) / f.mt, tn = (b.next + f.nt - 1) / f.nt;
    n += tm * tn;
    area += (double)tm * f.mt * tn * f.nt;
    useful += (double)b.mext * b.next;
  }
  return std::make_pair(n, useful > 0 ? area / useful : 1.0);
}

// Default configuration when the autotuner has not run: the largest tile that gives every compute
// unit two tiles with little padding.
static int default_config(const tamm_plan* p) {
  int best = 0;
  double best_score = -1;
  for (int c = 0; c < cfg_count(p->prec); ++c) {
    auto tw = tiles_for(p, c);
    const TileCfg f = cfg_get(p->prec, c);
    if ((p->prec == TAMM_PREC_F64 && f.kt != 16) || f.threads != 256 || f.mt > 128 || f.nt > 128) continue;
    double score = (double)f.mt * f.nt / tw.second;
    if (tw.first < 512) score *= (double)tw.first / 512.0;
    if (score > best_score) {
      best_score = score;
      best = c;
    }
  }
  return best;
}

// Launch order of the work items for the chip's eight accelerator dies (XCDs), each with its own
// L2: the dispatcher hands workgroup b to die b % 8.  The longest-first list is cut into chunks of
// `chunk` consecutive items (neighbouring tiles of one output block, which share operand panels)
// and chunk c goes to die c % 8, so every die works through whole chunks in longest-first order
// and tiles that read the same rows of A or columns of B run together behind one L2.  Slots left
// empty by dies with fewer items are squeezed out, which only moves a few tail items to another
// die.  A chunk of 0 or 1 keeps the list as it is.
static void xcd_order(std::vector<WorkItem>& work, int chunk) {
  constexpr int kDies = 8;
  const size_t n = work.size();
  if (chunk <= 1 || n <= (size_t)kDies) return;
  const size_t nchunks = (n + chunk - 1) / chunk;
  std::vector<size_t> len(kDies, 0);
  for (size_t c = 0; c < nchunks; ++c) len[c % kDies] += std::min<size_t>(chunk, n - c * chunk);
  const size_t rows = *std::max_element(len.begin(), len.end());
  std::vector<int64_t> slot(rows * kDies, -1);
  for (int x = 0; x < kDies; ++x)
    for (size_t i = 0; i < len[x]; ++i) {
      const size_t c = (size_t)x + kDies * (i / chunk);  // the die's (i / chunk)-th chunk
      slot[i * kDies + x] = (int64_t)(c * chunk + i % chunk);
    }
  std::vector<WorkItem> out;
  out.reserve(n);
  for (int64_t l : slot)
    if (l >= 0) out.push_back(work[(size_t)l]);
  work.swap(out);
}

static int xcd_chunk() {
  static const int v = [] {
    const char* e = getenv("TAMM_XCD_CHUNK");
    return e ? std::max(0, atoi(e)) : 32;
  }();
  return v;
}

// Work decomposition for one kernel configuration: macro-tiles of every stored output block,
// heaviest first (longest-processing-time order), with the K splits of a tile adjacent, then laid
// out for the dies (xcd_order).
static int configure_work(tamm_plan* p, int config, int k_splits) {
  const int ncfg = cfg_count(p->prec);
  const int64_t nob = (int64_t)p->blocks.size();
  if (config < 0) config = default_config(p);
  if (config >= ncfg) return fail(TAMM_ERR_ARG, "kernel configuration %d does not exist (%d available)", config, ncfg);
  const TileCfg f = cfg_get(p->prec, config);
  const int64_t ntiles = tiles_for(p, config).first;
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
  // K splits per tile in proportion to its block's summed K extent: tiles of the heaviest blocks
  // get k_splits parts, lighter ones fewer (at least one), so that the parts cost about the same
  double max_cost = 0;
  for (const Tile& t : tiles) max_cost = std::max(max_cost, p->block_cost[t.ob]);
  struct Part {
    double cost;
    WorkItem w;
  };
  std::vector<Part> parts;
  p->reduce.clear();
  int64_t slots = 0;
  for (const Tile& t : tiles) {
    int ns = 1;
    if (k_splits > 1 && max_cost > 0)
      ns = (int)std::min<double>(k_splits, std::max(1.0, std::floor(k_splits * p->block_cost[t.ob] / max_cost + 0.5)));
    for (int s = 0; s < ns; ++s)
      parts.push_back(Part{t.cost / ns, WorkItem{0, t.ob, t.m0, t.n0, encode_split(s, ns), (int32_t)slots}});
    if (ns > 1) {
      p->reduce.push_back(ReduceItem{0, t.ob, t.m0, t.n0, (int32_t)slots, ns});
      slots += ns;
    }
    if (slots > INT32_MAX / 2) return fail(TAMM_ERR_UNSUPPORTED, "too many partial tiles");
  }
  // longest processing time first; the parts of a tile stay adjacent when their costs tie.  Order
  // 0 keeps the tiles of one block row by row (neighbours share A row panels); order 1 puts the
  // tiles that read the same B column panel -- the same N tiles of their blocks, the same first
  // column -- next to each other across the blocks and rows (for operations whose B panels are the
  // large ones, such as a few output rows against long columns)
  const std::vector<OutBlockDesc>& bd = p->blocks;
  if (p->tile_order == 1)
    std::stable_sort(parts.begin(), parts.end(), [&bd](const Part& x, const Part& y) {
      if (x.cost != y.cost) return x.cost > y.cost;
      const int32_t bx = bd[x.w.ob].b_tbase, by = bd[y.w.ob].b_tbase;
      if (bx != by) return bx < by;
      if (x.w.n0 != y.w.n0) return x.w.n0 < y.w.n0;
      if (x.w.ob != y.w.ob) return x.w.ob < y.w.ob;
      return x.w.m0 < y.w.m0;
    });
  else
    std::stable_sort(parts.begin(), parts.end(), [](const Part& x, const Part& y) { return x.cost > y.cost; });
  p->work.clear();
  for (const Part& q : parts) p->work.push_back(q.w);
  if (p->work.size() > (size_t)INT32_MAX / 2) return fail(TAMM_ERR_UNSUPPORTED, "too many work items");
  xcd_order(p->work, p->xcd_chunk >= 0 ? p->xcd_chunk : xcd_chunk());
  p->config = config;
  p->k_splits = k_splits;
  p->stats.work_items = (int64_t)p->work.size();
  p->stats.kernel_config = config;
  p->stats.k_splits = k_splits;
  p->stats.xcd_chunk = p->xcd_chunk >= 0 ? p->xcd_chunk : xcd_chunk();
  p->stats.tile_order = p->tile_order;
  p->stats.gather_layout = gather_layout(p);
  p->lay = make_layout(p, 0);
  size_t off = p->lay.end;
  p->off_work = off;
  off = align256(off + p->work.size() * sizeof(WorkItem));
  p->off_reduce = off;
  off = align256(off + p->reduce.size() * sizeof(ReduceItem));
  p->off_partial = off;
  if (slots > 0) off = align256(off + (size_t)slots * f.mt * f.nt * sizeof(double));
  if (p->prec == TAMM_PREC_BF16X3 || p->prec == TAMM_PREC_BF16X4_ALIGNED) {
    p->off_prepA = off;
    off = align256(off + p->prepA.size() * sizeof(PrepBlock));
    p->off_prepB = off;
    off = align256(off + p->prepB.size() * sizeof(PrepBlock));
    p->off_xA = off;
    off = align256(off + (size_t)p->A->numel * sizeof(uint64_t));
    p->off_xB = off;
    off = align256(off + (size_t)p->B->numel * sizeof(uint64_t));
  }
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

static int bind_plan(tamm_plan* p, void* dev_ptr, size_t bytes) {
  if (!dev_ptr || ((uintptr_t)dev_ptr) % 256) return fail(TAMM_ERR_WORKSPACE, "workspace must be non-null and 256-byte aligned");
  if (bytes < p->ws_size) return fail(TAMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, p->ws_size);
  char* ws = (char*)dev_ptr;
  int rc = upload_static(p, ws, p->lay);
  if (rc != TAMM_OK) return rc;
  if (!p->work.empty()) HIP_TRY(hipMemcpy(ws + p->off_work, p->work.data(), p->work.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  if (!p->reduce.empty())
    HIP_TRY(hipMemcpy(ws + p->off_reduce, p->reduce.data(), p->reduce.size() * sizeof(ReduceItem), hipMemcpyHostToDevice));
  if (!p->prepA.empty()) HIP_TRY(hipMemcpy(ws + p->off_prepA, p->prepA.data(), p->prepA.size() * sizeof(PrepBlock), hipMemcpyHostToDevice));
  if (!p->prepB.empty()) HIP_TRY(hipMemcpy(ws + p->off_prepB, p->prepB.data(), p->prepB.size() * sizeof(PrepBlock), hipMemcpyHostToDevice));
  p->ws = ws;
  p->ws_bytes = bytes;
  p->ws_bound = true;
  p->screened = false;
  p->executed = false;
  p->split_src_A = p->split_src_B = nullptr;  // the workspace holds no split yet
  return TAMM_OK;
}

extern "C" int tamm_plan_bind_workspace(tamm_plan* p, void* dev_ptr, size_t bytes) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  const int rc = bind_plan(p, dev_ptr, bytes);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_plan_stats_get(const tamm_plan* p, tamm_plan_stats* s) {
  if (!p || !s) return fail(TAMM_ERR_ARG, "null argument");
  *s = p->stats;
  return ok();
}

extern "C" int tamm_plan_config_count(const tamm_plan* p, int32_t* count) {
  if (!p || !count) return fail(TAMM_ERR_ARG, "null argument");
  *count = cfg_count(p->prec);
  return ok();
}

extern "C" int tamm_plan_set_config(tamm_plan* p, int32_t config, int32_t k_splits) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  if (config < 0 || config >= cfg_count(p->prec)) return fail(TAMM_ERR_ARG, "configuration %d does not exist", config);
  if (k_splits < 0 || k_splits > 64) return fail(TAMM_ERR_ARG, "k_splits must be in [0, 64]");
  const int rc = configure_work(p, config, k_splits);
  if (rc != TAMM_OK) return rc;
  return ok();
}

extern "C" int tamm_plan_set_constant(tamm_plan* p, int32_t which, int32_t constant) {
  if (!p || (which != 0 && which != 1)) return fail(TAMM_ERR_ARG, "null plan or operand not 0 or 1");
  const bool is_a = (which == 0) != p->swapped;  // lhs is A unless it holds out's last label
  (is_a ? p->const_A : p->const_B) = constant != 0;
  (is_a ? p->split_src_A : p->split_src_B) = nullptr;  // split again at the next execution
  return ok();
}

extern "C" int tamm_plan_set_order(tamm_plan* p, int32_t tile_order, int32_t chunk) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  if (tile_order != 0 && tile_order != 1) return fail(TAMM_ERR_ARG, "tile order must be 0 or 1");
  if (chunk < -1 || chunk > (1 << 20)) return fail(TAMM_ERR_ARG, "chunk must be -1, 0 or a positive item count");
  p->tile_order = tile_order;
  p->xcd_chunk = chunk;
  const int rc = configure_work(p, p->config, p->k_splits);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" const char* tamm_config_name(int32_t precision, int32_t config) {
  if (precision < TAMM_PREC_F64 || precision > TAMM_PREC_BF16X4_ALIGNED) return "";
  if (config < 0 || config >= cfg_count(precision)) return "";
  return cfg_get(precision, config).name;
}

static bool overlaps(const tamm_tensor* a, const tamm_tensor* b) {
  if (a->numel == 0 || b->numel == 0) return false;
  const char* a0 = (const char*)a->dev;
  const char* b0 = (const char*)b->dev;
  return a0 < b0 + b->numel * 8 && b0 < a0 + a->numel * 8;
}

static int check_tensors(const tamm_plan* p) {
  const tamm_tensor* ts[3] = {p->out, p->lhs, p->rhs};
  const char* nm[3] = {"out", "lhs", "rhs"};
  for (int x = 0; x < 3; ++x)
    if (!ts[x]->bound) return fail(TAMM_ERR_UNBOUND, "%s tensor has no bound storage", nm[x]);
  if (overlaps(p->out, p->lhs) || overlaps(p->out, p->rhs)) return fail(TAMM_ERR_ARG, "out storage overlaps an operand");
  return TAMM_OK;
}

static int check_bound(const tamm_plan* p) {
  if (!p->ws_bound) return fail(TAMM_ERR_UNBOUND, "plan workspace is not bound (or the configuration changed since binding)");
  return check_tensors(p);
}

extern "C" int tamm_plan_screen(tamm_plan* p, void* stream) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  int rc = check_bound(p);
  if (rc != TAMM_OK) return rc;
  ScreenParams sp{};
  sp.single = screen_desc(p, p->ws, p->lay);
  sp.n_items = sp.single.n_blocks;
  HIP_TRY(launch_screen(sp, (hipStream_t)stream));
  p->screened = true;
  return ok();
}

static int contract_launch(tamm_plan* p, double alpha, double beta, hipStream_t s) {
  ContractParams cp{};
  cp.single = problem_desc(p, p->ws, p->lay, p->k_splits > 1 ? (double*)(p->ws + p->off_partial) : nullptr, p->k_splits,
                           alpha, beta);
  cp.probs = nullptr;
  cp.work = (const WorkItem*)(p->ws + p->off_work);
  cp.next_item = nullptr;
  cp.n_work = (int32_t)p->work.size();
  const int layout = gather_layout(p);
  if (p->prec == TAMM_PREC_F64) {
    HIP_TRY(launch_contract_f64(p->config, layout, cp, 0, s));
  } else {
    if (p->prec != TAMM_PREC_F32) {
      // operand split into packed bfloat16 slices, then the contraction reads the split copies
      PrepParams pa{};
      pa.x = p->A->dev;
      pa.out = (uint64_t*)(p->ws + p->off_xA);
      pa.blocks = (const PrepBlock*)(p->ws + p->off_prepA);
      pa.pool = (const int32_t*)(p->ws + p->lay.pool);
      pa.n_items = p->prepA_items;
      pa.n_blocks = (int32_t)p->prepA.size();
      pa.aligned = p->prec == TAMM_PREC_BF16X4_ALIGNED ? 1 : 0;
      pa.planes = p->planes ? 1 : 0;
      pa.plane_stride = p->A->numel;
      // a constant operand keeps the split of an earlier execution from the same storage
      if (!(p->const_A && p->split_src_A == p->A->dev)) HIP_TRY(launch_prep_split(pa, !p->a_kc, s));
      p->split_src_A = p->const_A ? (const void*)p->A->dev : nullptr;
      PrepParams pbp = pa;
      pbp.x = p->B->dev;
      pbp.out = (uint64_t*)(p->ws + p->off_xB);
      pbp.blocks = (const PrepBlock*)(p->ws + p->off_prepB);
      pbp.n_items = p->prepB_items;
      pbp.n_blocks = (int32_t)p->prepB.size();
      pbp.plane_stride = p->B->numel;
      if (!(p->const_B && p->split_src_B == p->B->dev)) HIP_TRY(launch_prep_split(pbp, !p->b_kc, s));
      p->split_src_B = p->const_B ? (const void*)p->B->dev : nullptr;
      cp.single.A = (const double*)(p->ws + p->off_xA);
      cp.single.B = (const double*)(p->ws + p->off_xB);
      if (p->planes) {
        cp.single.a_plane = p->A->numel;
        cp.single.b_plane = p->B->numel;
      }
    }
    const bool planes = p->planes && p->prec != TAMM_PREC_F32;
    HIP_TRY(launch_contract_mixed(p->prec, p->config, planes ? kPlanesLayout : (layout & 3), cp, s));
  }
  if (p->k_splits > 1) {
    const TileCfg f = cfg_get(p->prec, p->config);
    ReduceParams r{};
    r.single = cp.single;
    r.probs = nullptr;
    r.items = (const ReduceItem*)(p->ws + p->off_reduce);
    r.n_items = (int32_t)p->reduce.size();
    r.tile_m = f.mt;
    r.tile_n = f.nt;
    HIP_TRY(launch_reduce(r, s));
  }
  return TAMM_OK;
}

extern "C" int tamm_plan_contract(tamm_plan* p, double alpha, double beta, void* stream) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  int rc = check_bound(p);
  if (rc != TAMM_OK) return rc;
  if (!p->screened) return fail(TAMM_ERR_UNBOUND, "the plan has not been screened on its bound workspace");
  rc = contract_launch(p, alpha, beta, (hipStream_t)stream);
  if (rc != TAMM_OK) return rc;
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
  if (!p->ws_bound || !p->screened) return fail(TAMM_ERR_UNBOUND, "plan has not been screened on a bound workspace");
  const size_t nob = p->blocks.size();
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(counts, p->ws + p->lay.counts, nob * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (k_tiles) {
    std::vector<PairDesc> pairs((size_t)nob * p->n_kt);
    HIP_TRY(hipMemcpy(pairs.data(), p->ws + p->lay.pairs, pairs.size() * sizeof(PairDesc), hipMemcpyDeviceToHost));
    const int nk = p->sd.nk;
    std::vector<int> t(nk);
    size_t w = 0;
    for (size_t b = 0; b < nob; ++b)
      for (int i = 0; i < counts[b]; ++i) {
        int rem = pairs[b * p->n_kt + i].kt;
        for (int q = nk - 1; q >= 0; --q) {
          t[q] = rem % p->sd.k_ntiles[q];
          rem /= p->sd.k_ntiles[q];
        }
        for (int j = 0; j < nk; ++j) k_tiles[w++] = t[p->k_lhs_order[j]];
      }
  }
  return ok();
}

extern "C" int tamm_plan_split_operand(const tamm_plan* p, int32_t which, void* out_dev, size_t bytes, void* stream) {
  if (!p || !out_dev || (which != 0 && which != 1)) return fail(TAMM_ERR_ARG, "null plan or buffer, or operand not 0 or 1");
  if (p->prec != TAMM_PREC_BF16X3 && p->prec != TAMM_PREC_BF16X4_ALIGNED)
    return fail(TAMM_ERR_UNSUPPORTED, "the plan's precision splits no operand");
  const int rc = check_bound(p);
  if (rc != TAMM_OK) return rc;
  const bool is_a = (which == 0) != p->swapped;  // lhs is A unless it holds out's last label
  const tamm_tensor* t = is_a ? p->A : p->B;
  if (bytes < (size_t)t->numel * sizeof(uint64_t))
    return fail(TAMM_ERR_WORKSPACE, "output buffer of %zu bytes is smaller than %lld words", bytes, (long long)t->numel);
  PrepParams pa{};
  pa.x = t->dev;
  pa.out = out_dev;
  pa.blocks = (const PrepBlock*)(p->ws + (is_a ? p->off_prepA : p->off_prepB));
  pa.pool = (const int32_t*)(p->ws + p->lay.pool);
  pa.n_items = is_a ? p->prepA_items : p->prepB_items;
  pa.n_blocks = (int32_t)(is_a ? p->prepA.size() : p->prepB.size());
  pa.aligned = p->prec == TAMM_PREC_BF16X4_ALIGNED ? 1 : 0;
  pa.planes = 0;  // packed words at the float64 element offsets
  HIP_TRY(launch_prep_split(pa, is_a ? !p->a_kc : !p->b_kc, (hipStream_t)stream));
  return ok();
}

extern "C" int tamm_plan_destroy(tamm_plan* p) {
  delete p;
  return ok();
}

// ---------------------------------------------------------------------------------------------
// one-shot contraction: plans cached inside the library, keyed by tensor handles and labels
// ---------------------------------------------------------------------------------------------
namespace {

struct ContractKey {
  const tamm_tensor* out;
  const tamm_tensor* lhs;
  const tamm_tensor* rhs;
  std::string labels;  // out, lhs and rhs labels joined by '/'
  int32_t precision;
  bool operator<(const ContractKey& o) const {
    return std::tie(out, lhs, rhs, labels, precision) < std::tie(o.out, o.lhs, o.rhs, o.labels, o.precision);
  }
};

struct ContractCache {
  std::mutex mu;
  std::map<ContractKey, std::unique_ptr<tamm_plan>> plans;
  struct Holder {
    const tamm_plan* plan;  // the plan whose tables the workspace holds
    size_t bytes;           // the workspace's length
  };
  std::map<const void*, Holder> holder;  // workspace start -> its holder
};

// Never destroyed: tensor handles may be released from other static destructors at exit.
ContractCache& contract_cache() {
  static ContractCache* c = new ContractCache;
  return *c;
}

// The cached plan for a contraction, created on first use.  The caller holds the cache lock.
int cached_plan(ContractCache& c, tamm_tensor* out, const char* ol, const tamm_tensor* lhs, const char* ll,
                const tamm_tensor* rhs, const char* rl, int32_t precision, tamm_plan** plan) {
  if (!out || !lhs || !rhs || !ol || !ll || !rl) return fail(TAMM_ERR_ARG, "null tensor or label string");
  ContractKey key{out, lhs, rhs, std::string(ol) + "/" + ll + "/" + rl, precision};
  auto it = c.plans.find(key);
  if (it != c.plans.end()) {
    *plan = it->second.get();
    return TAMM_OK;
  }
  tamm_plan* p = nullptr;
  const int rc = tamm_plan_create(out, ol, lhs, ll, rhs, rl, (tamm_precision)precision, &p);
  if (rc != TAMM_OK) return rc;
  c.plans.emplace(std::move(key), std::unique_ptr<tamm_plan>(p));
  *plan = p;
  return TAMM_OK;
}

}  // namespace

void tamm::contract_cache_evict(const tamm_tensor* t) {
  ContractCache& c = contract_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto it = c.plans.begin(); it != c.plans.end();) {
    if (it->first.out != t && it->first.lhs != t && it->first.rhs != t) {
      ++it;
      continue;
    }
    for (auto h = c.holder.begin(); h != c.holder.end();) h = h->second.plan == it->second.get() ? c.holder.erase(h) : std::next(h);
    it = c.plans.erase(it);
  }
}

extern "C" int tamm_contract_workspace_size(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs,
                                            const char* lhs_lbl, const tamm_tensor* rhs, const char* rhs_lbl,
                                            int32_t precision, size_t* bytes) {
  if (!bytes) return fail(TAMM_ERR_ARG, "null argument");
  ContractCache& c = contract_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  tamm_plan* p = nullptr;
  const int rc = cached_plan(c, out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl, precision, &p);
  if (rc != TAMM_OK) return rc;
  *bytes = p->ws_size;
  return ok();
}

extern "C" int tamm_contract(tamm_tensor* out, const char* out_lbl, const tamm_tensor* lhs, const char* lhs_lbl,
                             const tamm_tensor* rhs, const char* rhs_lbl, int32_t precision, double alpha, double beta,
                             void* workspace, size_t bytes, void* stream) {
  ContractCache& c = contract_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  tamm_plan* p = nullptr;
  int rc = cached_plan(c, out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl, precision, &p);
  if (rc != TAMM_OK) return rc;
  const auto h = c.holder.find(workspace);
  const bool holds = p->ws_bound && p->ws == (char*)workspace && p->ws_bytes == bytes && h != c.holder.end() &&
                     h->second.plan == p && h->second.bytes == bytes;
  if (!holds) {
    if (!workspace || ((uintptr_t)workspace) % 256)
      return fail(TAMM_ERR_WORKSPACE, "workspace must be non-null and 256-byte aligned");
    if (bytes < p->ws_size)
      return fail(TAMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, p->ws_size);
    // Earlier calls, on any stream, may still read tables in the range this upload overwrites:
    // drain the device before replacing them (a rare path: it runs when a workspace changes hands).
    const char* lo = (const char*)workspace;
    bool busy = false;
    for (auto it = c.holder.begin(); it != c.holder.end();) {
      const char* o = (const char*)it->first;
      if (o < lo + bytes && lo < o + it->second.bytes) {
        busy = true;
        it = c.holder.erase(it);
      } else {
        ++it;
      }
    }
    if (busy) HIP_TRY(hipDeviceSynchronize());
    rc = bind_plan(p, workspace, bytes);
    if (rc != TAMM_OK) return rc;
    c.holder[workspace] = ContractCache::Holder{p, bytes};
  }
  return tamm_plan_execute(p, alpha, beta, stream);
}

extern "C" int tamm_contract_cache_count(int64_t* plans) {
  if (!plans) return fail(TAMM_ERR_ARG, "null argument");
  ContractCache& c = contract_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  *plans = (int64_t)c.plans.size();
  return ok();
}

extern "C" int tamm_contract_cache_clear(void) {
  ContractCache& c = contract_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.holder.clear();
  c.plans.clear();
  return ok();
}

// ---------------------------------------------------------------------------------------------
// autotuner (plans)
// ---------------------------------------------------------------------------------------------
namespace {

struct CacheEntry {
  int config, k_splits, grid;
  double ms;
};

// The two timing events of an autotuner, destroyed on every exit path (HIP_TRY returns early).
struct TimerEvents {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int create() {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    return TAMM_OK;
  }
  ~TimerEvents() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

bool cache_lookup(const char* path, uint64_t sig, const char* kind, CacheEntry& e) {
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string s, k;
    CacheEntry c{};
    if (!(is >> s >> k >> c.config >> c.k_splits >> c.grid >> c.ms)) continue;
    if (k == kind && std::strtoull(s.c_str(), nullptr, 16) == sig) {
      e = c;
      found = true;  // the last entry wins
    }
  }
  return found;
}

void cache_store(const char* path, uint64_t sig, const char* kind, const CacheEntry& e) {
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  char buf[160];
  snprintf(buf, sizeof(buf), "%016llx %s %d %d %d %.6f\n", (unsigned long long)sig, kind, e.config, e.k_splits, e.grid, e.ms);
  f << buf;
}

}  // namespace

extern "C" int tamm_plan_autotune_workspace_size(const tamm_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  tamm_plan tmp = *p;
  size_t mx = 0;
  for (int c = 0; c < cfg_count(p->prec); ++c)
    for (int ks : {1, 2, 4, 8}) {
      if (configure_work(&tmp, c, ks) != TAMM_OK) continue;
      mx = std::max(mx, tmp.ws_size);
    }
  *bytes = mx;
  return ok();
}

extern "C" int tamm_plan_autotune(tamm_plan* p, void* workspace, size_t bytes, void* stream, const char* cache_path,
                                  int32_t reps) {
  if (!p) return fail(TAMM_ERR_ARG, "null plan");
  int rc = check_tensors(p);
  if (rc != TAMM_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  // cache entries of kind "plan2" hold the configuration, K splits and die chunk (grid field)
  CacheEntry best{-1, 1, -1, 1e30};
  if (!cache_lookup(cache_path, p->signature, "plan2", best)) {
    if (reps <= 0) reps = 3;
    TimerEvents ev;
    if ((rc = ev.create()) != TAMM_OK) return rc;
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    // one candidate: configure, bind, warm up, fastest of reps (alpha = 0, beta = 1 leaves out
    // unchanged for finite operands while doing the full work)
    auto trial = [&](int c, int ks, float* ms) -> int {
      *ms = 1e30f;
      if (configure_work(p, c, ks) != TAMM_OK || p->ws_size > bytes) return TAMM_OK;
      int r = bind_plan(p, workspace, bytes);
      if (r != TAMM_OK) return r;
      if ((r = tamm_plan_execute(p, 0.0, 1.0, stream)) != TAMM_OK) return r;
      for (int i = 0; i < reps; ++i) {
        HIP_TRY(hipEventRecord(e0, s));
        if ((r = tamm_plan_execute(p, 0.0, 1.0, stream)) != TAMM_OK) return r;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float one = 0;
        HIP_TRY(hipEventElapsedTime(&one, e0, e1));
        *ms = std::min(*ms, one);
      }
      return TAMM_OK;
    };
    const int chunk0 = p->xcd_chunk;
    const int64_t ntiles_max = tiles_for(p, 0).first;
    std::vector<CacheEntry> ranked;  // every (configuration, K splits) at the current launch order
    for (int c = 0; c < cfg_count(p->prec) && rc == TAMM_OK; ++c) {
      const int64_t nt = tiles_for(p, c).first;
      for (int ks : {1, 2, 4, 8}) {
        if (ks > 1 && nt * ks > 4 * std::max<int64_t>(ntiles_max, 2048)) continue;
        float ms = 0;
        if ((rc = trial(c, ks, &ms)) != TAMM_OK) break;
        if (ms < 1e29f) ranked.push_back(CacheEntry{c, ks, chunk0, ms});
        if (ms < best.ms) best = CacheEntry{c, ks, chunk0, ms};
      }
    }
    // tile orders and die chunks (they change only the launch order) for the three fastest
    // (configuration, K splits) of the first pass, since a configuration that loses at one order
    // can win at another; the cache's grid field holds chunk + order * 2^24
    if (rc == TAMM_OK && best.config >= 0) {
      best.grid = (chunk0 < 0 ? xcd_chunk() : chunk0) + (p->tile_order << 24);
      std::stable_sort(ranked.begin(), ranked.end(), [](const CacheEntry& x, const CacheEntry& y) { return x.ms < y.ms; });
      if (ranked.size() > 3) ranked.resize(3);
      std::vector<CacheEntry> finals{best};  // every candidate with its launch order
      for (const CacheEntry& cand : ranked)
        for (int order : {0, 1})
          for (int ch : {0, 16, 32, 64, 128}) {
            if (rc != TAMM_OK) break;  // a failed trial ends the search with its error
            p->xcd_chunk = ch;
            p->tile_order = order;
            float ms = 0;
            if ((rc = trial(cand.config, cand.k_splits, &ms)) != TAMM_OK) break;
            if (ms < 1e29f) finals.push_back(CacheEntry{cand.config, cand.k_splits, ch + (order << 24), ms});
            if (ms < best.ms) best = CacheEntry{cand.config, cand.k_splits, ch + (order << 24), ms};
          }
      // confirmation: the fastest single trial among candidates within a few per cent of each
      // other is partly chance, so the three fastest are timed again in turn, three rounds, and
      // the lowest median kept
      std::stable_sort(finals.begin(), finals.end(), [](const CacheEntry& x, const CacheEntry& y) { return x.ms < y.ms; });
      std::vector<CacheEntry> top;
      for (const CacheEntry& f : finals) {
        bool dup = false;
        for (const CacheEntry& t : top)
          dup = dup || (t.config == f.config && t.k_splits == f.k_splits && t.grid == f.grid);
        if (!dup) top.push_back(f);
        if (top.size() == 3) break;
      }
      if (rc == TAMM_OK && top.size() > 1) {
        std::vector<std::vector<float>> times(top.size());
        for (int round = 0; round < 3 && rc == TAMM_OK; ++round)
          for (size_t t = 0; t < top.size() && rc == TAMM_OK; ++t) {
            p->xcd_chunk = top[t].grid & 0xFFFFFF;
            p->tile_order = (top[t].grid >> 24) & 1;
            float ms = 0;
            if ((rc = trial(top[t].config, top[t].k_splits, &ms)) != TAMM_OK) break;
            times[t].push_back(ms);
          }
        if (rc == TAMM_OK) {
          size_t pick = 0;
          float pick_ms = 1e30f;
          for (size_t t = 0; t < top.size(); ++t) {
            std::vector<float> v = times[t];
            std::sort(v.begin(), v.end());
            if (v[v.size() / 2] < pick_ms) {
              pick_ms = v[v.size() / 2];
              pick = t;
            }
          }
          best = CacheEntry{top[pick].config, top[pick].k_splits, top[pick].grid, pick_ms};
        }
      }
    }
    if (rc != TAMM_OK) return rc;
    if (best.config < 0) return fail(TAMM_ERR_WORKSPACE, "no configuration fits the %zu-byte workspace", bytes);
    cache_store(cache_path, p->signature, "plan2", best);
  }
  p->xcd_chunk = best.grid < 0 ? -1 : (best.grid & 0xFFFFFF);
  p->tile_order = best.grid < 0 ? 0 : (best.grid >> 24) & 1;
  rc = configure_work(p, best.config, best.k_splits);
  if (rc != TAMM_OK) return rc;
  if (p->ws_size > bytes) return fail(TAMM_ERR_WORKSPACE, "cached configuration needs %zu bytes", p->ws_size);
  rc = bind_plan(p, workspace, bytes);
  return rc == TAMM_OK ? ok() : rc;
}

// ---------------------------------------------------------------------------------------------
// groups: contraction nodes executed together -- one screening launch and one persistent
// contraction launch per gather layout class (each with its own configuration), optionally
// captured once into a hipGraph and replayed.  A node is one plan, or several plans that write
// the same output tiles (a fused node, built by the scheduler): their pair lists are screened
// into one list per output block and one output tile's K loop runs over all of them.
// ---------------------------------------------------------------------------------------------
struct tamm_group {
  std::vector<std::vector<tamm_plan*>> nodes;  // member plans of each node
  std::vector<tamm_plan*> plans;               // every member plan, node by node
  std::vector<int32_t> node_first;             // index in `plans` (and segment index) of each node's first plan
  std::vector<Layout> lays;                    // static tables of each plan
  struct Fused {
    size_t blocks = 0, pairs = 0, counts = 0;  // regions of a fused node's own output descriptors and pair list
    int32_t stride = 0;                        // pair capacity per output block (sum over the members)
  };
  std::vector<Fused> fused;                    // per node (fused nodes only)
  size_t off_sdesc = 0, off_pdesc = 0, off_sitems = 0, off_work = 0, off_counter = 0, ws_size = 0;
  std::vector<int32_t> sitem_prob, sitem_block;  // screening items: first segment of the node, output block
  std::vector<WorkItem> work;       // grouped by gather layout class, each class longest first (prob = node)
  size_t work_capacity = 0;         // work items of the largest mix of per-class configurations
  int32_t cls_begin[kLayouts + 1] = {};  // work range of gather layout c: [cls_begin[c], cls_begin[c+1])
  int cfg[kLayouts] = {};   // kernel configuration of each layout class (its tile shape)
  int grid[kLayouts] = {};  // persistent grid of each layout class (0: automatic)
  uint64_t signature = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  std::vector<ProblemDesc> pdesc;   // host copy per node (alpha/beta updated per execute)
  std::vector<ScreenDesc> sdesc;    // host copy per plan (segment)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<double> g_alpha, g_beta;
  // side streams (default priority) and events that run the layout classes' launches
  // concurrently, forked after the screening launch and joined back into the caller's stream
  hipStream_t side[kLayouts] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kLayouts] = {};
};

static void group_drop_graph(tamm_group* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
}

// Gather layout of a node: its plans share the operand orientations; 16-byte gathers only when
// every member's tables allow them.
static int node_layout(const tamm_group* g, size_t q) {
  int lay = gather_layout(g->nodes[q][0]) & 3;
  bool pairs = true;
  for (const tamm_plan* p : g->nodes[q]) pairs = pairs && p->pairs;
  return lay | (pairs ? 4 : 0);
}

// Summed K extent of the surviving pairs of output block b over the node's plans.
static double node_block_cost(const tamm_group* g, size_t q, size_t b) {
  double c = 0;
  for (const tamm_plan* p : g->nodes[q]) c += p->block_cost[b];
  return c;
}

// Default configuration of a set of nodes: the one with the least padding, ties to the larger
// tile.
static int group_default_config(const tamm_group* g, int layout) {
  int config = 0;
  double best = 1e30;
  for (int c = 0; c < f64_config_count(); ++c) {
    const F64Config& f = f64_config(c);
    if (f.kt != 16 || f.wgm * f.wgn != 4 || f.mt > 128 || f.nt > 128) continue;
    double area = 0, useful = 0;
    for (size_t q = 0; q < g->nodes.size(); ++q) {
      if (layout >= 0 && node_layout(g, q) != layout) continue;
      for (const auto& b : g->nodes[q][0]->blocks) {
        area += (double)((b.mext + f.mt - 1) / f.mt) * f.mt * ((b.next + f.nt - 1) / f.nt) * f.nt;
        useful += (double)b.mext * b.next;
      }
    }
    const double score = (useful > 0 ? area / useful : 1.0) - 1e-6 * f.mt * f.nt;
    if (score < best) {
      best = score;
      config = c;
    }
  }
  return config;
}

// Work lists of every layout class with the class's configuration cfgs[c] (< 0: the class's
// default), each heaviest first, and the workspace layout.
static int group_configure_classes(tamm_group* g, const int* cfgs) {
  for (int c = 0; c < kLayouts; ++c) {
    const int k = cfgs[c] < 0 ? group_default_config(g, c) : cfgs[c];
    if (k >= f64_config_count()) return fail(TAMM_ERR_ARG, "configuration %d does not exist", k);
    g->cfg[c] = k;
  }
  struct Tile {
    double cost;
    WorkItem w;
  };
  g->work.clear();
  for (int c = 0; c < kLayouts; ++c) {
    const F64Config& f = f64_config(g->cfg[c]);
    std::vector<Tile> tiles;
    for (size_t q = 0; q < g->nodes.size(); ++q) {
      if (node_layout(g, q) != c) continue;
      const tamm_plan* p = g->nodes[q][0];
      int32_t t = 0;
      for (size_t b = 0; b < p->blocks.size(); ++b) {
        const auto& d = p->blocks[b];
        const double bc = node_block_cost(g, q, b);
        for (int32_t m0 = 0; m0 < d.mext; m0 += f.mt)
          for (int32_t n0 = 0; n0 < d.next; n0 += f.nt)
            tiles.push_back(Tile{bc * std::min(f.mt, d.mext - m0) * std::min(f.nt, d.next - n0),
                                 WorkItem{(int32_t)q, (int32_t)b, m0, n0, 0, t++}});
      }
    }
    std::stable_sort(tiles.begin(), tiles.end(), [](const Tile& x, const Tile& y) { return x.cost > y.cost; });
    g->cls_begin[c] = (int32_t)g->work.size();
    for (auto& t : tiles) g->work.push_back(t.w);
  }
  g->cls_begin[kLayouts] = (int32_t)g->work.size();
  size_t off = 0;
  g->lays.clear();
  for (auto* p : g->plans) {
    g->lays.push_back(make_layout(p, off));
    off = g->lays.back().end;
  }
  g->fused.assign(g->nodes.size(), tamm_group::Fused{});
  for (size_t q = 0; q < g->nodes.size(); ++q) {
    if (g->nodes[q].size() < 2) continue;
    tamm_group::Fused& F = g->fused[q];
    const size_t nob = g->nodes[q][0]->blocks.size();
    int64_t stride = 0;
    for (const tamm_plan* p : g->nodes[q]) stride += p->n_kt;
    F.stride = (int32_t)stride;
    F.blocks = align256(off);
    off = align256(F.blocks + nob * sizeof(OutBlockDesc));
    F.pairs = off;
    off = align256(off + nob * (size_t)stride * sizeof(PairDesc));
    F.counts = off;
    off = align256(off + nob * sizeof(int32_t));
  }
  g->off_sdesc = off;
  off = align256(off + g->plans.size() * sizeof(ScreenDesc));
  g->off_pdesc = off;
  off = align256(off + g->nodes.size() * sizeof(ProblemDesc));
  g->off_sitems = off;
  off = align256(off + g->sitem_prob.size() * 2 * sizeof(int32_t));
  g->off_work = off;
  // room for any mix of per-class configurations, so the autotuner's choice always fits the
  // workspace sized for the candidates
  off = align256(off + std::max(g->work.size(), g->work_capacity) * sizeof(WorkItem));
  g->off_counter = off;  // one work counter per gather layout
  off = align256(off + kLayouts * sizeof(int32_t));
  g->ws_size = off;
  g->bound = false;
  group_drop_graph(g);
  return TAMM_OK;
}

// One configuration for every class (< 0: each class's default).
static int group_configure(tamm_group* g, int config) {
  int cfgs[kLayouts];
  for (int c = 0; c < kLayouts; ++c) cfgs[c] = config;
  return group_configure_classes(g, cfgs);
}

// Plans that can share output tiles: float64, the same output tensor, the same flattening of the
// output's labels into rows (M) and columns (N), and the same operand orientations.
static int check_fusable(const std::vector<tamm_plan*>& node) {
  const tamm_plan* p0 = node[0];
  auto out_dims = [](const tamm_plan* p, const std::vector<int>& grp) {
    std::vector<int> d;
    for (int l : grp) d.push_back(p->labels[l].od);
    return d;
  };
  for (size_t i = 1; i < node.size(); ++i) {
    const tamm_plan* p = node[i];
    if (p->out != p0->out) return fail(TAMM_ERR_ARG, "fused plans must write the same output tensor");
    if (out_dims(p, p->M) != out_dims(p0, p0->M) || out_dims(p, p->N) != out_dims(p0, p0->N) || p->a_kc != p0->a_kc ||
        p->b_kc != p0->b_kc)
      return fail(TAMM_ERR_UNSUPPORTED, "fused plans must split the output into the same rows and columns");
  }
  int64_t stride = 0;
  for (const tamm_plan* p : node) stride += p->n_kt;
  if ((int64_t)p0->blocks.size() * stride > (int64_t)1 << 28) return fail(TAMM_ERR_UNSUPPORTED, "fused pair capacity too large");
  return TAMM_OK;
}

namespace tamm {

// Create a group of nodes (each node one plan, or several fusable plans writing the same output).
int group_create_nodes(const std::vector<std::vector<tamm_plan*>>& nodes, tamm_group** out) {
  *out = nullptr;
  if (nodes.empty()) return fail(TAMM_ERR_ARG, "a group needs at least one plan");
  auto g = std::make_unique<tamm_group>();
  uint64_t h = 0xCBF29CE484222325ULL;
  for (size_t q = 0; q < nodes.size(); ++q) {
    if (nodes[q].empty()) return fail(TAMM_ERR_ARG, "node %zu is empty", q);
    for (tamm_plan* p : nodes[q]) {
      if (!p) return fail(TAMM_ERR_ARG, "a member plan is null");
      if (p->prec != TAMM_PREC_F64) return fail(TAMM_ERR_UNSUPPORTED, "groups run float64 plans only");
    }
    int rc = check_fusable(nodes[q]);
    if (rc != TAMM_OK) return rc;
    for (size_t r = 0; r < q; ++r)
      if (nodes[r][0]->out == nodes[q][0]->out)
        return fail(TAMM_ERR_ARG, "members %zu and %zu write the same output tensor", r, q);
    g->nodes.push_back(nodes[q]);
    g->node_first.push_back((int32_t)g->plans.size());
    const uint32_t sz = (uint32_t)nodes[q].size();
    h = fnv(h, &sz, sizeof(sz));
    for (tamm_plan* p : nodes[q]) {
      g->plans.push_back(p);
      h = fnv(h, &p->signature, sizeof(uint64_t));
    }
    for (size_t b = 0; b < nodes[q][0]->blocks.size(); ++b) {
      g->sitem_prob.push_back(g->node_first.back());
      g->sitem_block.push_back((int32_t)b);
    }
  }
  g->signature = h;
  for (int c = 0; c < kLayouts; ++c) {
    size_t most = 0;
    for (int k = 0; k < f64_config_count(); ++k) {
      const F64Config& f = f64_config(k);
      size_t n = 0;
      for (size_t q = 0; q < g->nodes.size(); ++q)
        if (node_layout(g.get(), q) == c)
          for (const auto& b : g->nodes[q][0]->blocks)
            n += (size_t)((b.mext + f.mt - 1) / f.mt) * ((b.next + f.nt - 1) / f.nt);
      most = std::max(most, n);
    }
    g->work_capacity += most;
  }
  const int rc = group_configure(g.get(), -1);
  if (rc != TAMM_OK) return rc;
  *out = g.release();
  return TAMM_OK;
}

}  // namespace tamm

extern "C" int tamm_group_create(tamm_plan* const* plans, int32_t n, tamm_group** out) {
  if (!out) return fail(TAMM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!plans || n <= 0) return fail(TAMM_ERR_ARG, "a group needs at least one plan");
  std::vector<std::vector<tamm_plan*>> nodes;
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return fail(TAMM_ERR_ARG, "plan %d is null", i);
    nodes.push_back({plans[i]});
  }
  const int rc = group_create_nodes(nodes, out);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_group_workspace_size(const tamm_group* g, size_t* bytes) {
  if (!g || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = g->ws_size;
  return ok();
}

// Screening descriptors of every plan (segment) and problem descriptors of every node for the
// current tensor bindings and coefficients.
static void group_descs(const tamm_group* g, char* ws, const double* alpha, const double* beta, std::vector<ScreenDesc>& sds,
                        std::vector<ProblemDesc>& pds) {
  sds.clear();
  pds.clear();
  for (size_t q = 0; q < g->nodes.size(); ++q) {
    const int first = g->node_first[q];
    const tamm_plan* p0 = g->nodes[q][0];
    const Layout& L0 = g->lays[first];
    ProblemDesc pd = problem_desc(p0, ws, L0, nullptr, 1, alpha[q], beta[q]);
    const bool fused = g->nodes[q].size() > 1;
    const tamm_group::Fused& F = g->fused[q];
    if (fused) {
      pd.blocks = (const OutBlockDesc*)(ws + F.blocks);
      pd.pairs = (const PairDesc*)(ws + F.pairs);
      pd.counts = (const int32_t*)(ws + F.counts);
    }
    pds.push_back(pd);
    for (size_t i = 0; i < g->nodes[q].size(); ++i) {
      const tamm_plan* p = g->nodes[q][i];
      const Layout& L = g->lays[first + i];
      ScreenDesc s = screen_desc(p, ws, L);
      if (fused) {
        s.pairs = (PairDesc*)(ws + F.pairs);
        s.counts = (int32_t*)(ws + F.counts);
        s.pair_stride = F.stride;
        // element offsets and table starts relative to the first member's operands and pool
        s.a_base = (int64_t)((const double*)p->A->dev - (const double*)p0->A->dev);
        s.b_base = (int64_t)((const double*)p->B->dev - (const double*)p0->B->dev);
        s.pool_base = (int32_t)(((int64_t)L.pool - (int64_t)L0.pool) / (int64_t)sizeof(int32_t));
        s.next_seg = i + 1 < g->nodes[q].size() ? first + (int32_t)i + 1 : -1;
      }
      sds.push_back(s);
    }
  }
}

static int group_bind(tamm_group* g, void* dev_ptr, size_t bytes) {
  if (!dev_ptr || ((uintptr_t)dev_ptr) % 256) return fail(TAMM_ERR_WORKSPACE, "workspace must be non-null and 256-byte aligned");
  if (bytes < g->ws_size) return fail(TAMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes, g->ws_size);
  char* ws = (char*)dev_ptr;
  for (size_t q = 0; q < g->plans.size(); ++q) {
    int rc = upload_static(g->plans[q], ws, g->lays[q]);
    if (rc != TAMM_OK) return rc;
  }
  for (size_t q = 0; q < g->nodes.size(); ++q) {
    if (g->nodes[q].size() < 2) continue;
    std::vector<OutBlockDesc> d = g->nodes[q][0]->blocks;  // the first member's tables, the node's pair list
    for (size_t b = 0; b < d.size(); ++b) d[b].pair_base = (int32_t)(b * (size_t)g->fused[q].stride);
    if (!d.empty()) HIP_TRY(hipMemcpy(ws + g->fused[q].blocks, d.data(), d.size() * sizeof(OutBlockDesc), hipMemcpyHostToDevice));
  }
  std::vector<double> one(g->nodes.size(), 1.0), zero(g->nodes.size(), 0.0);
  group_descs(g, ws, one.data(), zero.data(), g->sdesc, g->pdesc);
  HIP_TRY(hipMemcpy(ws + g->off_sdesc, g->sdesc.data(), g->sdesc.size() * sizeof(ScreenDesc), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ws + g->off_pdesc, g->pdesc.data(), g->pdesc.size() * sizeof(ProblemDesc), hipMemcpyHostToDevice));
  std::vector<int32_t> items(g->sitem_prob);
  items.insert(items.end(), g->sitem_block.begin(), g->sitem_block.end());
  if (!items.empty()) HIP_TRY(hipMemcpy(ws + g->off_sitems, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!g->work.empty()) HIP_TRY(hipMemcpy(ws + g->off_work, g->work.data(), g->work.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  g->ws = ws;
  g->ws_bytes = bytes;
  g->bound = true;
  group_drop_graph(g);
  return TAMM_OK;
}

extern "C" int tamm_group_bind_workspace(tamm_group* g, void* dev_ptr, size_t bytes) {
  if (!g) return fail(TAMM_ERR_ARG, "null group");
  const int rc = group_bind(g, dev_ptr, bytes);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_group_set_config(tamm_group* g, int32_t config, int32_t grid) {
  if (!g) return fail(TAMM_ERR_ARG, "null group");
  if (grid < 0) return fail(TAMM_ERR_ARG, "grid must be >= 0");
  const int rc = group_configure(g, config);
  if (rc != TAMM_OK) return rc;
  for (int c = 0; c < kLayouts; ++c) g->grid[c] = grid;
  return ok();
}

// Persistent grid of one layout class: the tuned size, else every resident slot of the device
// (compute units x resident workgroups of the configuration).
static int group_grid(const tamm_group* g, int layout, int n_work) {
  if (g->grid[layout] > 0) return std::max(1, std::min<int>(g->grid[layout], n_work));
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return std::max(1, std::min<int>(f64_occupancy(g->cfg[layout], layout) * cus, n_work));
}

// The persistent contraction launch of one layout class (counter reset first); nothing for an
// empty class.  Consumes the last screening results.
static int group_enqueue_class(tamm_group* g, int c, hipStream_t s) {
  const int n = g->cls_begin[c + 1] - g->cls_begin[c];
  if (n <= 0) return TAMM_OK;
  const int grid = group_grid(g, c, n);
  int32_t* counter = (int32_t*)(g->ws + g->off_counter) + c;
  HIP_TRY(launch_set_counter(counter, grid, s));
  ContractParams cp{};
  cp.probs = (const ProblemDesc*)(g->ws + g->off_pdesc);
  cp.work = (const WorkItem*)(g->ws + g->off_work) + g->cls_begin[c];
  cp.next_item = counter;
  cp.n_work = n;
  HIP_TRY(launch_contract_f64(g->cfg[c], c, cp, grid, s));
  return TAMM_OK;
}

namespace tamm {

// Enqueue the group's kernels (screening, then per class a counter reset and the persistent
// contraction), consuming the descriptors in the workspace.
int group_enqueue(tamm_group* g, hipStream_t s) {
  ScreenParams sp{};
  sp.probs = (const ScreenDesc*)(g->ws + g->off_sdesc);
  sp.item_prob = (const int32_t*)(g->ws + g->off_sitems);
  sp.item_block = sp.item_prob + g->sitem_prob.size();
  sp.n_items = (int32_t)g->sitem_prob.size();
  HIP_TRY(launch_screen(sp, s));
  // one persistent launch per gather layout present in the group.  With several, they run
  // concurrently: the first on the caller's stream, the others on side streams that wait for the
  // screening and that the caller's stream then waits for, so the workgroups of one class take
  // the compute units the tail of another leaves free (each workgroup only pulls work items
  // from its own class's counter, so no launch waits on another)
  int present[kLayouts], np = 0;
  for (int c = 0; c < kLayouts; ++c)
    if (g->cls_begin[c + 1] > g->cls_begin[c]) present[np++] = c;
  static const bool serial = [] {
    const char* e = getenv("TAMM_GROUP_SERIAL");
    return e && atoi(e) != 0;
  }();
  if (np <= 1 || serial) {
    for (int i = 0; i < np; ++i) {
      const int rc = group_enqueue_class(g, present[i], s);
      if (rc != TAMM_OK) return rc;
    }
    return TAMM_OK;
  }
  if (!g->ev_fork) HIP_TRY(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(g->ev_fork, s));
  for (int i = 1; i < np; ++i) {
    const int c = present[i];
    if (!g->side[c]) HIP_TRY(hipStreamCreateWithFlags(&g->side[c], hipStreamNonBlocking));
    if (!g->ev_join[c]) HIP_TRY(hipEventCreateWithFlags(&g->ev_join[c], hipEventDisableTiming));
    HIP_TRY(hipStreamWaitEvent(g->side[c], g->ev_fork, 0));
    const int rc = group_enqueue_class(g, c, g->side[c]);
    if (rc != TAMM_OK) return rc;
    HIP_TRY(hipEventRecord(g->ev_join[c], g->side[c]));
  }
  const int rc = group_enqueue_class(g, present[0], s);
  if (rc != TAMM_OK) return rc;
  for (int i = 1; i < np; ++i) HIP_TRY(hipStreamWaitEvent(s, g->ev_join[present[i]], 0));
  return TAMM_OK;
}

}  // namespace tamm

static int group_check(tamm_group* g) {
  if (!g->bound) return fail(TAMM_ERR_UNBOUND, "group workspace is not bound (or the configuration changed since binding)");
  for (auto* p : g->plans) {
    int rc = check_tensors(p);
    if (rc != TAMM_OK) return rc;
  }
  // nodes must be independent: no node writes storage that another node reads or writes
  for (size_t i = 0; i < g->nodes.size(); ++i)
    for (size_t j = 0; j < g->nodes.size(); ++j) {
      if (i == j) continue;
      const tamm_tensor* out = g->nodes[i][0]->out;
      for (const tamm_plan* b : g->nodes[j])
        if (overlaps(out, b->out) || overlaps(out, b->lhs) || overlaps(out, b->rhs))
          return fail(TAMM_ERR_ARG, "group members %zu and %zu are not independent (member %zu writes storage member %zu uses)",
                      i, j, i, j);
    }
  return TAMM_OK;
}

namespace tamm {

// Refresh the device descriptors when storage bindings or coefficients changed (after draining
// the stream: earlier launches may still read the old ones).
int group_update_desc(tamm_group* g, const double* alpha, const double* beta, hipStream_t s, bool* changed) {
  std::vector<ScreenDesc> sds;
  std::vector<ProblemDesc> pds;
  group_descs(g, g->ws, alpha, beta, sds, pds);
  const bool sc = memcmp(sds.data(), g->sdesc.data(), sds.size() * sizeof(ScreenDesc)) != 0;
  const bool pc = memcmp(pds.data(), g->pdesc.data(), pds.size() * sizeof(ProblemDesc)) != 0;
  *changed = sc || pc;
  if (*changed) {
    HIP_TRY(hipStreamSynchronize(s));
    if (sc) HIP_TRY(hipMemcpy(g->ws + g->off_sdesc, sds.data(), sds.size() * sizeof(ScreenDesc), hipMemcpyHostToDevice));
    if (pc) HIP_TRY(hipMemcpy(g->ws + g->off_pdesc, pds.data(), pds.size() * sizeof(ProblemDesc), hipMemcpyHostToDevice));
    g->sdesc.swap(sds);
    g->pdesc.swap(pds);
  }
  return TAMM_OK;
}

int group_check_bound(tamm_group* g) { return group_check(g); }
size_t group_node_count(const tamm_group* g) { return g->nodes.size(); }

}  // namespace tamm

// Whether the descriptors in the workspace match the current bindings and these coefficients.
static bool group_desc_current(const tamm_group* g, const double* alpha, const double* beta) {
  std::vector<ScreenDesc> sds;
  std::vector<ProblemDesc> pds;
  group_descs(g, g->ws, alpha, beta, sds, pds);
  return memcmp(sds.data(), g->sdesc.data(), sds.size() * sizeof(ScreenDesc)) == 0 &&
         memcmp(pds.data(), g->pdesc.data(), pds.size() * sizeof(ProblemDesc)) == 0;
}

extern "C" int tamm_group_execute(tamm_group* g, const double* alpha, const double* beta, void* stream) {
  if (!g || !alpha || !beta) return fail(TAMM_ERR_ARG, "null argument");
  int rc = group_check(g);
  if (rc != TAMM_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  bool changed = false;
  if (g->exec) {
    const size_t n = g->nodes.size();
    const bool same = std::equal(alpha, alpha + n, g->g_alpha.begin()) && std::equal(beta, beta + n, g->g_beta.begin());
    if (same && group_desc_current(g, alpha, beta)) {  // the captured graph used these descriptors
      HIP_TRY(hipGraphLaunch(g->exec, s));
      return ok();
    }
    group_drop_graph(g);
  }
  // eager path: descriptor refresh when something changed (after the stream drained, so that
  // earlier launches that read the old descriptors are finished), then the launches
  rc = group_update_desc(g, alpha, beta, s, &changed);
  if (rc != TAMM_OK) return rc;
  rc = group_enqueue(g, s);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_group_capture(tamm_group* g, const double* alpha, const double* beta, void* stream) {
  if (!g || !alpha || !beta) return fail(TAMM_ERR_ARG, "null argument");
  int rc = group_check(g);
  if (rc != TAMM_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  bool changed = false;
  rc = group_update_desc(g, alpha, beta, s, &changed);
  if (rc != TAMM_OK) return rc;
  group_drop_graph(g);
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(TAMM_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  rc = group_enqueue(g, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc != TAMM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(TAMM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(TAMM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  g->graph = graph;
  g->exec = exec;
  g->g_alpha.assign(alpha, alpha + g->nodes.size());
  g->g_beta.assign(beta, beta + g->nodes.size());
  return ok();
}

namespace tamm {

// Autotuner of a group (see tamm_group_autotune): per gather layout class, the fastest
// (configuration, grid) of the class's own launch, timed with alpha = 0, beta = 1.
int group_autotune(tamm_group* g, hipStream_t s, const char* cache_path, int32_t reps) {
  int rc = group_check(g);
  if (rc != TAMM_OK) return rc;
  void* ws = g->ws;
  const size_t bytes = g->ws_bytes;
  CacheEntry best[kLayouts];
  char tag[kLayouts][16];
  bool cached = true;
  for (int c = 0; c < kLayouts; ++c) {
    best[c] = CacheEntry{-1, 1, 0, 1e30};
    snprintf(tag[c], sizeof(tag[c]), "group%d", c);
    cached = cache_lookup(cache_path, g->signature, tag[c], best[c]) && cached;
  }
  if (!cached) {
    if (reps <= 0) reps = 3;
    for (int c = 0; c < kLayouts; ++c) best[c] = CacheEntry{-1, 1, 0, 1e30};
    std::vector<double> a0(g->nodes.size(), 0.0), b1(g->nodes.size(), 1.0);
    TimerEvents ev;
    if ((rc = ev.create()) != TAMM_OK) return rc;
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int k = 0; k < f64_config_count() && rc == TAMM_OK; ++k) {
      for (int mult : {0, 1, 2, 4}) {  // 0: every resident slot (occupancy-sized grid)
        if (rc != TAMM_OK) break;  // a failed launch ends the search with its error
        if ((rc = group_configure(g, k)) != TAMM_OK) break;
        if (g->ws_size > bytes) continue;
        for (int c = 0; c < kLayouts; ++c) g->grid[c] = mult * cus;
        if ((rc = group_bind(g, ws, bytes)) != TAMM_OK) break;
        // screening and a warm-up; alpha = 0, beta = 1 leaves every output unchanged (finite
        // operands), and the classes' launches below reuse that screening
        bool changed = false;
        if ((rc = group_update_desc(g, a0.data(), b1.data(), s, &changed)) != TAMM_OK) break;
        if ((rc = group_enqueue(g, s)) != TAMM_OK) break;
        for (int c = 0; c < kLayouts && rc == TAMM_OK; ++c) {
          if (g->cls_begin[c + 1] == g->cls_begin[c]) continue;
          HIP_TRY(hipEventRecord(e0, s));
          for (int r = 0; r < reps && rc == TAMM_OK; ++r) rc = group_enqueue_class(g, c, s);
          HIP_TRY(hipEventRecord(e1, s));
          HIP_TRY(hipEventSynchronize(e1));
          float ms = 0;
          HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
          ms /= reps;
          if (ms < best[c].ms) best[c] = CacheEntry{k, 1, mult * cus, ms};
        }
      }
    }
    if (rc != TAMM_OK) return rc;
    for (int c = 0; c < kLayouts; ++c)
      if (g->cls_begin[c + 1] != g->cls_begin[c] && best[c].config < 0)
        return fail(TAMM_ERR_WORKSPACE, "no configuration fits the bound workspace");
    for (int c = 0; c < kLayouts; ++c) cache_store(cache_path, g->signature, tag[c], best[c]);
  }
  int cfgs[kLayouts];
  for (int c = 0; c < kLayouts; ++c) cfgs[c] = best[c].config;  // < 0 (empty class): default
  rc = group_configure_classes(g, cfgs);
  if (rc != TAMM_OK) return rc;
  for (int c = 0; c < kLayouts; ++c) g->grid[c] = best[c].config >= 0 ? best[c].grid : 0;
  if (g->ws_size > bytes) return fail(TAMM_ERR_WORKSPACE, "cached configuration needs %zu bytes", g->ws_size);
  return group_bind(g, ws, bytes);
}

size_t group_workspace_size(const tamm_group* g) { return g->ws_size; }

// The largest workspace any configuration of the group needs (the autotuner's candidates).
size_t group_autotune_workspace_size(tamm_group* g) {
  size_t best = g->ws_size;
  int cfgs[kLayouts];
  for (int c = 0; c < kLayouts; ++c) cfgs[c] = g->cfg[c];
  for (int k = 0; k < f64_config_count(); ++k)
    if (group_configure(g, k) == TAMM_OK) best = std::max(best, g->ws_size);
  (void)group_configure_classes(g, cfgs);
  return best;
}

int group_bind_ws(tamm_group* g, void* ws, size_t bytes) { return group_bind(g, ws, bytes); }

}  // namespace tamm

extern "C" int tamm_group_autotune(tamm_group* g, void* stream, const char* cache_path, int32_t reps) {
  if (!g) return fail(TAMM_ERR_ARG, "null group");
  const int rc = group_autotune(g, (hipStream_t)stream, cache_path, reps);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_group_stats(const tamm_group* g, int32_t* config, int32_t* grid, int64_t* work_items) {
  if (!g) return fail(TAMM_ERR_ARG, "null group");
  // the class with the most work items speaks for the group
  int big = 0;
  for (int c = 1; c < kLayouts; ++c)
    if (g->cls_begin[c + 1] - g->cls_begin[c] > g->cls_begin[big + 1] - g->cls_begin[big]) big = c;
  if (config) *config = g->cfg[big];
  if (grid) *grid = g->grid[big];
  if (work_items) *work_items = (int64_t)g->work.size();
  return ok();
}

extern "C" int tamm_group_destroy(tamm_group* g) {
  if (g) {
    group_drop_graph(g);
    for (int c = 0; c < kLayouts; ++c) {
      if (g->side[c]) (void)hipStreamDestroy(g->side[c]);
      if (g->ev_join[c]) (void)hipEventDestroy(g->ev_join[c]);
    }
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  }
  delete g;
  return ok();
}

namespace tamm {

void plan_io(const tamm_plan* p, tamm_tensor** out, const tamm_tensor** lhs, const tamm_tensor** rhs, int* precision) {
  *out = p->out;
  *lhs = p->lhs;
  *rhs = p->rhs;
  *precision = p->prec;
}

bool plans_fusable(tamm_plan* a, tamm_plan* b) {
  const std::vector<tamm_plan*> node{a, b};
  return a->prec == TAMM_PREC_F64 && b->prec == TAMM_PREC_F64 && check_fusable(node) == TAMM_OK;
}

}  // namespace tamm
