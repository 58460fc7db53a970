// Host side of the C ABI, part 4: the element-wise operations of the operation grammar -- SetOp
// (assign one value to every stored element) and AddOp (add a scaled tensor read through a label
// permutation), prepared once and executed many times.
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "host.h"

using namespace tamm;

struct tamm_add {
  tamm_tensor* out = nullptr;
  const tamm_tensor* in = nullptr;
  bool identity = true;  // in_lbl == out_lbl
  int32_t ydim = -1;     // transpose mode: out dimension of in's last label
  int32_t chunk = 4096;  // direct mode: elements per item
  std::vector<AddBlock> blocks;
  std::vector<AddItem> items;
  size_t off_blocks = 0, off_items = 0, ws_size = 0;
  char* ws = nullptr;
  bool bound = false;
};

extern "C" int tamm_set(tamm_tensor* out, double alpha, void* stream) {
  if (!out) return fail(TAMM_ERR_ARG, "null tensor");
  if (!out->bound) return fail(TAMM_ERR_UNBOUND, "tensor storage not bound");
  HIP_TRY(launch_fill(out->dev, out->numel, alpha, (hipStream_t)stream));
  return ok();
}

extern "C" int tamm_add_create(tamm_tensor* out, const char* out_lbl, const tamm_tensor* in, const char* in_lbl,
                               tamm_add** ap) {
  if (!ap) return fail(TAMM_ERR_ARG, "null output pointer");
  *ap = nullptr;
  if (!out || !in || !out_lbl || !in_lbl) return fail(TAMM_ERR_ARG, "null tensor or label string");
  const int r = out->rank;
  if ((int)strlen(out_lbl) != r || (int)strlen(in_lbl) != in->rank || in->rank != r)
    return fail(TAMM_ERR_SHAPE, "label strings must have one letter per dimension and both tensors the same rank");
  // in_lbl must be a permutation of out_lbl; perm[d] = in dimension of out dimension d
  int perm[kMaxRank];
  for (int d = 0; d < r; ++d) {
    const char c = out_lbl[d];
    if (!((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'))) return fail(TAMM_ERR_LABEL, "label '%c' is not a letter", c);
    for (int e = 0; e < d; ++e)
      if (out_lbl[e] == c) return fail(TAMM_ERR_LABEL, "label '%c' repeats inside '%s'", c, out_lbl);
    const char* q = strchr(in_lbl, c);
    if (!q) return fail(TAMM_ERR_LABEL, "label '%c' of out does not appear in '%s'", c, in_lbl);
    perm[d] = (int)(q - in_lbl);
    if (!out->dims[d]->same(*in->dims[perm[d]])) return fail(TAMM_ERR_LABEL, "label '%c' binds two different tiled spaces", c);
  }
  for (int d = 0; d < r; ++d)
    for (int e = 0; e < d; ++e)
      if (perm[d] == perm[e]) return fail(TAMM_ERR_LABEL, "'%s' is not a permutation of '%s'", in_lbl, out_lbl);
  auto a = std::make_unique<tamm_add>();
  a->out = out;
  a->in = in;
  for (int d = 0; d < r; ++d) a->identity = a->identity && perm[d] == d;
  const int in_last = in->rank - 1;
  for (int d = 0; d < r; ++d)
    if (perm[d] == in_last && d != r - 1) a->ydim = d;
  const int nob = (int)out->block_off.size();
  std::vector<int32_t> ot(r);
  for (int b = 0; b < nob; ++b) {
    AddBlock B{};
    B.out_off = out->block_off[b];
    int64_t in_lin = 0, n = 1;
    int64_t in_ext[kMaxRank];
    for (int d = 0; d < r; ++d) {
      ot[d] = out->block_tiles[(size_t)b * r + d];
      B.ext[d] = (int32_t)out->dims[d]->size[ot[d]];
      n *= B.ext[d];
      in_ext[perm[d]] = B.ext[d];
      in_lin += (int64_t)ot[d] * in->tstride[perm[d]];
    }
    if (n > INT32_MAX) return fail(TAMM_ERR_UNSUPPORTED, "block %d has more than 2^31 elements", b);
    int64_t in_stride[kMaxRank], s = 1;
    for (int e = r - 1; e >= 0; --e) {
      in_stride[e] = s;
      s *= in_ext[e];
    }
    for (int d = 0; d < r; ++d) B.istr[d] = (int32_t)in_stride[perm[d]];
    B.in_off = in->tile_off[in_lin];
    a->blocks.push_back(B);
    if (a->ydim < 0) {
      for (int64_t e = 0; e < n; e += a->chunk) a->items.push_back(AddItem{b, (int32_t)e, 0, 0});
    } else {
      const int ey = B.ext[a->ydim], ex = B.ext[r - 1];
      const int64_t nbatch = n / ((int64_t)ey * ex);
      for (int64_t t = 0; t < nbatch; ++t)
        for (int y = 0; y < ey; y += 32)
          for (int x = 0; x < ex; x += 32) a->items.push_back(AddItem{b, (int32_t)t, y, x});
    }
    if (a->items.size() > (size_t)INT32_MAX) return fail(TAMM_ERR_UNSUPPORTED, "too many work items");
  }
  size_t off = 0;
  a->off_blocks = off;
  off = align256(off + a->blocks.size() * sizeof(AddBlock));
  a->off_items = off;
  off = align256(off + a->items.size() * sizeof(AddItem));
  a->ws_size = std::max<size_t>(off, 256);
  *ap = a.release();
  return ok();
}

extern "C" int tamm_add_workspace_size(const tamm_add* a, size_t* bytes) {
  if (!a || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  *bytes = a->ws_size;
  return ok();
}

extern "C" int tamm_add_bind_workspace(tamm_add* a, void* workspace, size_t bytes) {
  if (!a) return fail(TAMM_ERR_ARG, "null argument");
  if (!workspace || ((uintptr_t)workspace) % 256 || bytes < a->ws_size)
    return fail(TAMM_ERR_WORKSPACE, "workspace must be 256-byte aligned and at least %zu bytes", a->ws_size);
  char* ws = (char*)workspace;
  if (!a->blocks.empty())
    HIP_TRY(hipMemcpy(ws + a->off_blocks, a->blocks.data(), a->blocks.size() * sizeof(AddBlock), hipMemcpyHostToDevice));
  if (!a->items.empty())
    HIP_TRY(hipMemcpy(ws + a->off_items, a->items.data(), a->items.size() * sizeof(AddItem), hipMemcpyHostToDevice));
  a->ws = ws;
  a->bound = true;
  return ok();
}

namespace tamm {

// Enqueue an AddOp (used by tamm_add_execute and the scheduler).
int add_enqueue(tamm_add* a, double alpha, double beta, hipStream_t s) {
  if (!a->bound) return fail(TAMM_ERR_UNBOUND, "AddOp workspace is not bound");
  if (!a->out->bound || !a->in->bound) return fail(TAMM_ERR_UNBOUND, "tensor storage not bound");
  const char* o0 = (const char*)a->out->dev;
  const char* i0 = (const char*)a->in->dev;
  const bool overlap = a->out->numel > 0 && a->in->numel > 0 && o0 < i0 + a->in->numel * 8 && i0 < o0 + a->out->numel * 8;
  if (overlap && !(a->identity && o0 == i0))
    return fail(TAMM_ERR_ARG, "out storage overlaps in (allowed only as the same storage with identical labels)");
  AddParams p{};
  p.out = a->out->dev;
  p.in = a->in->dev;
  p.blocks = (const AddBlock*)(a->ws + a->off_blocks);
  p.items = (const AddItem*)(a->ws + a->off_items);
  p.n_items = (int64_t)a->items.size();
  p.alpha = alpha;
  p.beta = beta;
  p.rank = a->out->rank;
  p.ydim = a->ydim;
  p.chunk = a->chunk;
  HIP_TRY(launch_add(p, s));
  return TAMM_OK;
}

const tamm_tensor* add_out(const tamm_add* a) { return a->out; }
const tamm_tensor* add_in(const tamm_add* a) { return a->in; }

// True when AddOp b can join a chain of AddOps into the same out whose transposed terms read
// through out dimension *ydim (-1: none so far): same out tensor, rank >= 2, in storage apart from
// out, and b's in ending in out's last label or in label *ydim.  Updates *ydim.
bool add_chain_accepts(const tamm_add* head, const tamm_add* b, int* ydim) {
  if (b->out != head->out || b->out->rank < 2) return false;
  if (b->out->bound && b->in->bound && b->out->numel > 0 && b->in->numel > 0) {
    const char* o0 = (const char*)b->out->dev;
    const char* i0 = (const char*)b->in->dev;
    if (o0 < i0 + b->in->numel * 8 && i0 < o0 + b->out->numel * 8) return false;
  } else if ((const void*)b->in == (const void*)b->out) {
    return false;
  }
  if (b->ydim < 0) return true;
  if (*ydim >= 0 && *ydim != b->ydim) return false;
  *ydim = b->ydim;
  return true;
}

// Work items of a chain: whole planes of out's last two dimensions when ydim is the
// second-to-last, every block's plane holds at most kAddPlaneMax elements and lies contiguous in
// every member's input (*plane = true); otherwise 32 x 32 tiles of the (ydim, last) plane.
int add_chain_items(const std::vector<const tamm_add*>& m, int ydim, std::vector<AddItem>& items, bool* plane) {
  const tamm_add* head = m[0];
  const int r = head->out->rank;
  bool pl = ydim == r - 2;
  for (size_t b = 0; b < head->blocks.size() && pl; ++b) {
    const int ey = head->blocks[b].ext[r - 2], ex = head->blocks[b].ext[r - 1];
    if ((int64_t)ey * ex > kAddPlaneMax) pl = false;
    for (const tamm_add* a : m) {
      const AddBlock& B = a->blocks[b];
      const bool contiguous = a->ydim < 0 ? (B.istr[r - 1] == 1 && B.istr[r - 2] == ex)
                                          : (B.istr[r - 2] == 1 && B.istr[r - 1] == ey);
      pl = pl && contiguous;
    }
  }
  *plane = pl;
  items.clear();
  for (size_t b = 0; b < head->blocks.size(); ++b) {
    const AddBlock& B = head->blocks[b];
    int64_t n = 1;
    for (int d = 0; d < r; ++d) n *= B.ext[d];
    const int ey = B.ext[ydim], ex = B.ext[r - 1];
    const int64_t nbatch = n / ((int64_t)ey * ex);
    for (int64_t t = 0; t < nbatch; ++t) {
      if (pl) {
        items.push_back(AddItem{(int32_t)b, (int32_t)t, 0, 0});
        continue;
      }
      for (int y = 0; y < ey; y += 32)
        for (int x = 0; x < ex; x += 32) items.push_back(AddItem{(int32_t)b, (int32_t)t, y, x});
    }
    if (items.size() > (size_t)INT32_MAX) return fail(TAMM_ERR_UNSUPPORTED, "too many work items");
  }
  return TAMM_OK;
}

// Enqueue a chain: out = beta*out + sum_t alpha[t]*in_t (items from add_chain_items, on device).
int add_chain_enqueue(const std::vector<tamm_add*>& m, const std::vector<double>& alpha, double beta, int ydim,
                      bool plane, const AddItem* items, int64_t n_items, hipStream_t s) {
  if (m.empty() || m.size() > (size_t)kMaxAddTerms || alpha.size() != m.size())
    return fail(TAMM_ERR_ARG, "an AddOp chain has 1 to %d members", kMaxAddTerms);
  AddMultiParams p{};
  p.out = m[0]->out->dev;
  for (size_t t = 0; t < m.size(); ++t) {
    const tamm_add* a = m[t];
    if (!a->bound) return fail(TAMM_ERR_UNBOUND, "AddOp workspace is not bound");
    if (!a->out->bound || !a->in->bound) return fail(TAMM_ERR_UNBOUND, "tensor storage not bound");
    const char* o0 = (const char*)a->out->dev;
    const char* i0 = (const char*)a->in->dev;
    if (a->out != m[0]->out || (a->out->numel > 0 && a->in->numel > 0 && o0 < i0 + a->in->numel * 8 && i0 < o0 + a->out->numel * 8))
      return fail(TAMM_ERR_ARG, "an AddOp chain needs one out and inputs apart from it");
    if (a->ydim >= 0 && a->ydim != ydim) return fail(TAMM_ERR_ARG, "AddOp chain member reads through another dimension");
    p.in[t] = a->in->dev;
    p.blocks[t] = (const AddBlock*)(a->ws + a->off_blocks);
    p.alpha[t] = alpha[t];
    p.trans[t] = a->ydim >= 0 ? 1 : 0;
  }
  p.items = items;
  p.n_items = n_items;
  p.beta = beta;
  p.rank = m[0]->out->rank;
  p.ydim = ydim;
  p.nterms = (int32_t)m.size();
  p.plane = plane ? 1 : 0;
  if (plane && ydim != p.rank - 2) return fail(TAMM_ERR_ARG, "plane mode needs the last two dimensions");
  HIP_TRY(launch_add_multi(p, s));
  return TAMM_OK;
}

}  // namespace tamm

extern "C" int tamm_add_execute(tamm_add* a, double alpha, double beta, void* stream) {
  if (!a) return fail(TAMM_ERR_ARG, "null argument");
  const int rc = add_enqueue(a, alpha, beta, (hipStream_t)stream);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_add_destroy(tamm_add* a) {
  delete a;
  return ok();
}
