// Host side of the C ABI, part 5: the scheduler.  Operations are queued (SetOp, AddOp, MultOp and
// the denominator update), then analysed once: contractions that only accumulate into the output
// of the previous contraction are fused with it into one node (their pairs share output tiles),
// and so are AddOps that only accumulate into the output of the previous AddOp (one launch reads
// and writes that output once for all of them); a dataflow analysis over the tensors each node
// reads and writes assigns every node to the first level after all the nodes it conflicts with,
// and each level runs as one grouped launch of its contraction nodes plus its element-wise
// nodes.  The whole schedule can be captured into one hipGraph and replayed.
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "host.h"

using namespace tamm;

namespace {

enum OpKind { OP_SET, OP_ADD, OP_CONTRACT, OP_DENOM };

struct Op {
  OpKind kind;
  double alpha = 1.0, beta = 0.0;
  tamm_tensor* out = nullptr;
  std::vector<const tamm_tensor*> reads;  // tensors read (out included when beta != 0)
  tamm_plan* plan = nullptr;
  tamm_add* add = nullptr;
  tamm_denominator* den = nullptr;
  std::vector<const double*> energy;
  int node = -1;
};

struct Node {
  std::vector<int> ops;  // queued operations, in queue order (several: a fused contraction or AddOp chain)
  int level = -1;
  int add_ydim = -1;               // AddOp chain: out dimension of its transposed terms' last label
  bool add_plane = false;          // AddOp chain: whole planes per work item
  std::vector<AddItem> add_items;  // AddOp chain: work items, uploaded at bind time
  size_t items_off = 0;
};

struct Level {
  std::vector<int> contract_nodes;  // nodes run as one group
  std::vector<int> elem_nodes;      // element-wise nodes, queue order
  tamm_group* group = nullptr;
  std::vector<double> alpha, beta;  // per group node
  size_t ws_off = 0, ws_size = 0;
};

bool same_storage(const tamm_tensor* a, const tamm_tensor* b) {
  if (a == b) return true;
  if (!a->bound || !b->bound || a->numel == 0 || b->numel == 0) return false;
  const char* a0 = (const char*)a->dev;
  const char* b0 = (const char*)b->dev;
  return a0 < b0 + b->numel * 8 && b0 < a0 + a->numel * 8;
}

}  // namespace

struct tamm_sched {
  std::vector<Op> ops;
  std::vector<Node> nodes;
  std::vector<Level> levels;
  bool built = false;
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_size = 0;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> graph_bindings;  // storage of every tensor when the graph was captured
};

static void sched_drop_graph(tamm_sched* s) {
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->exec = nullptr;
  s->graph = nullptr;
}

static void sched_free(tamm_sched* s) {
  sched_drop_graph(s);
  for (Level& L : s->levels)
    if (L.group) (void)tamm_group_destroy(L.group);
  s->levels.clear();
}

extern "C" int tamm_sched_create(tamm_sched** out) {
  if (!out) return fail(TAMM_ERR_ARG, "null output pointer");
  *out = new tamm_sched();
  return ok();
}

static int queue(tamm_sched* s, Op op) {
  if (s->built) return fail(TAMM_ERR_ARG, "the schedule is built; no operation can be queued any more");
  s->ops.push_back(std::move(op));
  return ok();
}

extern "C" int tamm_sched_set(tamm_sched* s, tamm_tensor* out, double alpha) {
  if (!s || !out) return fail(TAMM_ERR_ARG, "null argument");
  Op op{OP_SET};
  op.alpha = alpha;
  op.out = out;
  return queue(s, std::move(op));
}

extern "C" int tamm_sched_add(tamm_sched* s, tamm_add* a, double alpha, double beta) {
  if (!s || !a) return fail(TAMM_ERR_ARG, "null argument");
  Op op{OP_ADD};
  op.alpha = alpha;
  op.beta = beta;
  op.add = a;
  op.out = const_cast<tamm_tensor*>(add_out(a));
  op.reads.push_back(add_in(a));
  if (beta != 0.0) op.reads.push_back(op.out);
  return queue(s, std::move(op));
}

extern "C" int tamm_sched_contract(tamm_sched* s, tamm_plan* p, double alpha, double beta) {
  if (!s || !p) return fail(TAMM_ERR_ARG, "null argument");
  Op op{OP_CONTRACT};
  op.alpha = alpha;
  op.beta = beta;
  op.plan = p;
  const tamm_tensor *lhs, *rhs;
  int prec = 0;
  plan_io(p, &op.out, &lhs, &rhs, &prec);
  if (prec != TAMM_PREC_F64) return fail(TAMM_ERR_UNSUPPORTED, "the scheduler runs float64 contractions");
  op.reads = {lhs, rhs};
  if (beta != 0.0) op.reads.push_back(op.out);
  return queue(s, std::move(op));
}

extern "C" int tamm_sched_denominator(tamm_sched* s, tamm_denominator* d, const double* const* energy) {
  if (!s || !d || !energy) return fail(TAMM_ERR_ARG, "null argument");
  Op op{OP_DENOM};
  op.den = d;
  const tamm_tensor* in;
  denominator_io(d, &op.out, &in);
  op.reads.push_back(in);
  op.energy.assign(energy, energy + op.out->rank);
  return queue(s, std::move(op));
}

// Reads and writes of a node (the union over its operations).
static void node_io(const tamm_sched* s, const Node& n, std::vector<const tamm_tensor*>& r, std::vector<const tamm_tensor*>& w) {
  r.clear();
  w.clear();
  for (int i : n.ops) {
    const Op& op = s->ops[i];
    w.push_back(op.out);
    r.insert(r.end(), op.reads.begin(), op.reads.end());
  }
}

static bool touches(const std::vector<const tamm_tensor*>& set, const tamm_tensor* t) {
  for (const tamm_tensor* x : set)
    if (same_storage(x, t)) return true;
  return false;
}

static bool conflict(const tamm_sched* s, const Node& a, const Node& b) {
  std::vector<const tamm_tensor*> ra, wa, rb, wb;
  node_io(s, a, ra, wa);
  node_io(s, b, rb, wb);
  for (const tamm_tensor* t : wa)
    if (touches(rb, t) || touches(wb, t)) return true;
  for (const tamm_tensor* t : wb)
    if (touches(ra, t)) return true;
  return false;
}

extern "C" int tamm_sched_build(tamm_sched* s) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  if (s->built) return fail(TAMM_ERR_ARG, "the schedule is already built");
  if (s->ops.empty()) return fail(TAMM_ERR_ARG, "the schedule has no operation");
  // ---- fusion: a contraction that accumulates (beta = 1) into the output of the contraction
  // chain that last touched that output joins the chain when it has the same alpha, the plans
  // can share output tiles, and no operation queued in between writes what the chain reads
  std::vector<int> chain_of(s->ops.size(), -1);
  for (size_t j = 0; j < s->ops.size(); ++j) {
    Op& op = s->ops[j];
    if (op.kind == OP_CONTRACT && op.beta == 1.0) {
      int last = -1;  // last earlier operation touching op.out
      for (int k = (int)j - 1; k >= 0 && last < 0; --k) {
        const Op& o = s->ops[k];
        if (same_storage(o.out, op.out) || touches(o.reads, op.out)) last = k;
      }
      if (last >= 0 && s->ops[last].kind == OP_CONTRACT && s->ops[last].out == op.out && s->ops[last].alpha == op.alpha) {
        const int head_node = chain_of[last];
        Node& chain = s->nodes[head_node];
        bool ok_fuse = plans_fusable(s->ops[chain.ops[0]].plan, op.plan);
        std::vector<const tamm_tensor*> cr, cw;
        node_io(s, chain, cr, cw);
        for (int k = chain.ops[0] + 1; k < (int)j && ok_fuse; ++k) {
          if (chain_of[k] == head_node) continue;
          if (touches(cr, s->ops[k].out)) ok_fuse = false;
        }
        if (ok_fuse) {
          chain.ops.push_back((int)j);
          chain_of[j] = head_node;
          continue;
        }
      }
    }
    if (op.kind == OP_ADD && op.beta == 1.0) {
      int last = -1;  // last earlier operation touching op.out
      for (int k = (int)j - 1; k >= 0 && last < 0; --k) {
        const Op& o = s->ops[k];
        if (same_storage(o.out, op.out) || touches(o.reads, op.out)) last = k;
      }
      if (last >= 0 && s->ops[last].kind == OP_ADD && s->ops[last].out == op.out) {
        const int head_node = chain_of[last];
        Node& chain = s->nodes[head_node];
        const tamm_add* head = s->ops[chain.ops[0]].add;
        int ydim = chain.add_ydim;
        bool ok_fuse = (int)chain.ops.size() < kMaxAddTerms;
        if (ok_fuse && chain.ops.size() == 1) ok_fuse = add_chain_accepts(head, head, &ydim);
        ok_fuse = ok_fuse && add_chain_accepts(head, op.add, &ydim);
        std::vector<const tamm_tensor*> cr, cw;
        node_io(s, chain, cr, cw);
        for (int k = chain.ops[0] + 1; k < (int)j && ok_fuse; ++k) {
          if (chain_of[k] == head_node) continue;
          if (touches(cr, s->ops[k].out)) ok_fuse = false;
        }
        if (ok_fuse) {
          chain.ops.push_back((int)j);
          chain.add_ydim = ydim;
          chain_of[j] = head_node;
          continue;
        }
      }
    }
    chain_of[j] = (int)s->nodes.size();
    s->nodes.push_back(Node{{(int)j}, -1});
  }
  // ---- levels: nodes in the order of their last operation; each goes one level after the
  // latest earlier node it conflicts with (shares a tensor that one of the two writes)
  std::vector<int> order(s->nodes.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return s->nodes[a].ops.back() < s->nodes[b].ops.back(); });
  int nlev = 0;
  for (size_t x = 0; x < order.size(); ++x) {
    Node& n = s->nodes[order[x]];
    int lev = 0;
    for (size_t y = 0; y < x; ++y) {
      const Node& m = s->nodes[order[y]];
      if (conflict(s, m, n)) lev = std::max(lev, m.level + 1);
    }
    n.level = lev;
    nlev = std::max(nlev, lev + 1);
    for (int i : n.ops) s->ops[i].node = order[x];
  }
  s->levels.assign(nlev, Level{});
  for (size_t x = 0; x < order.size(); ++x) {
    const Node& n = s->nodes[order[x]];
    Level& L = s->levels[n.level];
    if (s->ops[n.ops[0]].kind == OP_CONTRACT) L.contract_nodes.push_back(order[x]);
    else L.elem_nodes.push_back(order[x]);
  }
  // ---- one group per level with contractions; workspace regions sized for the autotuner
  size_t off = 0;
  for (Level& L : s->levels) {
    if (L.contract_nodes.empty()) continue;
    std::vector<std::vector<tamm_plan*>> gn;
    for (int q : L.contract_nodes) {
      std::vector<tamm_plan*> members;
      for (int i : s->nodes[q].ops) members.push_back(s->ops[i].plan);
      gn.push_back(members);
      L.alpha.push_back(s->ops[s->nodes[q].ops[0]].alpha);
      L.beta.push_back(s->ops[s->nodes[q].ops[0]].beta);
    }
    const int rc = group_create_nodes(gn, &L.group);
    if (rc != TAMM_OK) {
      sched_free(s);
      s->nodes.clear();
      return rc;
    }
    L.ws_off = align256(off);
    L.ws_size = group_autotune_workspace_size(L.group);
    off = L.ws_off + L.ws_size;
  }
  // ---- AddOp chains: work items over the (ydim, last) plane (ydim: rank - 2 when every term
  // reads directly), in their own workspace regions
  for (Node& n : s->nodes) {
    if (n.ops.size() < 2 || s->ops[n.ops[0]].kind != OP_ADD) continue;
    std::vector<const tamm_add*> m;
    for (int i : n.ops) m.push_back(s->ops[i].add);
    if (n.add_ydim < 0) n.add_ydim = add_out(m[0])->rank - 2;
    const int rc = add_chain_items(m, n.add_ydim, n.add_items, &n.add_plane);
    if (rc != TAMM_OK) {
      sched_free(s);
      s->nodes.clear();
      return rc;
    }
    n.items_off = align256(off);
    off = n.items_off + n.add_items.size() * sizeof(AddItem);
  }
  s->ws_size = std::max<size_t>(align256(off), 256);
  s->built = true;
  return ok();
}

extern "C" int tamm_sched_workspace_size(const tamm_sched* s, size_t* bytes) {
  if (!s || !bytes) return fail(TAMM_ERR_ARG, "null argument");
  if (!s->built) return fail(TAMM_ERR_ARG, "the schedule is not built");
  *bytes = s->ws_size;
  return ok();
}

extern "C" int tamm_sched_bind_workspace(tamm_sched* s, void* ws, size_t bytes) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  if (!s->built) return fail(TAMM_ERR_ARG, "the schedule is not built");
  if (!ws || ((uintptr_t)ws) % 256 || bytes < s->ws_size)
    return fail(TAMM_ERR_WORKSPACE, "workspace must be 256-byte aligned and at least %zu bytes", s->ws_size);
  sched_drop_graph(s);
  for (Level& L : s->levels) {
    if (!L.group) continue;
    const int rc = group_bind_ws(L.group, (char*)ws + L.ws_off, L.ws_size);
    if (rc != TAMM_OK) return rc;
  }
  for (const Node& n : s->nodes)
    if (!n.add_items.empty())
      HIP_TRY(hipMemcpy((char*)ws + n.items_off, n.add_items.data(), n.add_items.size() * sizeof(AddItem),
                        hipMemcpyHostToDevice));
  s->ws = (char*)ws;
  s->ws_bytes = bytes;
  s->bound = true;
  return ok();
}

// Storage of every tensor the schedule touches (a captured graph is valid only for these).
static std::vector<const void*> bindings(const tamm_sched* s) {
  std::vector<const void*> b;
  for (const Op& op : s->ops) {
    b.push_back(op.out->dev);
    for (const tamm_tensor* t : op.reads) b.push_back(t->dev);
    for (const double* e : op.energy) b.push_back(e);
  }
  return b;
}

static int sched_check(tamm_sched* s) {
  if (!s->built || !s->bound) return fail(TAMM_ERR_UNBOUND, "the schedule is not built and bound");
  for (const Op& op : s->ops) {
    if (!op.out->bound) return fail(TAMM_ERR_UNBOUND, "a tensor of the schedule has no storage");
    for (const tamm_tensor* t : op.reads)
      if (!t->bound) return fail(TAMM_ERR_UNBOUND, "a tensor of the schedule has no storage");
  }
  for (Level& L : s->levels)
    if (L.group) {
      const int rc = group_check_bound(L.group);
      if (rc != TAMM_OK) return rc;
    }
  return TAMM_OK;
}

// Descriptors of every level's group for the current bindings (synchronises when they change).
static int sched_update(tamm_sched* s, hipStream_t st) {
  for (Level& L : s->levels)
    if (L.group) {
      bool changed = false;
      const int rc = group_update_desc(L.group, L.alpha.data(), L.beta.data(), st, &changed);
      if (rc != TAMM_OK) return rc;
    }
  return TAMM_OK;
}

static int sched_enqueue(tamm_sched* s, hipStream_t st) {
  for (Level& L : s->levels) {
    if (L.group) {
      const int rc = group_enqueue(L.group, st);
      if (rc != TAMM_OK) return rc;
    }
    for (int q : L.elem_nodes) {
      const Node& n = s->nodes[q];
      if (n.ops.size() > 1) {  // AddOp chain: the head's beta, then every member's term
        std::vector<tamm_add*> m;
        std::vector<double> alpha;
        for (int i : n.ops) {
          m.push_back(s->ops[i].add);
          alpha.push_back(s->ops[i].alpha);
        }
        const int rc = add_chain_enqueue(m, alpha, s->ops[n.ops[0]].beta, n.add_ydim, n.add_plane,
                                         (const AddItem*)(s->ws + n.items_off), (int64_t)n.add_items.size(), st);
        if (rc != TAMM_OK) return rc;
        continue;
      }
      const Op& op = s->ops[n.ops[0]];
      int rc = TAMM_OK;
      switch (op.kind) {
        case OP_SET:
          HIP_TRY(launch_fill(op.out->dev, op.out->numel, op.alpha, st));
          break;
        case OP_ADD: rc = add_enqueue(op.add, op.alpha, op.beta, st); break;
        case OP_DENOM: rc = denominator_enqueue(op.den, op.energy.data(), st); break;
        default: rc = fail(TAMM_ERR_ARG, "unexpected operation");
      }
      if (rc != TAMM_OK) return rc;
    }
  }
  return TAMM_OK;
}

extern "C" int tamm_sched_execute(tamm_sched* s, void* stream) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  int rc = sched_check(s);
  if (rc != TAMM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (s->exec) {
    if (bindings(s) == s->graph_bindings) {
      HIP_TRY(hipGraphLaunch(s->exec, st));
      return ok();
    }
    sched_drop_graph(s);
  }
  rc = sched_update(s, st);
  if (rc == TAMM_OK) rc = sched_enqueue(s, st);
  return rc == TAMM_OK ? ok() : rc;
}

extern "C" int tamm_sched_capture(tamm_sched* s, void* stream) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  int rc = sched_check(s);
  if (rc != TAMM_OK) return rc;
  rc = sched_update(s, (hipStream_t)stream);
  if (rc != TAMM_OK) return rc;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  sched_drop_graph(s);
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(TAMM_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  rc = sched_enqueue(s, cs);
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
  s->graph = graph;
  s->exec = exec;
  s->graph_bindings = bindings(s);
  return ok();
}

extern "C" int tamm_sched_autotune(tamm_sched* s, void* stream, const char* cache_path, int32_t reps) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  int rc = sched_check(s);
  if (rc != TAMM_OK) return rc;
  sched_drop_graph(s);
  for (Level& L : s->levels) {
    if (!L.group) continue;
    rc = group_autotune(L.group, (hipStream_t)stream, cache_path, reps);
    if (rc != TAMM_OK) return rc;
  }
  return ok();
}

extern "C" int tamm_sched_info(const tamm_sched* s, int32_t* levels, int32_t* nodes, int32_t* fused_ops) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  if (!s->built) return fail(TAMM_ERR_ARG, "the schedule is not built");
  int32_t f = 0;
  for (const Node& n : s->nodes)
    if (n.ops.size() > 1) f += (int32_t)n.ops.size();
  if (levels) *levels = (int32_t)s->levels.size();
  if (nodes) *nodes = (int32_t)s->nodes.size();
  if (fused_ops) *fused_ops = f;
  return ok();
}

extern "C" int tamm_sched_op_info(const tamm_sched* s, int32_t op, int32_t* level, int32_t* node) {
  if (!s) return fail(TAMM_ERR_ARG, "null schedule");
  if (!s->built) return fail(TAMM_ERR_ARG, "the schedule is not built");
  if (op < 0 || op >= (int32_t)s->ops.size()) return fail(TAMM_ERR_ARG, "operation %d does not exist", op);
  const int n = s->ops[op].node;
  if (level) *level = s->nodes[n].level;
  if (node) *node = n;
  return ok();
}

extern "C" int tamm_sched_destroy(tamm_sched* s) {
  if (s) sched_free(s);
  delete s;
  return ok();
}
