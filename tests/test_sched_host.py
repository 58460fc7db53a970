"""Host-only checks of the scheduler's analysis (Sec. III-A Fig. 4 queue-then-execute; Sec. III-B
dataflow levels): which queued operations fuse into one node and which level each node runs at.
Building a schedule makes no GPU call, so these run without a GPU on structure-only tensors."""

import pytest

from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd.synth import TERMS


def spaces():
    return tm.Space.spin(6, 6, 3), tm.Space.spin(10, 10, 5)


def tensor(o, v, pattern):
    return tm.Tensor([o if c == "o" else v for c in pattern], device=None)


def plan(out, ol, lhs, ll, rhs, rl):
    return tm.Plan(out, ol, lhs, ll, rhs, rl, bind=False)


def doubles_iteration_queue():
    """The doubles-residual iteration as it is queued in the GPU tests (no denominator: that
    needs device memory)."""
    o, v = spaces()
    t = {n: tensor(o, v, p) for n, p in [("V_vvvv", "vvvv"), ("V_ovvo", "ovvo"), ("V_oovv", "oovv"),
                                          ("V_vvvo", "vvvo"), ("V_ovoo", "ovoo"), ("T2", "vvoo"), ("T1", "vo"),
                                          ("W", "oooo"), ("R", "vvoo"), ("X", "vvoo"), ("Zv", "vvoo"),
                                          ("Zo", "vvoo")]}
    s = tm.Scheduler()
    s.contract(plan(t["W"], "mnij", t["V_oovv"], "mnef", t["T2"], "efij"), 0.5, 0.0)    # 0 level 0
    s.contract(plan(t["R"], "abij", t["V_vvvv"], "abcd", t["T2"], "cdij"), 0.5, 0.0)    # 1 fused with 2
    s.contract(plan(t["R"], "abij", t["W"], "mnij", t["T2"], "abmn"), 0.5, 1.0)         # 2 level 1
    s.contract(plan(t["X"], "abij", t["V_ovvo"], "mbej", t["T2"], "aeim"), 1.0, 0.0)    # 3 level 0
    s.contract(plan(t["Zv"], "abij", t["V_vvvo"], "abej", t["T1"], "ei"), 1.0, 0.0)     # 4 level 0
    s.contract(plan(t["Zo"], "abij", t["V_ovoo"], "mbij", t["T1"], "am"), -1.0, 0.0)    # 5 level 0
    adds = [("X", "abij", 1.0), ("X", "abji", -1.0), ("X", "baij", -1.0), ("X", "baji", 1.0),
            ("Zv", "abij", 1.0), ("Zv", "abji", -1.0), ("Zo", "abij", 1.0), ("Zo", "baij", -1.0)]
    for name, lbl, sign in adds:                                                        # 6..13
        s.add(tm.Add(t["R"], "abij", t[name], lbl, bind=False), sign, 1.0)
    return s, t


def test_doubles_iteration_fusion_and_levels():
    s, _ = doubles_iteration_queue()
    s.build()
    info = s.info()
    # ladder + hole-hole ladder share output tiles; the eight AddOps into R form one chain
    assert info["fused_ops"] == 2 + 8
    assert info["nodes"] == 6                     # 14 operations: W, the ladders, X, Zv, Zo, the chain
    lv = [s.op_info(i)[0] for i in range(14)]
    nd = [s.op_info(i)[1] for i in range(14)]
    assert nd[1] == nd[2] and len(set(nd[6:])) == 1 and len(set(nd)) == 6
    assert lv[0] == 0 and lv[3] == 0 and lv[4] == 0 and lv[5] == 0   # independent terms together
    assert lv[1] == lv[2] == 1                    # after W (read by the hole-hole ladder)
    assert lv[6:] == [2] * 8                      # one launch after the ladders wrote R
    assert info["levels"] == 3
    with pytest.raises(tm.TammError):
        s.set(tm.Tensor(list(spaces()), device=None), 1.0)  # no queueing after build


def test_no_fusion_when_alpha_differs_or_inputs_change_in_between():
    o, v = spaces()
    V, T, W, R = tensor(o, v, "vvvv"), tensor(o, v, "vvoo"), tensor(o, v, "oooo"), tensor(o, v, "vvoo")
    Voovv = tensor(o, v, "oovv")
    # different alpha: two nodes in consecutive levels (write-after-write on R)
    s = tm.Scheduler()
    s.contract(plan(R, "abij", V, "abcd", T, "cdij"), 0.5, 0.0)
    s.contract(plan(R, "abij", W, "mnij", T, "abmn"), 0.25, 1.0)
    s.build()
    assert s.info()["fused_ops"] == 0 and [s.op_info(i)[0] for i in range(2)] == [0, 1]
    # an operation in between writes what the first contraction reads (T): no fusion, and the
    # three run in program order
    s = tm.Scheduler()
    s.contract(plan(R, "abij", V, "abcd", T, "cdij"), 0.5, 0.0)
    s.set(T, 1.0)
    s.contract(plan(R, "abij", W, "mnij", T, "abmn"), 0.5, 1.0)
    s.build()
    assert s.info()["fused_ops"] == 0 and [s.op_info(i)[0] for i in range(3)] == [0, 1, 2]
    # an operation in between writes an input of the second one only: fusion, after it
    s = tm.Scheduler()
    s.contract(plan(R, "abij", V, "abcd", T, "cdij"), 0.5, 0.0)
    s.contract(plan(W, "mnij", Voovv, "mnef", T, "efij"), 1.0, 0.0)
    s.contract(plan(R, "abij", W, "mnij", T, "abmn"), 0.5, 1.0)
    s.build()
    assert s.info()["fused_ops"] == 2
    assert [s.op_info(i)[0] for i in range(3)] == [1, 0, 1]


def test_addop_chains_and_where_they_break():
    o, v = spaces()
    R, X, Y, Z = tensor(o, v, "vvoo"), tensor(o, v, "vvoo"), tensor(o, v, "oovv"), tensor(o, v, "vvoo")

    def nodes_levels(s, n):
        s.build()
        return [s.op_info(i)[1] for i in range(n)], [s.op_info(i)[0] for i in range(n)]

    # a head with beta = 0, then accumulating terms read directly (baij) and through the second
    # occupied label (abji, baji): one node
    s = tm.Scheduler()
    for lbl, beta in (("abij", 0.0), ("baij", 1.0), ("abji", 1.0), ("baji", 1.0)):
        s.add(tm.Add(R, "abij", X, lbl, bind=False), 1.0, beta)
    nd, lv = nodes_levels(s, 4)
    assert len(set(nd)) == 1 and lv == [0] * 4 and s.info()["fused_ops"] == 4
    # beta != 1 starts a new chain (whose direct head then takes a term read through out
    # dimension 1); so does a term read through another dimension than the chain's (ijab ends in
    # b, out dimension 1, after abji fixed dimension 2)
    s = tm.Scheduler()
    s.add(tm.Add(R, "abij", X, "abji", bind=False), 1.0, 1.0)
    s.add(tm.Add(R, "abij", X, "abij", bind=False), 1.0, 0.5)
    s.add(tm.Add(R, "abij", Y, "ijab", bind=False), 1.0, 1.0)
    nd, lv = nodes_levels(s, 3)
    assert nd[0] != nd[1] and nd[1] == nd[2] and lv == [0, 1, 1]
    s = tm.Scheduler()
    s.add(tm.Add(R, "abij", X, "abji", bind=False), 1.0, 1.0)
    s.add(tm.Add(R, "abij", Y, "ijab", bind=False), 1.0, 1.0)
    s.add(tm.Add(R, "abij", X, "abij", bind=False), 1.0, 1.0)
    nd, lv = nodes_levels(s, 3)
    assert nd[0] != nd[1] and nd[1] == nd[2] and lv == [0, 1, 1]
    # an operation in between writes what the chain reads: no fusion
    s = tm.Scheduler()
    s.add(tm.Add(R, "abij", X, "abij", bind=False), 1.0, 1.0)
    s.set(X, 2.0)
    s.add(tm.Add(R, "abij", Z, "baij", bind=False), 1.0, 1.0)
    nd, lv = nodes_levels(s, 3)
    assert len(set(nd)) == 3 and lv == [0, 1, 1]  # the second term needs only the first
    # ... but an operation in between that writes only the new member's input does not stop it
    s = tm.Scheduler()
    s.add(tm.Add(R, "abij", X, "abij", bind=False), 1.0, 1.0)
    s.set(Z, 2.0)
    s.add(tm.Add(R, "abij", Z, "baij", bind=False), 1.0, 1.0)
    nd, lv = nodes_levels(s, 3)
    assert nd[0] == nd[2] and lv == [1, 0, 1]
    # out added to itself stays a node of its own; at most eight terms per chain
    s = tm.Scheduler()
    s.add(tm.Add(R, "abij", X, "abij", bind=False), 1.0, 1.0)
    s.add(tm.Add(R, "abij", R, "abij", bind=False), 1.0, 1.0)
    nd, _ = nodes_levels(s, 2)
    assert nd[0] != nd[1]
    s = tm.Scheduler()
    for k in range(10):
        s.add(tm.Add(R, "abij", X if k % 2 else Z, "abij", bind=False), 1.0, 1.0)
    nd, lv = nodes_levels(s, 10)
    assert nd[:8] == [nd[0]] * 8 and nd[8] == nd[9] != nd[0] and lv == [0] * 8 + [1] * 2


def test_fusion_needs_the_same_row_column_split():
    # the ring splits R into (b,j) x (a,i): it cannot share the ladder's (a,b) x (i,j) tiles
    o, v = spaces()
    V, Vr, T, R = tensor(o, v, "vvvv"), tensor(o, v, "ovvo"), tensor(o, v, "vvoo"), tensor(o, v, "vvoo")
    s = tm.Scheduler()
    s.contract(plan(R, "abij", V, "abcd", T, "cdij"), 1.0, 0.0)
    s.contract(plan(R, "abij", Vr, "mbej", T, "aeim"), 1.0, 1.0)
    s.build()
    assert s.info()["fused_ops"] == 0 and [s.op_info(i)[0] for i in range(2)] == [0, 1]


def test_reader_after_writer_and_independent_readers():
    o, v = spaces()
    A, B, C = tensor(o, v, "vvoo"), tensor(o, v, "vvoo"), tensor(o, v, "vvoo")
    s = tm.Scheduler()
    s.set(A, 1.0)                                             # 0: writes A
    s.add(tm.Add(B, "abij", A, "baij", bind=False), 2.0, 0.0)  # 1: reads A, writes B
    s.add(tm.Add(C, "abij", A, "abji", bind=False), 1.0, 0.0)  # 2: reads A, writes C (independent of 1)
    s.set(A, 0.0)                                             # 3: writes A after two readers
    s.build()
    assert [s.op_info(i)[0] for i in range(4)] == [0, 1, 1, 2]
    assert s.info()["levels"] == 3


def test_float64_only_and_build_errors():
    o, v = spaces()
    V, T, R = tensor(o, v, "vvvv"), tensor(o, v, "vvoo"), tensor(o, v, "vvoo")
    s = tm.Scheduler()
    with pytest.raises(tm.TammError):
        s.contract(tm.Plan(R, "abij", V, "abcd", T, "cdij", precision="f32", bind=False), 1.0, 0.0)
    with pytest.raises(tm.TammError):
        s.build()  # nothing queued
    assert TERMS  # the term table exists for the GPU tests
