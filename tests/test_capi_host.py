"""Host-only checks of the C ABI (no GPU needed): exported symbols, tiling, block structure,
label analysis, plan statistics against the oracle's screening counts, and error codes."""

import ctypes

import numpy as np
import pytest

import oracle
from paper_2201_01257_amd import _lib
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd.synth import TERMS

lib = _lib.load()


def test_library_exports_every_declared_function():
    names = _lib.header_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    # every declared function has a ctypes signature in the binding and vice versa
    assert sorted(_lib.SIGNATURES) == names


@pytest.mark.parametrize("na,nb,tile", [(100, 100, 40), (20, 20, 40), (5, 5, 5), (37, 11, 16), (3, 0, 2), (0, 4, 3)])
def test_spin_tiling_matches_oracle(na, nb, tile):
    s = tm.Space.spin(na, nb, tile)
    o = oracle.Space.spin_blocked(na, nb, tile)
    assert list(s.sizes) == o.sizes and list(s.spins) == o.spins and list(s.offsets) == o.offsets


def test_fig1_tiling_through_the_abi():
    tM = tm.Space.explicit([10, 20])
    tK = tm.Space.fixed(20, 5)
    tN = tm.Space.fixed(100, 10)
    dense = lambda t, s: True  # noqa: E731
    A = tm.Tensor([tM, tK], nonzero=dense, device=None)
    assert A.shape == (30, 20) and A.nblocks == 8
    assert tN.ntiles == 10 and list(tK.sizes) == [5, 5, 5, 5]


def test_block_table_matches_oracle_storage_order():
    o = tm.Space.spin(3, 2, 2)
    v = tm.Space.spin(4, 5, 3)
    T = tm.Tensor([v, v, o, o], device=None)
    os_ = oracle.Space.spin_blocked(3, 2, 2)
    vs = oracle.Space.spin_blocked(4, 5, 3)
    ref = oracle.BlockTensor([vs, vs, os_, os_])
    stored = ref.stored_tiles()
    assert [tuple(x) for x in T.block_tiles] == stored
    sizes = [int(np.prod(ref.block_shape(t))) for t in stored]
    assert list(T.block_off) == list(np.concatenate([[0], np.cumsum(sizes)[:-1]]))
    assert T.numel == ref.nnz()


def term_structures(term, occ, vir, device=None):
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), alpha = TERMS[term]
    o = tm.Space.spin(*occ)
    v = tm.Space.spin(*vir)
    sp = lambda p: [o if c == "o" else v for c in p]  # noqa: E731
    os_ = oracle.Space.spin_blocked(*occ)
    vs = oracle.Space.spin_blocked(*vir)
    osp = lambda p: [os_ if c == "o" else vs for c in p]  # noqa: E731
    gpu = (tm.Tensor(sp(op), device=device), ol, tm.Tensor(sp(lp), device=device), ll, tm.Tensor(sp(rp), device=device), rl)
    ref = (oracle.BlockTensor(osp(op)), ol, oracle.BlockTensor(osp(lp)), ll, oracle.BlockTensor(osp(rp)), rl)
    return gpu, ref


@pytest.mark.parametrize("term", list(TERMS))
@pytest.mark.parametrize("occ,vir", [((20, 20, 40), (100, 100, 40)), ((5, 5, 5), (20, 20, 5)), ((3, 2, 2), (5, 4, 3))])
def test_plan_statistics_match_oracle_screen(term, occ, vir):
    gpu, ref = term_structures(term, occ, vir)
    p = tm.Plan(*gpu, bind=False)
    st = p.stats()
    s = oracle.screen(*ref)
    assert st["tasks"] == s["tasks"]
    assert st["out_blocks"] == s["out_blocks"]
    assert st["dropped"] == s["dropped"] == 0
    assert st["useful_flops"] == s["useful_flops"]


def test_plan_statistics_with_user_predicate_dropped():
    sp = tm.Space.fixed(9, 3)
    osp = oracle.Space.fixed(9, 3)

    def rule(seed):
        return lambda t, s: (hash((seed,) + tuple(int(x) for x in t)) % 3) != 0

    out = tm.Tensor([sp, sp], nonzero=rule(1), device=None)
    L = tm.Tensor([sp, sp], nonzero=rule(2), device=None)
    R = tm.Tensor([sp, sp], nonzero=rule(3), device=None)
    st = tm.Plan(out, "ab", L, "ac", R, "cb", bind=False).stats()
    s = oracle.screen(oracle.BlockTensor([osp, osp], rule(1)), "ab", oracle.BlockTensor([osp, osp], rule(2)), "ac",
                      oracle.BlockTensor([osp, osp], rule(3)), "cb")
    assert (st["tasks"], st["dropped"], st["useful_flops"]) == (s["tasks"], s["dropped"], s["useful_flops"])
    assert st["dropped"] > 0


def status_of(fn):
    with pytest.raises(tm.TammError) as e:
        fn()
    return e.value.status


def test_error_codes():
    o = tm.Space.spin(2, 2, 2)
    v = tm.Space.spin(3, 3, 3)
    V = tm.Tensor([v, v, v, v], device=None)
    T = tm.Tensor([v, v, o, o], device=None)
    R = tm.Tensor([v, v, o, o], device=None)
    assert status_of(lambda: tm.Plan(R, "abij", V, "abcd", T, "cdi", bind=False)) == "TAMM_ERR_SHAPE"
    assert status_of(lambda: tm.Plan(R, "abij", V, "abcc", T, "cdij", bind=False)) == "TAMM_ERR_LABEL"
    assert status_of(lambda: tm.Plan(R, "abij", V, "abcd", T, "cxij", bind=False)) == "TAMM_ERR_LABEL"
    assert status_of(lambda: tm.Plan(R, "ab1j", V, "abcd", T, "cdij", bind=False)) == "TAMM_ERR_LABEL"
    # label d bound to virtual (V) and to occupied (T) spaces
    assert status_of(lambda: tm.Plan(R, "abij", V, "abcd", T, "cidj", bind=False)) == "TAMM_ERR_LABEL"
    for prec in ("f32", "bf16x3", "bf16x4_aligned"):
        tm.Plan(R, "abij", V, "abcd", T, "cdij", precision=prec, bind=False)  # every precision plans
    h0 = ctypes.c_void_p()
    assert lib.tamm_plan_create(R._h, b"abij", V._h, b"abcd", T._h, b"cdij", 7, ctypes.byref(h0)) == -1  # bad precision
    # Fig. 4 as printed: B(i,l) with B declared over (tK, tN) binds i to two spaces
    tM = tm.Space.explicit([10, 20])
    tK = tm.Space.fixed(20, 5)
    tN = tm.Space.fixed(100, 10)
    dense = lambda t, s: True  # noqa: E731
    A = tm.Tensor([tM, tK], nonzero=dense, device=None)
    B = tm.Tensor([tK, tN], nonzero=dense, device=None)
    C = tm.Tensor([tM, tN], nonzero=dense, device=None)
    assert status_of(lambda: tm.Plan(C, "ia", A, "il", B, "il", bind=False)) == "TAMM_ERR_LABEL"
    tm.Plan(C, "ia", A, "il", B, "la", bind=False)  # the consistent binding plans fine
    # executing without bound storage/workspace is refused before any GPU work
    p = tm.Plan(R, "abij", V, "abcd", T, "cdij", bind=False)
    assert status_of(lambda: p.execute(1.0, 0.0, stream=ctypes.c_void_p(0))) == "TAMM_ERR_UNBOUND"
    assert status_of(lambda: p.set_config(99)) == "TAMM_ERR_ARG"
    # null arguments
    h = ctypes.c_void_p()
    assert lib.tamm_space_create(None, None, 3, ctypes.byref(h)) == -1
    assert lib.tamm_space_create_spin(-1, 2, 2, ctypes.byref(h)) == -1
    assert lib.tamm_tensor_create(None, 2, None, None, ctypes.byref(h)) == -1
    assert lib.tamm_plan_create(None, b"ab", None, b"ab", None, b"ab", 0, ctypes.byref(h)) == -1
    assert lib.tamm_last_error()
    assert lib.tamm_tensor_bind(V._h, None, 0) == -1
    assert lib.tamm_tensor_bind(V._h, ctypes.c_void_p(4096), 8) == -6  # smaller than needed


def test_every_kernel_config_plans():
    o = tm.Space.spin(20, 20, 40)
    v = tm.Space.spin(100, 100, 40)
    V = tm.Tensor([v, v, v, v], device=None)
    T = tm.Tensor([v, v, o, o], device=None)
    R = tm.Tensor([v, v, o, o], device=None)
    p = tm.Plan(R, "abij", V, "abcd", T, "cdij", bind=False)
    for c in range(p.config_count()):
        p.set_config(c, 1)
        tiles = p.stats()["work_items"]
        for ks in (1, 2, 5):
            p.set_config(c, ks)
            st = p.stats()
            assert st["kernel_config"] == c and st["k_splits"] == ks
            # each tile is split into 1..ks parts, the heaviest blocks' tiles into ks
            assert tiles <= st["work_items"] <= tiles * ks
            assert ks == 1 or st["work_items"] > tiles
            assert p.workspace_size() > 0
            assert p.config_name().startswith("f64_")


def test_operand_blocks_beyond_the_gather_range_are_rejected():
    # one 512^3 block (2^27 elements, 1 GiB): the gathers address operand blocks below 2^27 elements
    big = tm.Space.fixed(512, 512)
    small = tm.Space.fixed(4, 4)
    dense = lambda t, s: True  # noqa: E731
    A = tm.Tensor([big, big, big], nonzero=dense, device=None)
    B = tm.Tensor([big, small], nonzero=dense, device=None)
    C = tm.Tensor([big, big, small], nonzero=dense, device=None)
    assert status_of(lambda: tm.Plan(C, "abj", A, "abk", B, "kj", bind=False)) == "TAMM_ERR_UNSUPPORTED"
    # one tile smaller and the same contraction plans
    ok = tm.Space.fixed(500, 500)
    A2 = tm.Tensor([ok, ok, ok], nonzero=dense, device=None)
    B2 = tm.Tensor([ok, small], nonzero=dense, device=None)
    C2 = tm.Tensor([ok, ok, small], nonzero=dense, device=None)
    tm.Plan(C2, "abj", A2, "abk", B2, "kj", bind=False)


def test_gather_layout_pairs_only_for_adjacent_table_pairs():
    # even tile sizes: every grouped pair of table entries is adjacent -> 16-byte gathers
    even = term_structures("ladder", (12, 12, 12), (16, 24, 16), None)[0]
    st = tm.Plan(*even, bind=False).stats()
    assert st["gather_layout"] & 4
    assert st["gather_layout"] & 3 == 2  # V[abcd]: A gathered along k; T[cdij]: B along rows
    # an odd tile size on the stride-1 labels -> 8-byte gathers
    odd = term_structures("ladder", (11, 11, 11), (15, 4, 15), None)[0]
    assert not tm.Plan(*odd, bind=False).stats()["gather_layout"] & 4


def test_group_classes_and_workspace_independent_of_configuration():
    # members of two gather layout classes (ladder: A k-contiguous; t1_v: neither operand is);
    # one configuration for all classes or each class's default, the workspace size is the same
    o = tm.Space.spin(6, 6, 4)
    v = tm.Space.spin(10, 10, 5)
    plans = []
    for term in ("ladder", "t1_v", "ring"):
        (on, op, ol), (ln, lp, ll), (rn, rp, rl), _ = TERMS[term]
        sp = {"o": o, "v": v}
        mk = lambda pat: tm.Tensor([sp[c] for c in pat], device=None)  # noqa: E731
        plans.append(tm.Plan(mk(op), ol, mk(lp), ll, mk(rp), rl, bind=False))
    layouts = {p.stats()["gather_layout"] for p in plans}
    assert len(layouts) >= 2
    lib = _lib.load()
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    g = ctypes.c_void_p()
    assert lib.tamm_group_create(arr, len(plans), ctypes.byref(g)) == 0
    try:
        sizes = set()
        n = ctypes.c_size_t()
        for c in [-1] + list(range(plans[0].config_count())):
            assert lib.tamm_group_set_config(g, c, 0) == 0
            assert lib.tamm_group_workspace_size(g, ctypes.byref(n)) == 0
            sizes.add(n.value)
            cfg, grid, items = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
            assert lib.tamm_group_stats(g, ctypes.byref(cfg), ctypes.byref(grid), ctypes.byref(items)) == 0
            assert items.value > 0 and (c < 0 or cfg.value == c)
        assert len(sizes) == 1
        assert lib.tamm_group_set_config(g, 999, 0) == -1
        assert lib.tamm_group_set_config(g, 0, -1) == -1
    finally:
        lib.tamm_group_destroy(g)


def test_one_shot_plan_cache_on_the_host():
    # the cache keys plans by handles, labels and precision; destroying a tensor evicts its plans;
    # workspace errors are raised before any GPU call
    lib = _lib.load()
    assert lib.tamm_contract_cache_clear() == 0
    o = tm.Space.spin(4, 4, 3)
    v = tm.Space.spin(7, 7, 4)
    V = tm.Tensor([v, v, v, v], device=None)
    T = tm.Tensor([v, v, o, o], device=None)
    R = tm.Tensor([v, v, o, o], device=None)
    count = lambda: tm.contract_cache_count()  # noqa: E731

    def ws_size(out, lhs, rhs, labels=(b"abij", b"abcd", b"cdij"), prec=0):
        n = ctypes.c_size_t()
        rc = lib.tamm_contract_workspace_size(out._h, labels[0], lhs._h, labels[1], rhs._h, labels[2], prec,
                                              ctypes.byref(n))
        return rc, n.value

    rc, n = ws_size(R, V, T)
    assert rc == 0 and count() == 1
    assert n == tm.Plan(R, "abij", V, "abcd", T, "cdij", bind=False).workspace_size()
    assert ws_size(R, V, T) == (0, n) and count() == 1          # cache hit
    assert ws_size(R, V, T, prec=2)[0] == 0 and count() == 2     # another precision, another plan
    assert ws_size(R, V, T, labels=(b"abij", b"abcc", b"cdij"))[0] == -2 and count() == 2  # label error, nothing cached
    # null, misaligned and short workspaces are refused before the upload
    s0 = ctypes.c_void_p(0)
    call = lambda ws, nb: lib.tamm_contract(R._h, b"abij", V._h, b"abcd", T._h, b"cdij", 0, 1.0, 0.0,  # noqa: E731
                                            ctypes.c_void_p(ws), nb, s0)
    assert call(None, n) == -7
    assert call(4096 + 8, n) == -7
    assert call(4096, n - 1) == -7
    assert count() == 2
    T2 = tm.Tensor([v, v, o, o], device=None)
    assert ws_size(R, V, T2)[0] == 0 and count() == 3
    del T2                                                       # evicts the plan that names it
    assert count() == 2
    del R                                                        # evicts both plans for out R
    assert count() == 0
    R3 = tm.Tensor([v, v, o, o], device=None)
    assert ws_size(R3, V, T)[0] == 0 and count() == 1
    assert lib.tamm_contract_cache_clear() == 0 and count() == 0


def test_one_shot_plan_cache_from_several_threads():
    # the cache lock: threads asking for the same and for distinct contractions at once end with
    # one cached plan per distinct key and identical sizes for identical keys
    import threading

    lib = _lib.load()
    assert lib.tamm_contract_cache_clear() == 0
    o = tm.Space.spin(4, 4, 3)
    v = tm.Space.spin(7, 7, 4)
    V = tm.Tensor([v, v, v, v], device=None)
    T = tm.Tensor([v, v, o, o], device=None)
    outs = [tm.Tensor([v, v, o, o], device=None) for _ in range(4)]
    sizes = {}
    errors = []

    def work(i):
        for rep in range(20):
            out = outs[(i + rep) % len(outs)]
            n = ctypes.c_size_t()
            rc = lib.tamm_contract_workspace_size(out._h, b"abij", V._h, b"abcd", T._h, b"cdij", 0, ctypes.byref(n))
            if rc != 0:
                errors.append(rc)
            sizes.setdefault(id(out), set()).add(n.value)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert errors == []
    assert tm.contract_cache_count() == len(outs)
    assert all(len(s) == 1 for s in sizes.values()) and len({min(s) for s in sizes.values()}) == 1
    assert lib.tamm_contract_cache_clear() == 0
