"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each pin is chosen so that a plausible mistake in the oracle (a dropped tile pair, a wrong sign,
a transposed operand, a wrong beta rule, a wrong tiling remainder, a wrong block rule) fails at
least one test here: dense brute force with numpy.einsum, the ladder as one BLAS GEMM, the
Eq. (cc9)-(cc11) factorisation identity, closed-form block counts, the worked example of
Fig. 1, and invariants (tiling, linearity, label permutation, symmetry inheritance).
"""

import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import BlockTensor, Space, add, contract, screen, set_value, spin_conserving

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------------------------
# helpers (test side; independent of the oracle's loops)
# ---------------------------------------------------------------------------------------------
def dense_masked(tensor_spaces, dense, nonzero=None):
    """Zero the unstored blocks of a dense array (by the given block rule) and return it."""
    x = BlockTensor.from_dense(tensor_spaces, dense, nonzero)
    return x.to_dense()


def rel_err(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    n = np.linalg.norm(np.asarray(b))
    return d / n if n > 0 else d


def random_spin_space(rng, max_tiles=3, max_tile=4):
    na = int(rng.integers(1, 7))
    nb = int(rng.integers(1, 7))
    tile = int(rng.integers(1, max_tile + 1))
    return Space.spin_blocked(na, nb, tile)


def random_problem(rng, n_m, n_n, n_k, nonzero=None):
    """Random label pattern with n_m out&lhs, n_n out&rhs, n_k lhs&rhs labels and random orders."""
    letters = list("abcdefghijklmnop")
    rng.shuffle(letters)
    m = letters[:n_m]
    n = letters[n_m:n_m + n_n]
    k = letters[n_m + n_n:n_m + n_n + n_k]
    out_l = list(m + n)
    lhs_l = list(m + k)
    rhs_l = list(k + n)
    for lst in (out_l, lhs_l, rhs_l):
        rng.shuffle(lst)
    spaces = {c: random_spin_space(rng) for c in m + n + k}
    return "".join(out_l), "".join(lhs_l), "".join(rhs_l), spaces


def make(spaces, lbl, rng, nonzero=None):
    sp = [spaces[c] for c in lbl]
    dense = rng.standard_normal(tuple(s.extent for s in sp))
    return BlockTensor.from_dense(sp, dense, nonzero)


# ---------------------------------------------------------------------------------------------
# tiling: Fig. 1 worked example and the spin-tiling readings
# ---------------------------------------------------------------------------------------------
def test_fig1_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "fig1_tiling.json")))
    sp = g["spaces"]
    tN = Space.fixed(sp["N"]["range"], sp["N"]["tiling"]["fixed"])
    tM = Space.explicit(sp["M"]["range"], sp["M"]["tiling"]["explicit"])
    tK = Space.fixed(sp["K"]["range"], sp["K"]["tiling"]["fixed"])
    everything = lambda t, s: True  # noqa: E731  (Fig. 1 tensors are dense)
    A = BlockTensor([tM, tK], everything)
    assert list(A.shape) == g["printed_facts"]["A{tM,tK}"]["shape"]
    assert len(A.stored_tiles()) == g["printed_facts"]["A{tM,tK}"]["blocks"]
    assert tM.sizes == g["printed_facts"]["tM_tile_sizes"]
    assert tK.sizes == g["printed_facts"]["tK_tile_sizes"]
    assert tN.ntiles == g["implied_facts"]["tN_tiles"]
    assert len(BlockTensor([tK, tN], everything).stored_tiles()) == g["implied_facts"]["B{tK,tN}_blocks"]
    assert len(BlockTensor([tM, tN], everything).stored_tiles()) == g["implied_facts"]["C{tM,tN}_blocks"]


def test_fig4_program_gives_zero():
    g = json.load(open(os.path.join(GOLDEN, "fig4_ops.json")))
    rng = np.random.default_rng(4)
    tM = Space.explicit(30, [10, 20])
    tK = Space.fixed(20, 5)
    tN = Space.fixed(100, 10)
    dense_rule = lambda t, s: True  # noqa: E731
    A = set_value(BlockTensor.zeros([tM, tK], dense_rule), 1.0)                 # A(i,l) = 1.0
    assert all(np.all(b == 1.0) for b in A.blocks.values())
    # B = A ; B += -1 * A  (on B's own, consistent, label binding): B becomes exactly zero
    A2 = set_value(BlockTensor.zeros([tK, tN], dense_rule), 1.0)
    B = BlockTensor.from_dense([tK, tN], rng.standard_normal((20, 100)), dense_rule)
    B = add(B, "la", A2, "la", 1.0, 0.0)                                         # B(l,a) = A(l,a)
    assert all(np.all(b == 1.0) for b in B.blocks.values())
    B = add(B, "la", A2, "la", -1.0, 1.0)                                        # B(l,a) += -1.0 * A(l,a)
    assert all(np.all(b == g["expected"]["B"]) for b in B.blocks.values())
    C = BlockTensor.zeros([tM, tN], dense_rule)
    C = contract(C, "ia", A, "il", B, "la", alpha=0.5, beta=0.0)              # C(i,a) = 0.5*A(i,l)*B(l,a)
    assert all(np.all(b == g["expected"]["C"]) for b in C.blocks.values())
    # The printed binding B(i,l) against B{tK,tN} binds label i to two different spaces: rejected.
    Bbad = BlockTensor.zeros([tK, tN], dense_rule)
    with pytest.raises(ValueError):
        contract(C, "ia", A, "il", Bbad, "ia", 0.5, 0.0)


@pytest.mark.parametrize(
    "na,nb,tile,sizes,spins",
    [
        (100, 100, 40, [40, 40, 20, 40, 40, 20], [0, 0, 0, 1, 1, 1]),  # remainder tile last
        (20, 20, 40, [20, 20], [0, 1]),                                  # clamp to the sub-space
        (5, 5, 5, [5, 5], [0, 1]),
        (20, 20, 5, [5] * 8, [0] * 4 + [1] * 4),
        (16, 16, 32, [16, 16], [0, 1]),
        (3, 3, 8, [3, 3], [0, 1]),
        (37, 37, 16, [16, 16, 5, 16, 16, 5], [0, 0, 0, 1, 1, 1]),
    ],
)
def test_spin_tiling_readings(na, nb, tile, sizes, spins):
    s = Space.spin_blocked(na, nb, tile)
    assert s.sizes == sizes and s.spins == spins
    assert s.extent == na + nb
    assert s.offsets[0] == 0 and all(s.offsets[i + 1] == s.offsets[i] + s.sizes[i] for i in range(s.ntiles - 1))


def test_fixed_tiling_remainder_and_explicit_cover():
    assert Space.fixed(100, 10).sizes == [10] * 10
    assert Space.fixed(23, 10).sizes == [10, 10, 3]
    with pytest.raises(ValueError):
        Space.explicit(30, [10, 10])


# ---------------------------------------------------------------------------------------------
# block rule and screening counts: closed forms and an indicator-tensor count (numpy.einsum)
# ---------------------------------------------------------------------------------------------
def test_spin_rule_closed_form_fractions():
    # with equally many alpha and beta tiles, the stored fraction of rank-4 blocks is
    # P(s_a+s_b = s_c+s_d) = (1/4)^2 + (1/2)^2 + (1/4)^2 = 3/8
    sp = Space.spin_blocked(8, 8, 2)  # 4 alpha + 4 beta tiles
    t = BlockTensor([sp] * 4)
    assert len(t.stored_tiles()) * 8 == 3 * sp.ntiles ** 4
    assert spin_conserving((0, 1, 1, 0)) and not spin_conserving((0, 0, 1, 1))
    assert spin_conserving((1, 1)) and not spin_conserving((0, 1))


def indicator(x: BlockTensor) -> np.ndarray:
    shape = tuple(s.ntiles for s in x.spaces)
    s = np.zeros(shape)
    for t in x.stored_tiles():
        s[t] = 1.0
    return s


def indicator_counts(out, ol, lhs, ll, rhs, rl):
    """Surviving triples, dropped pairs and useful flops from tile-level indicator tensors."""
    so, sl, sr = indicator(out), indicator(lhs), indicator(rhs)
    labels = sorted(set(ol) | set(ll) | set(rl))
    full = "".join(labels)
    pair = np.einsum(f"{ll},{rl}->{full}", sl, sr)
    so_full = np.einsum(f"{ol},{full}->{full}", so, np.ones(pair.shape))
    sizes = {}
    for x, lbl in ((out, ol), (lhs, ll), (rhs, rl)):
        for d, c in enumerate(lbl):
            sizes[c] = np.array(x.spaces[d].sizes, dtype=float)
    ext = np.ones(pair.shape)
    for i, c in enumerate(labels):
        shp = [1] * len(labels)
        shp[i] = -1
        ext = ext * sizes[c].reshape(shp)
    tasks = int(round((pair * so_full).sum()))
    dropped = int(round((pair * (1 - so_full)).sum()))
    flops = int(round(2 * (pair * so_full * ext).sum()))
    return tasks, dropped, flops


TERM_LABELS = {
    "ladder": ("abij", "vvoo", "abcd", "vvvv", "cdij", "vvoo"),
    "ring": ("abij", "vvoo", "mbej", "ovvo", "aeim", "vvoo"),
    "hh_int": ("mnij", "oooo", "mnef", "oovv", "efij", "vvoo"),
    "hh": ("abij", "vvoo", "mnij", "oooo", "abmn", "vvoo"),
    "t1_v": ("abij", "vvoo", "abej", "vvvo", "ei", "vo"),
    "t1_o": ("abij", "vvoo", "mbij", "ovoo", "am", "vo"),
}


def term_tensors(term, occ, vir):
    ol, op, ll, lp, rl, rp = TERM_LABELS[term]
    sp = lambda p: [occ if c == "o" else vir for c in p]  # noqa: E731
    return BlockTensor(sp(op)), ol, BlockTensor(sp(lp)), ll, BlockTensor(sp(rp)), rl


@pytest.mark.parametrize(
    "term,occ,vir,expected_tasks,expected_out",
    [
        # cfg: O=10, V=40, tiles of 5 (ladder only): 96 stored R blocks, 2560 surviving pairs
        ("ladder", (5, 5, 5), (20, 20, 5), 2560, 96),
        # cfg: O=40, V=200, tiles of 40: all six terms
        ("ladder", (20, 20, 40), (100, 100, 40), 810, 54),
        ("ring", (20, 20, 40), (100, 100, 40), 270, 54),
        ("hh_int", (20, 20, 40), (100, 100, 40), 90, 6),
        ("hh", (20, 20, 40), (100, 100, 40), 90, 54),
        ("t1_v", (20, 20, 40), (100, 100, 40), 162, 54),
        ("t1_o", (20, 20, 40), (100, 100, 40), 54, 54),
    ],
)
def test_screen_counts_match_indicator_einsum_and_closed_forms(term, occ, vir, expected_tasks, expected_out):
    o = Space.spin_blocked(*occ)
    v = Space.spin_blocked(*vir)
    out, ol, lhs, ll, rhs, rl = term_tensors(term, o, v)
    s = screen(out, ol, lhs, ll, rhs, rl)
    tasks, dropped, flops = indicator_counts(out, ol, lhs, ll, rhs, rl)
    assert s["tasks"] == tasks == expected_tasks
    assert s["out_blocks"] == expected_out
    assert s["dropped"] == dropped == 0
    assert s["useful_flops"] == flops


def test_useful_fractions_closed_forms():
    # equal alpha/beta tile counts: 4x4->4 terms keep 10/64 of all tile triples, T1 terms 3/16
    o = Space.spin_blocked(4, 4, 2)
    v = Space.spin_blocked(4, 4, 2)
    for term, frac in (("ladder", 10 / 64), ("ring", 10 / 64), ("hh_int", 10 / 64), ("hh", 10 / 64),
                       ("t1_v", 3 / 16), ("t1_o", 3 / 16)):
        out, ol, lhs, ll, rhs, rl = term_tensors(term, o, v)
        s = screen(out, ol, lhs, ll, rhs, rl)
        n_labels = len(set(ol) | set(ll) | set(rl))
        assert s["tasks"] == pytest.approx(frac * 4 ** n_labels)


def test_factorised_cost_exponents():
    g = json.load(open(os.path.join(GOLDEN, "eq_cc9_cc11_cost.json")))
    for no, nu in ((2, 3), (4, 6), (3, 7)):
        o = Space([no])
        v = Space([nu])
        d = lambda t, s: True  # noqa: E731
        I = BlockTensor([o] * 4, d)
        V = BlockTensor([o, o, v, v], d)
        T = BlockTensor([v, v, o, o], d)
        R = BlockTensor([v, v, o, o], d)
        f1 = screen(I, "mnij", V, "mnef", T, "efij")["useful_flops"]
        f2 = screen(R, "abij", I, "mnij", T, "abmn")["useful_flops"]
        e = g["factorised_cost_exponents"]
        assert f1 == f2 == 2 * no ** e["n_o"] * nu ** e["n_u"]


# ---------------------------------------------------------------------------------------------
# contraction values: dense brute force, GEMM special case, Eq. (cc9)-(cc11) identity
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("term", list(TERM_LABELS))
def test_terms_match_dense_einsum(term):
    rng = np.random.default_rng(hash(term) % 2**32)
    o = Space.spin_blocked(3, 2, 2)     # uneven alpha/beta, remainder tiles
    v = Space.spin_blocked(5, 4, 3)
    out, ol, lhs, ll, rhs, rl = term_tensors(term, o, v)
    L = BlockTensor.from_dense(lhs.spaces, rng.standard_normal(lhs.shape))
    Rh = BlockTensor.from_dense(rhs.spaces, rng.standard_normal(rhs.shape))
    O0 = BlockTensor.from_dense(out.spaces, rng.standard_normal(out.shape))
    alpha, beta = -0.7, 0.3
    got = contract(O0, ol, L, ll, Rh, rl, alpha, beta).to_dense()
    ref = beta * O0.to_dense() + alpha * np.einsum(f"{ll},{rl}->{ol}", L.to_dense(), Rh.to_dense())
    ref = dense_masked(out.spaces, ref)
    assert rel_err(got, ref) < 1e-13
    assert np.linalg.norm(ref) > 0


@pytest.mark.parametrize("seed", range(8))
def test_random_label_patterns_match_dense_einsum(seed):
    rng = np.random.default_rng(100 + seed)
    n_m, n_n, n_k = (int(x) for x in rng.integers(1, 3, size=3))
    ol, ll, rl, spaces = random_problem(rng, n_m, n_n, n_k)
    L = make(spaces, ll, rng)
    R = make(spaces, rl, rng)
    O0 = make(spaces, ol, rng)
    got = contract(O0, ol, L, ll, R, rl, 1.3, -0.4).to_dense()
    ref = -0.4 * O0.to_dense() + 1.3 * np.einsum(f"{ll},{rl}->{ol}", L.to_dense(), R.to_dense())
    # only out's stored blocks are kept (odd-rank tensors have no spin rule and store every block)
    ref = dense_masked(O0.spaces, ref)
    assert rel_err(got, ref) < 1e-13


def test_user_predicate_drops_and_counts():
    rng = np.random.default_rng(7)
    sp = Space.fixed(9, 3)

    def rule_from(seed):
        def rule(tiles, spins):
            return (hash((seed,) + tuple(tiles)) % 3) != 0
        return rule

    ol, ll, rl = "ab", "ac", "cb"
    out = BlockTensor.from_dense([sp, sp], rng.standard_normal((9, 9)), rule_from(1))
    L = BlockTensor.from_dense([sp, sp], rng.standard_normal((9, 9)), rule_from(2))
    R = BlockTensor.from_dense([sp, sp], rng.standard_normal((9, 9)), rule_from(3))
    got = contract(out, ol, L, ll, R, rl, 1.0, 1.0)
    ref = out.to_dense() + L.to_dense() @ R.to_dense()
    ref = dense_masked([sp, sp], ref, rule_from(1))
    assert rel_err(got.to_dense(), ref) < 1e-13
    s = screen(out, ol, L, ll, R, rl)
    tasks, dropped, flops = indicator_counts(out, ol, L, ll, R, rl)
    assert (s["tasks"], s["dropped"], s["useful_flops"]) == (tasks, dropped, flops)
    assert dropped > 0


def test_ladder_is_one_gemm():
    rng = np.random.default_rng(11)
    o = Space.spin_blocked(3, 3, 2)
    v = Space.spin_blocked(4, 4, 3)
    V = BlockTensor.from_dense([v] * 4, rng.standard_normal((8,) * 4))
    T = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((8, 8, 6, 6)))
    R = BlockTensor.zeros([v, v, o, o])
    got = contract(R, "abij", V, "abcd", T, "cdij", 1.0, 0.0).to_dense()
    ref = (V.to_dense().reshape(64, 64) @ T.to_dense().reshape(64, 36)).reshape(8, 8, 6, 6)
    assert rel_err(got, ref) < 1e-14


def test_eq_cc9_to_cc11_factorisation_identity():
    rng = np.random.default_rng(12)
    o = Space.spin_blocked(2, 2, 1)
    v = Space.spin_blocked(4, 4, 2)
    Vd = dense_masked([o, o, v, v], rng.standard_normal((4, 4, 8, 8)))
    Td = dense_masked([v, v, o, o], rng.standard_normal((8, 8, 4, 4)))
    direct = 0.25 * np.einsum("mnef,efij,abmn->abij", Vd, Td, Td)  # Eq. (cc9), n_o^4 n_u^4
    V = BlockTensor.from_dense([o, o, v, v], Vd)
    T = BlockTensor.from_dense([v, v, o, o], Td)
    I = contract(BlockTensor.zeros([o] * 4), "mnij", V, "mnef", T, "efij", 1.0, 0.0)        # Eq. (cc10)
    R = contract(BlockTensor.zeros([v, v, o, o]), "abij", I, "mnij", T, "abmn", 0.25, 0.0)  # Eq. (cc11)
    assert rel_err(R.to_dense(), direct) < 1e-13
    assert np.linalg.norm(direct) > 0


# ---------------------------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------------------------
def test_linearity_in_alpha_beta_and_beta_zero_ignores_nan():
    rng = np.random.default_rng(13)
    o = Space.spin_blocked(3, 3, 2)
    v = Space.spin_blocked(4, 3, 2)
    V = BlockTensor.from_dense([v] * 4, rng.standard_normal((7,) * 4))
    T = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((7, 7, 6, 6)))
    R0 = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((7, 7, 6, 6)))
    a, b = 0.37, -1.9
    full = contract(R0, "abij", V, "abcd", T, "cdij", a, b).to_dense()
    unit = contract(R0, "abij", V, "abcd", T, "cdij", 1.0, 0.0).to_dense()
    assert rel_err(full, a * unit + b * R0.to_dense()) < 1e-14
    Rnan = R0.copy()
    for blk in Rnan.blocks.values():
        blk[...] = np.nan
    z = contract(Rnan, "abij", V, "abcd", T, "cdij", a, 0.0).to_dense()
    assert np.all(np.isfinite(z)) and rel_err(z, a * unit) < 1e-15


def test_tiling_invariance():
    rng = np.random.default_rng(14)
    Vd = rng.standard_normal((10,) * 4)
    Td = rng.standard_normal((10, 10, 6, 6))
    results = []
    for tv, to in ((1, 1), (2, 3), (5, 3), (5, 2), (3, 1)):
        v = Space.spin_blocked(5, 5, tv)
        o = Space.spin_blocked(3, 3, to)
        V = BlockTensor.from_dense([v] * 4, Vd)
        T = BlockTensor.from_dense([v, v, o, o], Td)
        R = BlockTensor.zeros([v, v, o, o])
        results.append(contract(R, "abij", V, "abcd", T, "cdij", 1.0, 0.0).to_dense())
    for r in results[1:]:
        assert rel_err(r, results[0]) < 1e-14


def test_label_permutation_invariance():
    rng = np.random.default_rng(15)
    o = Space.spin_blocked(3, 2, 2)
    v = Space.spin_blocked(3, 4, 2)
    Vd = dense_masked([o, v, v, o], rng.standard_normal((5, 7, 7, 5)))
    Td = dense_masked([v, v, o, o], rng.standard_normal((7, 7, 5, 5)))
    V = BlockTensor.from_dense([o, v, v, o], Vd)
    T = BlockTensor.from_dense([v, v, o, o], Td)
    R = BlockTensor.zeros([v, v, o, o])
    ref = contract(R, "abij", V, "mbej", T, "aeim", 1.0, 0.0).to_dense()
    # store V as V'[e,j,m,b] = V[m,b,e,j] and relabel; spin rule on (e,j | m,b) is the same rule
    Vp = BlockTensor.from_dense([v, o, o, v], np.transpose(Vd, (2, 3, 0, 1)))
    got = contract(R, "abij", Vp, "ejmb", T, "aeim", 1.0, 0.0).to_dense()
    assert rel_err(got, ref) < 1e-14
    # store T transposed as T'[i,m,a,e] and swap lhs/rhs
    Tp = BlockTensor.from_dense([o, o, v, v], np.transpose(Td, (2, 3, 0, 1)))
    got2 = contract(R, "abij", Tp, "imae", V, "mbej", 1.0, 0.0).to_dense()
    assert rel_err(got2, ref) < 1e-14


def test_symmetry_inheritance():
    rng = np.random.default_rng(16)
    o = Space.spin_blocked(3, 3, 2)
    v = Space.spin_blocked(4, 4, 3)
    W = rng.standard_normal((8,) * 4)
    Vd = W + W.transpose(1, 0, 3, 2)               # V[abcd] = V[badc]
    X = rng.standard_normal((8, 8, 6, 6))
    Td = X + X.transpose(1, 0, 3, 2)               # T[cdij] = T[dcji]
    V = BlockTensor.from_dense([v] * 4, Vd)
    T = BlockTensor.from_dense([v, v, o, o], Td)
    R = contract(BlockTensor.zeros([v, v, o, o]), "abij", V, "abcd", T, "cdij", 1.0, 0.0).to_dense()
    assert rel_err(R, R.transpose(1, 0, 3, 2)) < 1e-14


def test_additivity_over_split_k_tiles():
    # splitting the summed range into two tensors over the two halves adds up to the whole
    rng = np.random.default_rng(17)
    a = Space.fixed(6, 2)
    k1 = Space.fixed(4, 2)
    k2 = Space.fixed(5, 2)
    k = Space.fixed(9, 2)
    allr = lambda t, s: True  # noqa: E731
    Ld = rng.standard_normal((6, 9))
    Rd = rng.standard_normal((9, 6))
    whole = contract(BlockTensor.zeros([a, a], allr), "ij", BlockTensor.from_dense([a, k], Ld, allr), "ik",
                     BlockTensor.from_dense([k, a], Rd, allr), "kj", 1.0, 0.0).to_dense()
    p1 = contract(BlockTensor.zeros([a, a], allr), "ij", BlockTensor.from_dense([a, k1], Ld[:, :4], allr), "ik",
                  BlockTensor.from_dense([k1, a], Rd[:4], allr), "kj", 1.0, 0.0)
    p2 = contract(p1, "ij", BlockTensor.from_dense([a, k2], Ld[:, 4:], allr), "ik",
                  BlockTensor.from_dense([k2, a], Rd[4:], allr), "kj", 1.0, 1.0).to_dense()
    assert rel_err(p2, whole) < 1e-14


def test_label_errors():
    sp = Space.fixed(4, 2)
    x = BlockTensor.zeros([sp, sp], lambda t, s: True)
    with pytest.raises(ValueError):
        contract(x, "ij", x, "ik", x, "kk", 1.0, 0.0)     # repeated label
    with pytest.raises(ValueError):
        contract(x, "ij", x, "ik", x, "kl", 1.0, 0.0)     # l in one tensor only, j in one only
    with pytest.raises(ValueError):
        contract(x, "ijk", x, "ik", x, "kj", 1.0, 0.0)    # rank mismatch
    with pytest.raises(ValueError):
        oracle.parse_labels("ij", "ijk", "kj")           # j occurs in all three tensors


# ---------------------------------------------------------------------------------------------
# denominator update: closed form, element by element
# ---------------------------------------------------------------------------------------------
def test_denominator_update_elementwise():
    rng = np.random.default_rng(18)
    o = Space.spin_blocked(2, 2, 1)
    v = Space.spin_blocked(3, 3, 2)
    e_o = rng.uniform(-2, -0.5, 4)
    e_v = rng.uniform(0.2, 3, 6)
    R = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((6, 6, 4, 4)))
    T = oracle.denominator_update(R, e_o, e_v).to_dense()
    Rd = R.to_dense()
    for a, b, i, j in itertools.product(range(6), range(6), range(4), range(4)):
        d = e_o[i] + e_o[j] - e_v[a] - e_v[b]
        assert T[a, b, i, j] == Rd[a, b, i, j] / d  # same operation order: bitwise
    R1 = BlockTensor.from_dense([v, o], rng.standard_normal((6, 4)))
    T1 = oracle.denominator_update(R1, e_o, e_v).to_dense()
    R1d = R1.to_dense()
    for a, i in itertools.product(range(6), range(4)):
        assert T1[a, i] == R1d[a, i] / (e_o[i] - e_v[a])


def test_denominator_update_exact_powers_of_two():
    # energies on a grid where every denominator is minus a power of two: the division is then an
    # exact scaling, so T' = R * 2^-k holds bitwise (independent of how the quotient is formed)
    o = Space.spin_blocked(2, 2, 1)
    v = Space.spin_blocked(2, 2, 1)
    e_o = np.array([-1.0, -1.0, -1.0, -1.0])
    e_v = np.array([1.0, 1.0, 3.0, 3.0])          # D = -2 - e_a - e_b in {-4, -6, -8}
    rng = np.random.default_rng(19)
    R = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((4, 4, 4, 4)))
    T = oracle.denominator_update(R, e_o, e_v).to_dense()
    Rd = R.to_dense()
    for a, b in itertools.product(range(4), range(4)):
        s_ab = e_v[a] + e_v[b]
        if s_ab in (2.0, 6.0):                     # D = -4 or -8
            assert np.array_equal(T[a, b], Rd[a, b] * (-1.0 / (2.0 + s_ab)))
    # every quotient times its denominator gives back the residual to within one rounding
    e_o = rng.uniform(-2, -0.5, 4)
    e_v = rng.uniform(0.2, 3, 4)
    T = oracle.denominator_update(R, e_o, e_v).to_dense()
    D = e_o[None, None, :, None] + e_o[None, None, None, :] - e_v[:, None, None, None] - e_v[None, :, None, None]
    assert np.all(np.abs(T * D - Rd) <= 2.0 ** -51 * np.abs(Rd))
    assert np.all(T * Rd <= 0)                     # D < 0 everywhere


@pytest.mark.parametrize("term", list(TERM_LABELS))
def test_sampled_out_tiles_equal_the_full_contraction(term):
    # the restriction to listed output blocks (used for sampled checks of large problems) gives
    # exactly the blocks of the full contraction, for every term on ragged tilings
    rng = np.random.default_rng(sum(map(ord, term)))
    o = Space.spin_blocked(3, 2, 2)
    v = Space.spin_blocked(5, 4, 3)
    out, ol, lhs, ll, rhs, rl = term_tensors(term, o, v)
    L = BlockTensor.from_dense(lhs.spaces, rng.standard_normal(lhs.shape))
    Rh = BlockTensor.from_dense(rhs.spaces, rng.standard_normal(rhs.shape))
    O0 = BlockTensor.from_dense(out.spaces, rng.standard_normal(out.shape))
    full = contract(O0, ol, L, ll, Rh, rl, 0.75, 0.5)
    tiles = O0.stored_tiles()
    pick = [tiles[i] for i in rng.choice(len(tiles), size=min(5, len(tiles)), replace=False)]
    part = contract(O0, ol, L, ll, Rh, rl, 0.75, 0.5, out_tiles=pick)
    assert sorted(part.blocks) == sorted(pick)
    for t in pick:
        assert np.array_equal(part.blocks[t], full.blocks[t])
    # and the full contraction itself against dense einsum on exactly these blocks
    ref = 0.5 * O0.to_dense() + 0.75 * np.einsum(f"{ll},{rl}->{ol}", L.to_dense(), Rh.to_dense())
    for t in pick:
        assert rel_err(part.blocks[t], ref[O0.block_slices(t)]) < 1e-13
    with pytest.raises(ValueError):
        unstored = next(t for t in O0.all_tiles() if not O0.is_stored(tuple(t)))
        contract(O0, ol, L, ll, Rh, rl, 1.0, 0.0, out_tiles=[tuple(unstored)])
