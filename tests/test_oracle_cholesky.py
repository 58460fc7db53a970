"""Pins of the Cholesky-vector ladder oracle (Eq. (cc12), Sec. IV-A-1) against what the mathematics
fixes, without the oracle's own block loop:

* exactness: vectors from a textbook Cholesky factorisation (numpy.linalg.cholesky) of a positive
  definite matrix of pair integrals M[(pr),(qs)] must give back v[p,q,r,s] = (pr|qs) - (ps|qr),
  read straight from M with the spin selection -- this fixes which index pairs share an
  auxiliary sum (a swapped r and s, or q and r, fails);
* brute force: the ladder on dense zero-filled arrays, both Eq. (cc12) terms summed over L by
  one ``numpy.einsum`` each without forming V;
* symmetries of the rebuilt integrals for symmetric vectors (exchange antisymmetry, particle
  exchange, bra-ket);
* a special case: one vector of the form u_p u_q (integers, so exact) makes both terms equal
  on same-spin blocks, so V vanishes there, while on a block (alpha, beta, alpha, beta) only the
  first term survives and V = u_a u_b u_c u_d;
* the factorisation the GPU path uses (contract the pair product G[a,c,b,d] = sum_L B[a,c,L]
  B[b,d,L] with T[c,d,i,j] - T[d,c,i,j]) is an identity of the same definition.
"""

import itertools

import numpy as np
import pytest

import oracle
from oracle.cholesky import cholesky_ladder, cholesky_tensor, spin_diagonal, v_from_cholesky
from paper_2201_01257_amd import synth


def spaces(n_vir, t_vir, n_occ, t_occ, n_aux, t_aux):
    v = oracle.Space.spin_blocked(n_vir // 2, n_vir - n_vir // 2, t_vir)
    o = oracle.Space.spin_blocked(n_occ // 2, n_occ - n_occ // 2, t_occ)
    x = oracle.Space.fixed(n_aux, t_aux)
    return v, o, x


def spin_of(space, p):
    return space.index_spin(p)


def test_exact_cholesky_reproduces_pair_integrals():
    n_sp = 3  # spatial orbitals per spin; spin-orbitals 0..2 alpha, 3..5 beta
    pairs = [(p, r) for p in range(n_sp) for r in range(p, n_sp)]
    idx = {pr: i for i, pr in enumerate(pairs)}
    rng = np.random.default_rng(12)
    X = rng.normal(size=(len(pairs), len(pairs) + 2))
    M = X @ X.T + 0.1 * np.eye(len(pairs))  # positive definite over unordered pairs
    C = np.linalg.cholesky(M)  # M = C C^T, one auxiliary index per column
    n_aux = C.shape[1]
    v_space = oracle.Space.spin_blocked(n_sp, n_sp, 2)  # tiles [2, 1, 2, 1]: ragged
    aux = oracle.Space.fixed(n_aux, 4)  # ragged auxiliary tiles
    n = 2 * n_sp

    def sp(p):
        return p % n_sp

    def pair(p, q):
        a, b = sorted((sp(p), sp(q)))
        return idx[(a, b)]

    dense_b = np.zeros((n, n, n_aux))
    for p in range(n):
        for q in range(n):
            if spin_of(v_space, p) == spin_of(v_space, q):
                dense_b[p, q, :] = C[pair(p, q), :]
    V = v_from_cholesky(cholesky_tensor(v_space, aux, dense_b))
    got = np.zeros((n,) * 4)
    for t in V.stored_tiles():
        got[V.block_slices(t)] = V.blocks[t]
    want = np.zeros((n,) * 4)
    for p, q, r, s in itertools.product(range(n), repeat=4):
        sps = [spin_of(v_space, x) for x in (p, q, r, s)]
        val = 0.0
        if sps[0] == sps[2] and sps[1] == sps[3]:
            val += M[pair(p, r), pair(q, s)]
        if sps[0] == sps[3] and sps[1] == sps[2]:
            val -= M[pair(p, s), pair(q, r)]
        want[p, q, r, s] = val
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("beta", [0.0, 0.7])
@pytest.mark.parametrize("shape", [(10, 5, 6, 3, 9, 4), (12, 4, 8, 4, 7, 7)], ids=["ragged", "even"])
def test_ladder_matches_dense_brute_force(shape, beta):
    n_vir, t_vir, n_occ, t_occ, n_aux, t_aux = shape
    v, o, x = spaces(*shape)
    orb = synth.Orbitals(n_occ, n_vir, n_aux=n_aux)
    Bd = orb.dense("B_vvx", "vvx")
    Td = orb.dense("T2", "vvoo")
    R0 = orb.dense("N_R", "vvoo")
    B = cholesky_tensor(v, x, Bd)
    T = oracle.BlockTensor.from_dense([v, v, o, o], Td)
    R = oracle.BlockTensor.from_dense([v, v, o, o], R0)
    got = cholesky_ladder(R, T, B, 0.5, beta).to_dense()
    dense = np.einsum("acL,bdL,cdij->abij", Bd, Bd, Td, optimize=True)
    dense -= np.einsum("adL,bcL,cdij->abij", Bd, Bd, Td, optimize=True)
    want = 0.5 * dense + beta * R.to_dense()
    mask = np.zeros_like(want, dtype=bool)
    for t in R.stored_tiles():
        mask[R.block_slices(t)] = True
    want[~mask] = 0.0
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_rebuilt_integrals_symmetries():
    v, o, x = spaces(10, 3, 4, 2, 6, 6)
    orb = synth.Orbitals(4, 10, n_aux=6)
    V = v_from_cholesky(cholesky_tensor(v, x, orb.dense("B_vvx", "vvx")))
    d = np.zeros((10,) * 4)
    for t in V.stored_tiles():
        d[V.block_slices(t)] = V.blocks[t]
    tol = 1e-15 * np.max(np.abs(d))
    assert np.max(np.abs(d + np.transpose(d, (0, 1, 3, 2)))) <= tol  # v[abcd] = -v[abdc]
    assert np.max(np.abs(d + np.transpose(d, (1, 0, 2, 3)))) <= tol  # v[abcd] = -v[bacd]
    assert np.max(np.abs(d - np.transpose(d, (1, 0, 3, 2)))) <= tol  # v[abcd] = v[badc]
    assert np.max(np.abs(d - np.transpose(d, (2, 3, 0, 1)))) <= tol  # v[abcd] = v[cdab]
    assert np.max(np.abs(d)) > 0


def test_single_product_vector_special_case():
    v = oracle.Space.spin_blocked(3, 3, 2)
    x = oracle.Space.fixed(1, 1)
    u = np.array([1.0, -2.0, 3.0, 1.0, -2.0, 3.0])
    dense = np.zeros((6, 6, 1))
    for p in range(6):
        for q in range(6):
            if (p < 3) == (q < 3):
                dense[p, q, 0] = u[p] * u[q]
    V = v_from_cholesky(cholesky_tensor(v, x, dense))
    seen = set()
    for t in V.stored_tiles():
        spins = tuple(v.spins[i] for i in t)
        blk = V.blocks[t]
        if len(set(spins)) == 1:
            assert np.array_equal(blk, np.zeros(V.block_shape(t)))
        elif spins == (0, 1, 0, 1):
            ua, ub, uc, ud = (u[v.offsets[i]:v.offsets[i] + v.sizes[i]] for i in t)
            assert np.array_equal(blk, np.einsum("a,b,c,d->abcd", ua, ub, uc, ud))
        seen.add(spins)
    assert {(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 0, 1)} <= seen


def test_pair_product_route_is_the_same_operation():
    n_vir, n_occ, n_aux = 8, 4, 5
    orb = synth.Orbitals(n_occ, n_vir, n_aux=n_aux)
    Bd = orb.dense("B_vvx", "vvx")
    Td = orb.dense("T2", "vvoo")
    v, o, x = spaces(n_vir, 4, n_occ, 2, n_aux, 5)
    ref = cholesky_ladder(oracle.BlockTensor.zeros([v, v, o, o]), oracle.BlockTensor.from_dense([v, v, o, o], Td),
                          cholesky_tensor(v, x, Bd), 0.5, 0.0).to_dense()
    G = np.einsum("acL,bdL->acbd", Bd, Bd)
    Tm = Td - np.transpose(Td, (1, 0, 2, 3))
    alt = 0.5 * np.einsum("acbd,cdij->abij", G, Tm)
    mask = ref != 0
    assert np.max(np.abs(alt[mask] - ref[mask])) <= 1e-14 * np.max(np.abs(ref))


def test_spin_diagonal_rule_and_synthetic_vectors():
    orb = synth.Orbitals(4, 10, n_aux=7)
    B = orb.dense("B_vvx", "vvx")
    na = orb.n_vir_alpha
    assert np.array_equal(B, np.transpose(B, (1, 0, 2)))  # (pq|L) = (qp|L)
    assert np.array_equal(B[:na, :na], B[na:, na:])  # alpha and beta copies of a spatial pair
    assert not np.any(B[:na, na:]) and not np.any(B[na:, :na])  # spin-mixed pairs vanish
    assert spin_diagonal((0, 1, 0), (1, 1, 0)) and not spin_diagonal((0, 1, 0), (0, 1, 0))
    assert abs(np.std(B[:na, :na]) - synth.cholesky_sigma(7)) < 0.3 * synth.cholesky_sigma(7)
