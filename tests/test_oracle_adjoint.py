"""Pins of the oracle's adjoint: the dot-product (transpose) identity and central finite differences.

L = 1/2 ||R||^2 with R linear in T (and in each V tensor) is quadratic along any single-element
perturbation, so a central difference is exact up to rounding for any step.
"""

import numpy as np

from oracle import BlockTensor, Space, contract, contract_vjp


def inner(x: BlockTensor, y: BlockTensor) -> float:
    return float(sum(np.vdot(b, y.blocks[t]) for t, b in x.blocks.items()))


def rand_like(x: BlockTensor, rng) -> BlockTensor:
    y = BlockTensor(x.spaces, x.nonzero)
    for t in x.stored_tiles():
        y.blocks[t] = rng.standard_normal(x.block_shape(t))
    return y


def test_dot_product_identity_all_operands():
    rng = np.random.default_rng(21)
    o = Space.spin_blocked(3, 2, 2)
    v = Space.spin_blocked(4, 3, 3)
    V = rand_like(BlockTensor([o, v, v, o]), rng)
    T = rand_like(BlockTensor([v, v, o, o]), rng)
    R0 = rand_like(BlockTensor([v, v, o, o]), rng)
    g = rand_like(R0, rng)
    alpha, beta = 0.8, -0.35
    gV, gT, gR0 = contract_vjp(g, "abij", V, "mbej", T, "aeim", alpha, beta)
    zero = BlockTensor.zeros(R0.spaces)
    dV = rand_like(V, rng)
    dT = rand_like(T, rng)
    dR0 = rand_like(R0, rng)
    # <J_V dV, g> = <dV, gV>, and the same for T and R0
    lhs_v = inner(contract(zero, "abij", dV, "mbej", T, "aeim", alpha, 0.0), g)
    lhs_t = inner(contract(zero, "abij", V, "mbej", dT, "aeim", alpha, 0.0), g)
    lhs_r = inner(contract(dR0, "abij", V, "mbej", T, "aeim", 0.0, beta), g)
    assert abs(lhs_v - inner(dV, gV)) < 1e-12 * max(1.0, abs(lhs_v))
    assert abs(lhs_t - inner(dT, gT)) < 1e-12 * max(1.0, abs(lhs_t))
    assert abs(lhs_r - inner(dR0, gR0)) < 1e-12 * max(1.0, abs(lhs_r))


def loss(Vv, Vr, T, spaces_out):
    zero = BlockTensor.zeros(spaces_out)
    R = contract(zero, "abij", Vv, "abcd", T, "cdij", 0.5, 0.0)
    R = contract(R, "abij", Vr, "mbej", T, "aeim", 1.0, 1.0)
    return 0.5 * sum(float(np.sum(b * b)) for b in R.blocks.values()), R


def test_finite_differences_ladder_plus_ring():
    # the small finite-difference size: O=6 -> [3a,3b], V=16 -> [8a,8b]
    rng = np.random.default_rng(22)
    o = Space.spin_blocked(3, 3, 3)
    v = Space.spin_blocked(8, 8, 8)
    Vv = rand_like(BlockTensor([v] * 4), rng)
    Vr = rand_like(BlockTensor([o, v, v, o]), rng)
    T = rand_like(BlockTensor([v, v, o, o]), rng)
    out_spaces = [v, v, o, o]
    L0, R = loss(Vv, Vr, T, out_spaces)
    gVv, gT1, _ = contract_vjp(R, "abij", Vv, "abcd", T, "cdij", 0.5, 0.0)
    gVr, gT2, _ = contract_vjp(R, "abij", Vr, "mbej", T, "aeim", 1.0, 1.0)
    h = 1e-3
    # every element of T (both terms contribute)
    checked = 0
    for t, blk in T.blocks.items():
        for idx in np.ndindex(blk.shape):
            old = blk[idx]
            blk[idx] = old + h
            lp, _ = loss(Vv, Vr, T, out_spaces)
            blk[idx] = old - h
            lm, _ = loss(Vv, Vr, T, out_spaces)
            blk[idx] = old
            fd = (lp - lm) / (2 * h)
            an = gT1.blocks[t][idx] + gT2.blocks[t][idx]
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
            checked += 1
            if checked >= 300:
                break
        if checked >= 300:
            break
    # a seeded subset of V_vvvv elements
    keys = list(Vv.blocks)
    for n in range(40):
        t = keys[int(rng.integers(0, len(keys)))]
        blk = Vv.blocks[t]
        idx = tuple(int(rng.integers(0, s)) for s in blk.shape)
        old = blk[idx]
        blk[idx] = old + h
        lp, _ = loss(Vv, Vr, T, out_spaces)
        blk[idx] = old - h
        lm, _ = loss(Vv, Vr, T, out_spaces)
        blk[idx] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gVv.blocks[t][idx]) <= 1e-7 * max(1.0, abs(gVv.blocks[t][idx]))
    assert checked == 300
