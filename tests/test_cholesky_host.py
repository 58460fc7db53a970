"""Host-only checks (no GPU) of row views and of the Cholesky-vector ladder's plans: the view's
blocks are the parent's rows at the parent's offsets, and the useful flops of the pair products
and strip ladders equal counts taken straight from the spin rules (B spin-diagonal: G[a,c,b,d]
needs s_a = s_c and s_b = s_d; T and R conserve spin), summed tile by tile here."""

import itertools

import numpy as np
import pytest

from paper_2201_01257_amd import core as tm


def test_row_view_is_the_parents_rows():
    o = tm.Space.spin(3, 2, 2)
    v = tm.Space.spin(4, 5, 3)
    T = tm.Tensor([v, v, o, o], device=None)
    for lo, hi in [(0, 1), (1, 3), (2, v.ntiles), (0, v.ntiles)]:
        V = T.view_rows(lo, hi)
        rows = [b for b in range(T.nblocks) if lo <= T.block_tiles[b][0] < hi]
        assert V.nblocks == len(rows)
        base = int(T.block_off[rows[0]])
        assert V.view_base == base
        assert np.array_equal(V.block_off, T.block_off[rows] - base)
        shifted = T.block_tiles[rows].copy()
        shifted[:, 0] -= lo
        assert np.array_equal(V.block_tiles, shifted)
        end = int(T.block_off[rows[-1]]) + int(np.prod(T.block_lo_ext(rows[-1])[1]))
        assert V.numel == end - base
        assert list(V.spaces[0].sizes) == list(v.sizes[lo:hi])


def test_row_view_rejects_bad_ranges():
    v = tm.Space.spin(4, 4, 2)
    T = tm.Tensor([v, v], device=None)
    for lo, hi in [(-1, 1), (2, 2), (3, 1), (0, v.ntiles + 1)]:
        with pytest.raises(tm.TammError):
            T.view_rows(lo, hi)


def expected_flops(v, o, aux, strip_tiles):
    nv = v.ntiles
    build = ladder = 0
    for ta, tc, tb, td in itertools.product(range(nv), repeat=4):
        if v.spins[ta] == v.spins[tc] and v.spins[tb] == v.spins[td]:
            build += 2 * v.sizes[ta] * v.sizes[tc] * v.sizes[tb] * v.sizes[td] * aux.extent
    for ta, tb, ti, tj in itertools.product(range(nv), range(nv), range(o.ntiles), range(o.ntiles)):
        if v.spins[ta] + v.spins[tb] != o.spins[ti] + o.spins[tj]:
            continue  # R block not stored
        for tc, td in itertools.product(range(nv), repeat=2):
            if v.spins[tc] != v.spins[ta] or v.spins[td] != v.spins[tb]:
                continue  # G block not stored
            if v.spins[tc] + v.spins[td] != o.spins[ti] + o.spins[tj]:
                continue  # T block not stored
            ladder += 2 * v.sizes[ta] * v.sizes[tb] * v.sizes[tc] * v.sizes[td] * o.sizes[ti] * o.sizes[tj]
    strips = -(-nv // max(strip_tiles, 1))
    return build, ladder, strips


@pytest.mark.parametrize("strip_tiles", [0, 1, 2, 5])
@pytest.mark.parametrize("shape", [(20, 40, 5, 8, 13, 5), (40, 200, 40, 40, 755, 755)], ids=["ragged", "bench"])
def test_plan_flops_from_spin_rules(shape, strip_tiles):
    n_occ, n_vir, t_occ, t_vir, n_aux, t_aux = shape
    o = tm.Space.spin(n_occ // 2, n_occ - n_occ // 2, t_occ)
    v = tm.Space.spin(n_vir // 2, n_vir - n_vir // 2, t_vir)
    x = tm.Space.fixed(n_aux, t_aux)
    R = tm.Tensor([v, v, o, o], device=None)
    T = tm.Tensor([v, v, o, o], device=None)
    B = tm.Tensor([v, v, x], nonzero=tm.spin_diagonal, device=None)
    c = tm.CholeskyLadder(R, T, B, strip_tiles=strip_tiles)
    st = c.stats()
    build, ladder, strips = expected_flops(v, o, x, strip_tiles)
    assert (st["build_flops"], st["ladder_flops"], st["strips"]) == (build, ladder, strips)
    assert st["tm_elements"] == T.numel
    # the largest strip of G: s_a = s_c and s_b = s_d blocks of the strip's a tiles
    per = max(strip_tiles, 1)
    gmax = 0
    for lo in range(0, v.ntiles, per):
        n = 0
        for ta in range(lo, min(lo + per, v.ntiles)):
            for tc, tb, td in itertools.product(range(v.ntiles), repeat=3):
                if v.spins[ta] == v.spins[tc] and v.spins[tb] == v.spins[td]:
                    n += v.sizes[ta] * v.sizes[tc] * v.sizes[tb] * v.sizes[td]
        gmax = max(gmax, n)
    assert st["g_max_elements"] == gmax


def test_rejects_mismatched_spaces():
    o = tm.Space.spin(2, 2, 2)
    v = tm.Space.spin(4, 4, 2)
    w = tm.Space.spin(4, 4, 3)
    x = tm.Space.fixed(5, 5)
    R = tm.Tensor([v, v, o, o], device=None)
    with pytest.raises(tm.TammError):
        tm.CholeskyLadder(R, tm.Tensor([w, w, o, o], device=None), tm.Tensor([v, v, x], nonzero=tm.spin_diagonal, device=None))
    with pytest.raises(tm.TammError):
        tm.CholeskyLadder(R, tm.Tensor([v, v, o, o], device=None), tm.Tensor([v, v, x, x], device=None))
