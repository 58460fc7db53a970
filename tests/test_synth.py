"""The shared input generator: determinism, tiling independence, stated distributions and symmetries."""

import numpy as np
import pytest

from paper_2201_01257_amd import synth


def test_build_and_determinism():
    synth.build_library()
    a = synth.Orbitals(10, 40)
    b = synth.Orbitals(10, 40)
    assert np.array_equal(a.e_occ, b.e_occ) and np.array_equal(a.e_vir, b.e_vir)
    assert np.array_equal(a.dense("V_vvvv", "vvvv"), b.dense("V_vvvv", "vvvv"))
    c = synth.Orbitals(10, 40, seed=7)
    assert not np.array_equal(a.e_occ, c.e_occ)


def test_energy_ranges():
    o = synth.Orbitals(400, 2000)
    assert o.e_occ.min() >= -2.0 and o.e_occ.max() < -0.5
    assert o.e_vir.min() >= 0.2 and o.e_vir.max() < 3.0
    assert abs(o.e_occ.mean() - (-1.25)) < 0.05 and abs(o.e_vir.mean() - 1.6) < 0.05


def test_boxes_are_slices_of_the_dense_tensor():
    o = synth.Orbitals(6, 10)
    for name, pat in (("V_vvvv", "vvvv"), ("V_ovvo", "ovvo"), ("T2", "vvoo"), ("T1", "vo"), ("N_W_oooo", "oooo")):
        d = o.dense(name, pat)
        lo = [1] * len(pat)
        ext = [min(3, o.extent(c) - 1) for c in pat]
        box = o.fill(name, pat, lo, ext)
        sl = tuple(slice(l, l + e) for l, e in zip(lo, ext))
        assert np.array_equal(box, d[sl])


def test_spin_zeros_and_symmetries():
    o = synth.Orbitals(6, 8)
    V = o.dense("V_vvvv", "vvvv")
    assert np.array_equal(V, V.transpose(1, 0, 3, 2))
    assert np.array_equal(V, V.transpose(2, 3, 0, 1))
    Voo = o.dense("V_oovv", "oovv")
    assert np.array_equal(Voo, Voo.transpose(1, 0, 3, 2))
    Vr = o.dense("V_ovvo", "ovvo")
    assert np.array_equal(Vr, Vr.transpose(3, 2, 1, 0))
    s_v = (np.arange(8) >= 4).astype(int)
    s_o = (np.arange(6) >= 3).astype(int)
    allowed = (s_v[:, None, None, None] + s_v[None, :, None, None]) == (s_v[None, None, :, None] + s_v[None, None, None, :])
    assert np.all(V[~allowed] == 0.0) and np.all(V[allowed] != 0.0)
    T1 = o.dense("T1", "vo")
    assert np.all(T1[s_v[:, None] != s_o[None, :]] == 0.0)


def test_amplitudes_are_normal_over_denominator():
    o = synth.Orbitals(4, 6)
    T = o.dense("T2", "vvoo")
    for (c, d, i, j) in [(0, 1, 0, 1), (3, 4, 0, 3), (5, 5, 3, 3)]:
        if T[c, d, i, j] == 0.0:
            continue
        lin = ((c * 6 + d) * 4 + i) * 4 + j
        w = synth.SIGMA * synth.normal_at(o.seed, "T2", lin)
        den = o.e_occ[i] + o.e_occ[j] - o.e_vir[c] - o.e_vir[d]
        assert T[c, d, i, j] == w / den


def test_stated_normal_statistics():
    o = synth.Orbitals(20, 40)
    x = o.dense("N_stats", "vvoo")
    x = x[x != 0.0]
    assert abs(x.mean()) < 0.01 * 0.1 * 5 and abs(x.std() - 0.1) < 0.003
    V = o.dense("V_vvvv", "vvvv")
    v = V[V != 0.0]
    assert abs(v.std() - 0.1) < 0.003


def test_batched_workload_ranges():
    probs = synth.batched_problems()
    assert len(probs) == 256
    for p in probs:
        assert 8 <= p["n_occ"] <= 48 and p["n_occ"] % 2 == 0
        assert 32 <= p["n_vir"] <= 160 and p["n_vir"] % 2 == 0
        assert p["tile_occ"] in (16, 24, 32, 48, 64) and p["tile_vir"] in (16, 24, 32, 48, 64)
        assert p["term"] in synth.TERMS
    assert probs == synth.batched_problems()


def test_bad_boxes_rejected():
    o = synth.Orbitals(4, 6)
    with pytest.raises(ValueError):
        o.fill("V_vvvv", "vvvv", [0, 0, 0, 5], [1, 1, 1, 2])
    with pytest.raises(ValueError):
        o.fill("T2", "vvvv", [0] * 4, [1] * 4)
