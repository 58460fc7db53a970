"""Pin of the oracle's doubles iteration (oracle/iteration.py) against the same equations written
densely with numpy.einsum on zero-filled tensors: the block-sparse sequence (contractions, the
P(ij)P(ab) permuted additions, the denominator update) must reproduce the dense result, and the
antisymmetrised part must have the antisymmetry it is built to have."""

import numpy as np

from oracle import BlockTensor, Space
from oracle.iteration import INTERMEDIATES, doubles_iteration


def test_doubles_iteration_matches_dense_equations():
    rng = np.random.default_rng(31)
    o = Space.spin_blocked(2, 3, 2)   # uneven halves and remainder tiles
    v = Space.spin_blocked(3, 4, 2)
    sp = {"o": o, "v": v}
    pats = {"V_vvvv": "vvvv", "V_ovvo": "ovvo", "V_oovv": "oovv", "V_vvvo": "vvvo", "V_ovoo": "ovoo",
            "T2": "vvoo", "T1": "vo"}
    t, d = {}, {}
    for name, p in pats.items():
        spaces = [sp[c] for c in p]
        x = BlockTensor.from_dense(spaces, rng.standard_normal(tuple(s.extent for s in spaces)))
        t[name], d[name] = x, x.to_dense()
    for name, p in INTERMEDIATES.items():
        t[name] = BlockTensor.zeros([sp[c] for c in p])
    e_o = rng.uniform(-2, -0.5, o.extent)
    e_v = rng.uniform(0.2, 3, v.extent)
    res = doubles_iteration(t, e_o, e_v)

    W = 0.5 * np.einsum("mnef,efij->mnij", d["V_oovv"], d["T2"])
    R = 0.5 * np.einsum("abcd,cdij->abij", d["V_vvvv"], d["T2"]) + 0.5 * np.einsum("mnij,abmn->abij", W, d["T2"])
    X = np.einsum("mbej,aeim->abij", d["V_ovvo"], d["T2"])
    Zv = np.einsum("abej,ei->abij", d["V_vvvo"], d["T1"])
    Zo = -np.einsum("mbij,am->abij", d["V_ovoo"], d["T1"])
    swap_ij = (0, 1, 3, 2)
    swap_ab = (1, 0, 2, 3)
    R = R + X - X.transpose(swap_ij) - X.transpose(swap_ab) + X.transpose(swap_ij).transpose(swap_ab)
    R = R + Zv - Zv.transpose(swap_ij) + Zo - Zo.transpose(swap_ab)
    D = e_o[None, None, :, None] + e_o[None, None, None, :] - e_v[:, None, None, None] - e_v[None, :, None, None]
    mask = BlockTensor.from_dense([v, v, o, o], np.ones(R.shape)).to_dense()
    T2n = mask * R / D

    def rel(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)

    assert rel(res["W"].to_dense(), W) < 1e-13
    assert rel(res["R"].to_dense(), mask * R) < 1e-13
    assert rel(res["T2"].to_dense(), T2n) < 1e-13
    # the ring part alone is antisymmetric in (i,j) and in (a,b)
    Xa = X - X.transpose(swap_ij) - X.transpose(swap_ab) + X.transpose(swap_ij).transpose(swap_ab)
    assert np.allclose(Xa, -Xa.transpose(swap_ij), atol=1e-14) and np.allclose(Xa, -Xa.transpose(swap_ab), atol=1e-14)
