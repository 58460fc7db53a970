"""Pin of the oracle on the complex-by-real ladder in its rank-5 real form (interleaved (re, im) as a
trailing dimension): against NumPy's complex product of the dense arrays, an independent route."""

import numpy as np

import oracle
from paper_2201_01257_amd import synth


def test_rank5_real_form_equals_complex_product():
    orb = synth.Orbitals(8, 12)

    def spin4(t, s):
        return s[0] + s[1] == s[2] + s[3]

    sp = {"o": oracle.Space.spin_blocked(4, 4, 3), "v": oracle.Space.spin_blocked(6, 6, 4), "z": oracle.Space.fixed(2, 2)}

    def box(pat, t):
        return [sp[c].offsets[t[d]] for d, c in enumerate(pat)], [sp[c].sizes[t[d]] for d, c in enumerate(pat)]

    V = oracle.BlockTensor([sp["v"]] * 4)
    V.blocks = oracle.LazyBlocks(lambda t: orb.fill("V_vvvv", "vvvv", *box("vvvv", t)))
    T = oracle.BlockTensor([sp[c] for c in "vvooz"], spin4)
    T.blocks = oracle.LazyBlocks(lambda t: synth.fill_complex(orb, "T2", "N_T2im", "vvoo", *box("vvooz", t)))
    R = oracle.BlockTensor([sp[c] for c in "vvooz"], spin4)
    res = oracle.contract(R, "abijz", V, "abcd", T, "cdijz", 0.5, 0.0)
    Tc = orb.dense("T2", "vvoo") + 1j * orb.dense("N_T2im", "vvoo")
    ref = 0.5 * np.einsum("abcd,cdij->abij", orb.dense("V_vvvv", "vvvv"), Tc)
    got = np.zeros(ref.shape + (2,))
    for t, b in res.blocks.items():
        lo, ext = box("vvooz", t)
        got[tuple(slice(l, l + e) for l, e in zip(lo, ext))] = b
    assert np.allclose(got[..., 0] + 1j * got[..., 1], ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    assert np.count_nonzero(ref.imag) > 0 and np.count_nonzero(ref.real) > 0
