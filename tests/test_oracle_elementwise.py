"""Pins of the oracle's SetOp and AddOp (Sec. III-A, Fig. 3 rules 5-7) against dense numpy:
permuted addition equals ``beta*out + alpha*transpose(in)`` on zero-filled dense tensors masked to
out's stored blocks, for every permutation of rank 2-4 and for block rules under which a permuted
block is not stored; P(ij)P(ab) antisymmetrisation gives an antisymmetric result; ``=`` never
reads out."""

import itertools

import numpy as np
import pytest

from oracle import BlockTensor, Space, add, set_value


def masked(spaces, dense, nonzero=None):
    return BlockTensor.from_dense(spaces, dense, nonzero).to_dense()


@pytest.mark.parametrize("rank", [2, 3, 4])
def test_add_every_permutation_matches_dense_transpose(rank):
    rng = np.random.default_rng(40 + rank)
    spaces = [Space.spin_blocked(int(rng.integers(1, 5)), int(rng.integers(1, 5)), int(rng.integers(1, 4)))
              for _ in range(rank)]
    letters = "abcd"[:rank]
    for perm in itertools.permutations(range(rank)):
        in_lbl = "".join(letters[p] for p in perm)
        in_spaces = [spaces[letters.index(c)] for c in in_lbl]
        inp = BlockTensor.from_dense(in_spaces, rng.standard_normal(tuple(s.extent for s in in_spaces)))
        out = BlockTensor.from_dense(spaces, rng.standard_normal(tuple(s.extent for s in spaces)))
        got = add(out, letters, inp, in_lbl, -0.625, 1.5).to_dense()
        ref = 1.5 * out.to_dense() + -0.625 * np.einsum(f"{in_lbl}->{letters}", inp.to_dense())
        assert np.allclose(got, masked(spaces, ref), rtol=0, atol=1e-15)


def test_add_reads_unstored_in_blocks_as_zero():
    # out stored by the spin rule on (a,b,i,j); in over (a,i,b,j) is stored by the spin rule on
    # its own order, so some permuted blocks are missing: those contribute nothing
    rng = np.random.default_rng(5)
    o = Space.spin_blocked(2, 3, 2)
    v = Space.spin_blocked(3, 2, 2)
    out = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((5, 5, 5, 5)))
    inp = BlockTensor.from_dense([v, o, v, o], rng.standard_normal((5, 5, 5, 5)))
    assert any(not inp.is_stored((t[0], t[2], t[1], t[3])) for t in out.stored_tiles())
    got = add(out, "abij", inp, "aibj", 2.0, 0.0).to_dense()
    ref = 2.0 * np.einsum("aibj->abij", inp.to_dense())
    assert np.array_equal(got, masked(out.spaces, ref))


def test_antisymmetriser_gives_antisymmetric_result():
    rng = np.random.default_rng(6)
    o = Space.spin_blocked(2, 2, 1)
    v = Space.spin_blocked(3, 2, 2)
    X = BlockTensor.from_dense([v, v, o, o], rng.standard_normal((5, 5, 4, 4)))
    R = set_value(BlockTensor.zeros([v, v, o, o]), 0.0)
    for lbl, s in (("abij", 1.0), ("abji", -1.0), ("baij", -1.0), ("baji", 1.0)):
        R = add(R, "abij", X, lbl, s, 1.0)
    Rd = R.to_dense()
    assert np.linalg.norm(Rd) > 0
    assert np.allclose(Rd, -np.transpose(Rd, (0, 1, 3, 2)), rtol=0, atol=1e-14)
    assert np.allclose(Rd, -np.transpose(Rd, (1, 0, 2, 3)), rtol=0, atol=1e-14)


def test_set_and_assignment_semantics():
    rng = np.random.default_rng(7)
    o = Space.spin_blocked(2, 2, 2)
    v = Space.spin_blocked(2, 3, 2)
    out = BlockTensor.from_dense([v, o], rng.standard_normal((5, 4)))
    s = set_value(out, -3.5)
    assert sorted(s.blocks) == sorted(out.stored_tiles())
    assert all(np.all(b == -3.5) for b in s.blocks.values())
    nan = BlockTensor.zeros([v, o])
    nan.blocks = {t: np.full_like(b, np.nan) for t, b in nan.blocks.items()}
    inp = BlockTensor.from_dense([v, o], rng.standard_normal((5, 4)))
    got = add(nan, "ai", inp, "ai", 1.0, 0.0)                       # "=" never reads out
    assert np.array_equal(got.to_dense(), inp.to_dense())
    zero = add(inp, "ai", inp, "ai", -1.0, 1.0)                     # B -= B
    assert all(np.all(b == 0.0) for b in zero.blocks.values())


def test_add_label_errors():
    o = Space.spin_blocked(2, 2, 2)
    v = Space.spin_blocked(2, 3, 2)
    x = BlockTensor.zeros([v, o])
    with pytest.raises(ValueError):
        add(x, "ai", x, "aj", 1.0, 0.0)      # not a permutation
    with pytest.raises(ValueError):
        add(x, "ai", x, "ia", 1.0, 0.0)      # a binds v in out and o in in
