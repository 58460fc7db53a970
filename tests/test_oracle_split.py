"""Pins of the oracle's operand splits (oracle/split.py) against what the definitions fix.

* the rounding to 8 significant bits against an independent route: round to nearest even on the
  integer bit pattern of float32 values (ties of both parities, carries into the exponent);
* flushing below 2^-100;
* reconstruction bounds (closed forms): three plain slices leave at most 2^-24 |x|; the aligned
  lead leaves at most half its quantum 2^(E-9), and three more slices at most 2^(E-33);
* the lead slice is an integer of magnitude <= 256 times 2^(E-8) and exact in bfloat16;
* window boundaries: every 256-long run of a row takes its own maximum;
* the flattening order of the summed labels, both branches of its rule.
"""

import numpy as np
import pytest

from oracle import split as osp


def decode(words, s):
    """Slice s of packed words as float64 values."""
    bits = ((np.asarray(words, dtype=np.uint64) >> np.uint64(16 * s)) & np.uint64(0xFFFF)).astype(np.uint32)
    return (bits << np.uint32(16)).view(np.float32).astype(np.float64)


def rne_bf16_from_f32_bits(x32):
    """Independent route: round to nearest even on the float32 bit pattern (finite values)."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_rounding_matches_integer_route_on_float32_values():
    rng = np.random.default_rng(1)
    x32 = (rng.standard_normal(200000) * np.exp2(rng.integers(-60, 60, 200000))).astype(np.float32)
    # ties of both parities: low 16 bits exactly 0x8000 with bit 16 clear and set
    hi = rng.integers(0x3F800000 >> 16, 0x4F000000 >> 16, 4000).astype(np.uint32)
    ties = ((hi << np.uint32(16)) | np.uint32(0x8000)).view(np.float32)
    x32 = np.concatenate([x32, ties, -ties])
    assert np.array_equal(osp.round_bf16(x32.astype(np.float64)), rne_bf16_from_f32_bits(x32))


def test_rounding_ties_carries_and_flush():
    r = osp.round_bf16(np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 2 - 2.0 ** -9, -(1 + 2.0 ** -8),
                                 2.0 ** -101, -(2.0 ** -101), 2.0 ** -100, 0.0]))
    assert list(r) == [1.0, 1 + 2.0 ** -6, 2.0, -1.0, 0.0, 0.0, 2.0 ** -100, 0.0]


def test_plain_split_reconstruction_bound():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(100000) * np.exp2(rng.integers(-40, 40, 100000))
    w = osp.split_plain(x)
    s = [decode(w, k) for k in range(3)]
    assert np.array_equal(decode(w, 3), np.zeros_like(x))
    assert np.array_equal(s[0], osp.round_bf16(x))
    assert np.all(np.abs(x - (s[0] + s[1] + s[2])) <= 2.0 ** -24 * np.abs(x))


def test_aligned_split_lead_exactness_and_reconstruction():
    rng = np.random.default_rng(3)
    rows, kext = 37, 700  # windows of 256, 256 and a ragged 188
    x = rng.standard_normal((rows, kext)) * np.exp2(rng.integers(-20, 20, (rows, 1)))
    x[5, 300] = 1e6        # one large value: its window's grid is coarse
    x[9, :] = 0.0          # an all-zero row
    w = osp.split_aligned_rows(x)
    s = [decode(w, k) for k in range(4)]
    for k0 in range(0, kext, 256):
        win = slice(k0, k0 + 256)
        m = np.max(np.abs(x[:, win]), axis=1, keepdims=True)
        _, e = np.frexp(m)
        q = np.ldexp(1.0, e - 8)
        lead = s[0][:, win]
        n = lead / q
        assert np.array_equal(n, np.rint(n)) and np.all(np.abs(n) <= 256)
        assert np.all(np.abs(x[:, win] - lead) <= q / 2)
        total = lead + s[1][:, win] + s[2][:, win] + s[3][:, win]
        assert np.all(np.abs(x[:, win] - total) <= np.ldexp(1.0, e - 33))
    assert np.all(w[9] == 0)
    # window boundaries: row 5 has the large value in its second window only
    assert np.all(s[0][5, 256:512][np.abs(x[5, 256:512]) < 2.0 ** 11] == 0.0)
    assert np.count_nonzero(s[0][5, :256]) > 200


def test_summed_label_order_rule():
    # doubles terms: the operand without the output's last label sets the order
    assert osp.summed_label_order("abij", "abcd", "cdij") == "cd"
    assert osp.summed_label_order("abij", "mbej", "aeim") == "em"
    assert osp.summed_label_order("mnij", "mnef", "efij") == "ef"
    assert osp.summed_label_order("abij", "mnij", "abmn") == "mn"
    assert osp.summed_label_order("abij", "abej", "ei") == "e"
    assert osp.summed_label_order("abij", "mbij", "am") == "m"
    # the other branch: that operand's last label is not summed, the other operand's is
    assert osp.summed_label_order("ab", "cda", "bdc") == "dc"
    assert osp.summed_label_order("ab", "acd", "bdc") == "cd"


def test_split_block_follows_rows_and_flattened_k():
    rng = np.random.default_rng(4)
    blk = rng.standard_normal((3, 5, 7))              # labels "dax": rows a; summed x, d in order "xd"
    got = osp.split_block(blk, "dax", "xd", aligned=True)
    flat = np.transpose(blk, (1, 2, 0)).reshape(5, 21)  # [a][x*3 + d]
    ref = np.transpose(osp.split_aligned_rows(flat).reshape(5, 7, 3), (2, 0, 1))
    assert got.shape == blk.shape and np.array_equal(got, ref)
