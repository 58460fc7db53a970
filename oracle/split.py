"""Operand splits of the split-bfloat16 contraction paths, written from their definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in float64, one operand block
at a time; no code is shared with the HIP path.

The paper computes in float64 only; these splits belong to the mixed-precision extension of the
contraction, defined as follows (every narrowing rounds to nearest, ties to even):

* ``round_bf16(x)``: x rounded to 8 significant bits (the bfloat16 precision); magnitudes below
  2^-100 become zero.
* plain three-way split: ``b0 = round_bf16(x)``, ``b1 = round_bf16(x - b0)``,
  ``b2 = round_bf16(x - b0 - b1)``.
* aligned split: within one window (a row of an operand block and 256 consecutive flattened
  summed indices), with ``m`` the largest magnitude and ``E`` the exponent with
  ``2^(E-1) <= m < 2^E``, the lead is ``x`` rounded to a multiple of ``2^(E-8)`` (an integer of
  magnitude at most 256 times that power of two); the residual ``x - lead`` is split into three
  slices as in the plain split.  A window whose values are all zero splits into zeros.
* the flattened summed indices of a block run over the summed labels in the dimension order of
  the operand that does not hold the output's last label, unless only the other operand has a
  summed label as its last dimension (then in that operand's order); the last label varies
  fastest.  A row is one value of the operand's remaining labels.

The result of a split is given as one 64-bit word per element: slice s as bfloat16 bits in bits
16s..16s+15.

Pins (tests/test_oracle_split.py): ties and carries of the rounding against an independent
integer route on float32 bit patterns; reconstruction bounds of both splits (closed forms);
exactness of the lead slice in bfloat16; window boundaries; the flattening-order rule on the
contraction shapes of the doubles terms.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np

WINDOW = 256
FLUSH = 2.0 ** -100


def round_bf16(x: np.ndarray) -> np.ndarray:
    """x rounded to 8 significant bits, to nearest even; |x| < 2^-100 gives zero."""
    x = np.asarray(x, dtype=np.float64)
    f, e = np.frexp(x)                     # x = f * 2^e with 0.5 <= |f| < 1
    q = np.ldexp(np.ones_like(x), e - 8)   # 8 significant bits: the quantum is 2^(e-8)
    r = np.rint(x / q) * q                 # exact scaling, round half to even
    return np.where(np.abs(x) < FLUSH, 0.0, r)


def bf16_bits(y: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns of values that bfloat16 represents exactly."""
    f = np.asarray(y, dtype=np.float64).astype(np.float32)
    return (f.view(np.uint32) >> np.uint32(16)).astype(np.uint64)


def _pack(slices: Sequence[np.ndarray]) -> np.ndarray:
    w = np.zeros(np.shape(slices[0]), dtype=np.uint64)
    for s, v in enumerate(slices):
        w |= bf16_bits(v) << np.uint64(16 * s)
    return w


def split_plain(x: np.ndarray) -> np.ndarray:
    """Three-slice split of every element, packed."""
    x = np.asarray(x, dtype=np.float64)
    b0 = round_bf16(x)
    r1 = x - b0
    b1 = round_bf16(r1)
    b2 = round_bf16(r1 - b1)
    return _pack([b0, b1, b2])


def split_aligned_rows(x: np.ndarray) -> np.ndarray:
    """Aligned split of a [rows][k] array, windows of WINDOW along k in each row, packed."""
    x = np.asarray(x, dtype=np.float64)
    rows, kext = x.shape
    out = np.zeros((rows, kext), dtype=np.uint64)
    for k0 in range(0, kext, WINDOW):
        w = x[:, k0:k0 + WINDOW]
        m = np.max(np.abs(w), axis=1, keepdims=True) if w.size else np.zeros((rows, 1))
        _, e = np.frexp(m)                                  # 2^(e-1) <= m < 2^e
        q = np.ldexp(np.ones_like(m), e - 8)
        lead = np.where(m > 0, np.rint(w / q) * q, 0.0)
        r = w - lead
        s1 = round_bf16(r)
        r2 = r - s1
        s2 = round_bf16(r2)
        s3 = round_bf16(r2 - s2)
        out[:, k0:k0 + WINDOW] = _pack([lead, s1, s2, s3])
    return out


def summed_label_order(out_lbl: str, lhs_lbl: str, rhs_lbl: str) -> str:
    """The flattening order of the summed labels (see the module docstring)."""
    last = out_lbl[-1]
    a, b = (rhs_lbl, lhs_lbl) if last in lhs_lbl else (lhs_lbl, rhs_lbl)
    summed = lambda lbl: [c for c in lbl if c not in out_lbl]  # noqa: E731
    a_last_summed, b_last_summed = a[-1] not in out_lbl, b[-1] not in out_lbl
    return "".join(summed(b) if (not a_last_summed and b_last_summed) else summed(a))


def split_block(block: np.ndarray, block_lbl: str, k_order: str, aligned: bool) -> np.ndarray:
    """Packed split words of one operand block (array in its own label order), same shape."""
    row_lbl = [c for c in block_lbl if c not in k_order]
    perm = [block_lbl.index(c) for c in row_lbl] + [block_lbl.index(c) for c in k_order]
    t = np.transpose(block, perm)
    rows = int(np.prod([t.shape[i] for i in range(len(row_lbl))], dtype=np.int64))
    kext = int(np.prod(t.shape[len(row_lbl):], dtype=np.int64))
    flat = t.reshape(rows, kext)
    words = split_aligned_rows(flat) if aligned else split_plain(flat)
    return np.transpose(words.reshape(t.shape), np.argsort(perm))
