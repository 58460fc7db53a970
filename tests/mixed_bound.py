"""Element-wise error bounds of the mixed-precision contraction paths, derived from their definitions
and from the measured rounding of the matrix-core instructions.

Rounding of one matrix-core instruction D = C + sum_k A_k B_k (measured on crafted inputs whose
exact sums the host knows, tests/test_gpu_mfma_rounding.py):

* bfloat16 instructions (v_mfma_f32_16x16x32_bf16, v_mfma_f32_32x32x16_bf16): the products are
  exact; the accumulator and the products are aligned to the largest of them, every bit more than
  24 places below its leading bit is dropped without a sticky bit (2^12 + 2^-12 - 2^12 keeps
  2^-12, 2^8 + 2^-17 - 2^8 loses 2^-17; 1 - 1 + 2^-30 gives 0), the aligned terms are summed
  exactly (four quarter-ulps add up to one ulp) and the sum is rounded to nearest even once;
* float32 instructions (v_mfma_f32_16x16x4_f32, v_mfma_f32_32x32x2_f32): results as if the
  accumulator and then each product were added by ordinary float32 additions rounded to nearest
  even (four quarter-ulps added to 1 vanish one by one; 1 - 1 + 2^-30 keeps 2^-30).

Either way one instruction with K products is off by at most (K + 2) u M, u = 2^-24, M the largest
magnitude among its terms (each of the K + 1 terms loses less than u M, the final rounding less than
u |D| <= u (K + 1) M is covered by the count since M bounds the running sum it rounds).  Inside a
promotion window of W = 256 summed indices the accumulator and the products are bounded by the
window's sum S_w of |a_k b_k| (of the products that accumulator takes), so an accumulator that runs
n instructions per window is off by at most n (K + 2) u S_w.  With n_w windows per element and the
float64 promotion and epilogue:

  f32:    |err| <= (2u + u^2 + 64 * 6 u + (n_w + 1) 2^-52) S
          -- each operand rounded once (relative u); 64 instructions of 4 products per window.
  bf16x3: |err| <= (4.1 u + 8 * 34 u + 40 * 34 u * 0.0079 + (n_w + 1) 2^-52) S
          -- slices b_i = bf16(...) leave |x - b0 - b1 - b2| <= 2^-24 |x| and |b_i| <= 2^-8i |x|
          (1 + 2^-8), so the dropped products (i + j >= 3, and the remainders) sum to < 4.1 u |ab|;
          b0*b0 runs in its own accumulator (8 instructions of 32 products per window), the five
          products of order 1 and 2 (together <= 0.0079 |ab|) in another (40 per window).
  bf16x4_aligned: |err| <= (1.2e-9 + 72 * 34 u * 0.0079 + (n_w + 1) 2^-52) T
          -- T = sum_k over the (row, window) maxima of |a| and |b|: the lead slices are multiples
          of 2^(E-8) below a window maximum 2^(E-1) <= max < 2^E, their window sums are integers
          times one power of two below 2^24 of it, so aligned and summed exactly; the residual
          |x - lead| <= 2^-8 max is split in three bfloat16 slices (remainder <= 2^-32 max);
          dropped products of order >= 4 and remainders < 5 * 2^-32; the nine residual products
          (together <= 0.0079 max_a max_b) run 72 instructions per window.

S = sum_k |a_k| |b_k| is the same contraction on |lhs|, |rhs| (times |alpha|); T is it on operands
whose elements are replaced by their (row, window) maximum magnitude, windows as the header of the
library defines them (the flattening order of oracle.split, a specification of that layout).

These are worst-case bounds: they catch a wrong slice or a dropped product of order one (2^-8
relative), not the statistical size of the rounding error, which the tests bound separately with
the relative Frobenius error of each precision.
"""

from __future__ import annotations

import numpy as np

import oracle
from oracle import split as osplit

U = 2.0 ** -24
WINDOW = osplit.WINDOW


def step(K: int) -> float:
    """Worst-case error of one matrix-core instruction with K products, relative to its largest term."""
    return (K + 2) * U


def coefficient(precision: str, n_windows: int) -> float:
    f64 = (n_windows + 1) * 2.0 ** -52
    if precision == "f32":
        return 2 * U + U * U + (WINDOW // 4) * step(4) + f64
    if precision == "bf16x3":
        return 4.1 * U + (WINDOW // 32) * step(32) + 5 * (WINDOW // 32) * step(32) * 0.0079 + f64
    if precision == "bf16x4_aligned":
        return 1.2e-9 + 9 * (WINDOW // 32) * step(32) * 0.0079 + f64
    raise ValueError(precision)


def window_max(block: np.ndarray, block_lbl: str, k_order: str) -> np.ndarray:
    """Each element replaced by the largest magnitude of its (row, window) in the split layout."""
    row_lbl = [c for c in block_lbl if c not in k_order]
    perm = [block_lbl.index(c) for c in row_lbl] + [block_lbl.index(c) for c in k_order]
    t = np.abs(np.transpose(block, perm))
    rows = int(np.prod([t.shape[i] for i in range(len(row_lbl))], dtype=np.int64))
    flat = t.reshape(rows, -1)
    out = np.empty_like(flat)
    for k0 in range(0, flat.shape[1], WINDOW):
        w = flat[:, k0:k0 + WINDOW]
        out[:, k0:k0 + WINDOW] = np.max(w, axis=1, keepdims=True) if w.size else 0.0
    return np.transpose(out.reshape(t.shape), np.argsort(perm))


class _Mapped(dict):
    """Block dictionary applying ``fn`` to the blocks of another (lazily, cached)."""

    def __init__(self, src, fn):
        super().__init__()
        self._src, self._fn = src, fn

    def __missing__(self, key):
        v = self._fn(key, self._src[key])
        self[key] = v
        return v


def _mapped(t: oracle.BlockTensor, fn) -> oracle.BlockTensor:
    x = oracle.BlockTensor(t.spaces, t.nonzero)
    x.blocks = _Mapped(t.blocks, fn)
    return x


def bound_blocks(precision, out, ol, lhs, ll, rhs, rl, alpha, tiles):
    """Per sampled output block the element-wise bound (same shape as the block)."""
    k_order = osplit.summed_label_order(ol, ll, rl)
    if precision == "bf16x4_aligned":
        A = _mapped(lhs, lambda t, b: window_max(b, ll, k_order))
        B = _mapped(rhs, lambda t, b: window_max(b, rl, k_order))
    else:
        A = _mapped(lhs, lambda t, b: np.abs(b))
        B = _mapped(rhs, lambda t, b: np.abs(b))
    mag = oracle.contract(out, ol, A, ll, B, rl, abs(alpha), 0.0, out_tiles=tiles).blocks
    # windows per element: the summed extent of the element's surviving pairs, in windows
    scr = oracle.screen(out, ol, lhs, ll, rhs, rl)
    kl = [c for c in ll if c not in ol]
    res = {}
    for t in tiles:
        nw = 0
        for kt in scr["pairs"][t]:
            ext = 1
            for c, ti in zip(kl, kt):
                ext *= lhs.spaces[ll.index(c)].sizes[ti]
            nw += -(-ext // WINDOW)
        res[t] = coefficient(precision, nw) * mag[t]
    return res


def check(got, ref, bound, keys):
    """Largest ratio |got - ref| / bound over the sampled elements (must be <= 1)."""
    worst = 0.0
    for k in keys:
        d = np.abs(got[k] - ref[k])
        b = bound[k]
        if np.any(d > b):
            return float(np.max(d / np.maximum(b, 1e-300)))
        worst = max(worst, float(np.max(d / np.maximum(b, 1e-300))))
    return worst
