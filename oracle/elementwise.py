"""SetOp and AddOp of the operation grammar (oracle side; test infrastructure only).

arXiv 2201.01257, Sec. III-A, Fig. 3 and the SetOp / AddOp lines of Fig. 4:

* SetOp (rule 5), ``A(i,l) = alpha``: every element of the tensor takes the value alpha.  On a
  block-sparse tensor only the stored blocks exist, so only they are assigned.
* AddOp (rules 6-7), ``B(i,l) = A(i,l)``, ``B(i,l) += alpha * A(i,l)`` and the addition with a
  label permutation ``A(i,l) += alpha * D(l,i)``:

      out[L_out] <- beta * out[L_out] + alpha * in[L_in],   L_in a permutation of L_out,

  element by element over the stored blocks of out; a block of ``in`` that is not stored is zero.
  ``beta == 0`` (the ``=`` form) never reads out.

Plain loops over the stored blocks of out with one ``numpy.transpose`` per block.
"""

from __future__ import annotations

import numpy as np

from .blocksparse import BlockTensor


def set_value(out: BlockTensor, alpha: float) -> BlockTensor:
    """A new tensor with out's structure whose stored elements all equal alpha."""
    res = BlockTensor(out.spaces, out.nonzero)
    for t in out.stored_tiles():
        res.blocks[t] = np.full(out.block_shape(t), float(alpha))
    return res


def add(out: BlockTensor, out_lbl: str, inp: BlockTensor, in_lbl: str, alpha: float = 1.0,
        beta: float = 0.0) -> BlockTensor:
    """Return beta * out + alpha * inp read through the label permutation, on out's stored blocks."""
    if sorted(out_lbl) != sorted(in_lbl) or len(set(out_lbl)) != len(out_lbl):
        raise ValueError(f"{in_lbl!r} is not a permutation of {out_lbl!r}")
    if len(out_lbl) != out.rank or len(in_lbl) != inp.rank:
        raise ValueError("label strings must match the tensor ranks")
    for d, c in enumerate(out_lbl):
        a, b = out.spaces[d], inp.spaces[in_lbl.index(c)]
        if a.sizes != b.sizes or a.spins != b.spins:
            raise ValueError(f"label {c!r} binds two different tiled spaces")
    # axes[d] = dimension of in that holds out's label d: transposing in's block by it gives out's order
    axes = [in_lbl.index(c) for c in out_lbl]
    res = BlockTensor(out.spaces, out.nonzero)
    for ot in out.stored_tiles():
        it = tuple(ot[out_lbl.index(c)] for c in in_lbl)
        x = np.transpose(inp.blocks[it], axes) if inp.is_stored(it) else np.zeros(out.block_shape(ot))
        res.blocks[ot] = alpha * x if beta == 0.0 else beta * out.blocks[ot] + alpha * x
    return res
