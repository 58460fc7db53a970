"""Adjoint (vector-Jacobian product) of the block-sparse contraction (oracle side; tests only).

For ``out = beta * out0 + alpha * contract(lhs, rhs)`` and an upstream gradient ``g`` on the
stored blocks of ``out``:

    d/d lhs  = alpha * contract(g, rhs)   onto lhs's labels and lhs's stored blocks,
    d/d rhs  = alpha * contract(lhs, g)   onto rhs's labels and rhs's stored blocks,
    d/d out0 = beta * g.

Both are contractions of the same form as the forward one (each label still occurs in
exactly two tensors), so they reuse ``contract`` unchanged.  Gradients exist only on stored
blocks: unstored blocks are structural zeros, not parameters.  The paper defines no adjoint;
this is the chain rule applied to the bilinear map of Sec. III-A, Fig. 3, rule 8.
"""

from __future__ import annotations

from .blocksparse import BlockTensor, contract


def contract_vjp(g: BlockTensor, out_lbl: str, lhs: BlockTensor, lhs_lbl: str, rhs: BlockTensor, rhs_lbl: str,
                 alpha: float = 1.0, beta: float = 0.0):
    """Return (grad_lhs, grad_rhs, grad_out0) for the contraction described above."""
    g_lhs = contract(BlockTensor.zeros(lhs.spaces, lhs.nonzero), lhs_lbl, g, out_lbl, rhs, rhs_lbl, alpha, 0.0)
    g_rhs = contract(BlockTensor.zeros(rhs.spaces, rhs.nonzero), rhs_lbl, lhs, lhs_lbl, g, out_lbl, alpha, 0.0)
    g_out0 = BlockTensor(g.spaces, g.nonzero)
    g_out0.blocks = {t: beta * b for t, b in g.blocks.items()}
    return g_lhs, g_rhs, g_out0
