"""The particle-particle ladder over integrals rebuilt from Cholesky vectors (oracle side; test
infrastructure only).

arXiv 2201.01257, Sec. IV-A-1, Eq. (cc12): the two-electron integral tensor is approximated from
Cholesky vectors (pq|L) carrying an auxiliary index L,

    v[p,q,r,s] = sum_L (pr|L)(L|qs) - (ps|L)(L|qr),

which brings the storage from the fourth power of the orbital count down to about its third.
Sec. III-A's lambda tensors are the TAMM construct for such a tensor: its blocks are computed on
demand from a user function and never stored.

Oracle: the V_vvvv blocks are produced one at a time from that definition (one ``numpy.einsum``
per pair of Cholesky-vector blocks, summed over the auxiliary tiles whose blocks are stored),
and the ladder R[a,b,i,j] <- beta R + alpha sum_cd V[a,b,c,d] T[c,d,i,j] is then the plain
block-sparse contraction of ``blocksparse.contract``.  Nothing else is reordered or fused.

Readings:

* (pq|L) is the integral of a real orbital pair, so B[p,q,L] = B[q,p,L]; in a spin-orbital
  space it is zero unless p and q carry the same spin.  The tensor B is given over (vir, vir,
  aux); its storage rule is whatever non-zero check it was built with (spin-diagonal for the
  inputs of this build).
* V is stored with the default spin rule.  For spin-diagonal B both terms of Eq. (cc12) vanish
  outside spin-conserving blocks, so nothing is lost.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .blocksparse import BlockTensor, LazyBlocks, contract
from .tiling import Space


def spin_diagonal(tiles, spins) -> bool:
    """Storage rule of Cholesky vectors B[p,q,L]: p and q of one spin (L carries none)."""
    return spins[0] == spins[1]


def v_from_cholesky(b: BlockTensor) -> BlockTensor:
    """V[a,b,c,d] of Eq. (cc12) over B's first space, as a tensor whose blocks are computed on
    first access (a lambda tensor): sum over auxiliary tiles of B[a,c,L] B[b,d,L] minus
    B[a,d,L] B[b,c,L], each product skipped when either vector block is not stored."""
    if b.rank != 3:
        raise ValueError("Cholesky vectors are a rank-3 tensor B[p,q,L]")
    v, aux = b.spaces[0], b.spaces[2]
    if b.spaces[1].sizes != v.sizes or b.spaces[1].spins != v.spins:
        raise ValueError("both orbital dimensions of B must share one tiled space")
    out = BlockTensor([v, v, v, v])

    def block(tile):
        ta, tb, tc, td = tile
        acc = np.zeros(out.block_shape(tile))
        for tl in range(aux.ntiles):
            if b.is_stored((ta, tc, tl)) and b.is_stored((tb, td, tl)):
                acc += np.einsum("acL,bdL->abcd", b.blocks[(ta, tc, tl)], b.blocks[(tb, td, tl)], optimize=True)
            if b.is_stored((ta, td, tl)) and b.is_stored((tb, tc, tl)):
                acc -= np.einsum("adL,bcL->abcd", b.blocks[(ta, td, tl)], b.blocks[(tb, tc, tl)], optimize=True)
        return acc

    out.blocks = LazyBlocks(block)
    return out


def cholesky_ladder(r: BlockTensor, t: BlockTensor, b: BlockTensor, alpha: float = 0.5, beta: float = 0.0,
                    out_tiles: Optional[Sequence] = None) -> BlockTensor:
    """beta * R + alpha * sum_cd V[a,b,c,d] T[c,d,i,j] with V rebuilt from B by Eq. (cc12).

    R and T are over (vir, vir, occ, occ); ``out_tiles`` restricts the work to those output
    blocks (only the V blocks they read are ever built)."""
    return contract(r, "abij", v_from_cholesky(b), "abcd", t, "cdij", alpha, beta, out_tiles=out_tiles)


def cholesky_tensor(v: Space, aux: Space, dense: np.ndarray) -> BlockTensor:
    """A spin-diagonal Cholesky-vector tensor over (v, v, aux) from a dense array."""
    return BlockTensor.from_dense([v, v, aux], dense, nonzero=spin_diagonal)
