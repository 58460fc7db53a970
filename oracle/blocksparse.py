"""Block-sparse tensors and the tile-by-tile contraction (oracle side; test infrastructure only).

The operation is the contraction of the TAMM operation grammar (arXiv 2201.01257, Sec. III-A,
Fig. 3, rule 8; Fig. 4 shows ``C(i,a) = 0.5 * A(i,l) * B(l,a)``):

    out[L_out] <- beta * out[L_out] + alpha * sum_{L_K} lhs[L_lhs] * rhs[L_rhs]

where every index label occurs in exactly two of the three tensors and L_K are the labels of
lhs and rhs that out does not carry.  The operands are dense tensors whose unstored blocks are
exactly zero (Sec. III-A: zero blocks are not stored); the result is kept only on the stored
blocks of ``out``.

The algorithm is the plain one the paper's block decomposition implies: for every stored
output block, loop over every combination of tiles of the summed labels, skip the pair when
either operand block is not stored (the non-zero analysis of Sec. IV-A-1's spin-explicit
implementation and the non-zero check of Sec. III-A), and add the tile product.

Readings:

* ``beta == 0`` means ``out`` is never read (``=`` in the grammar), so NaNs in an old ``out``
  cannot leak; ``+=`` is ``beta = 1``; ``-=`` is ``alpha -> -alpha``.
* A stored output block with no surviving tile pair still becomes ``beta * out``.
* A tile pair whose operands are both stored but whose output block is not stored (possible
  only with a user non-zero check that is not spin conserving) is dropped and counted.
* Labels are single letters, one per tensor dimension, no repeats inside one tensor; a label
  must bind the same tiled space wherever it appears.
"""

from __future__ import annotations

from itertools import product
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from .tiling import Space, spin_conserving

Tile = Tuple[int, ...]
NonZero = Callable[[Tile, Tile], bool]  # (tile indices, tile spins) -> stored?


def _default_nonzero(tiles: Tile, spins: Tile) -> bool:
    return spin_conserving(spins)


class LazyBlocks(dict):
    """Block dictionary that produces a stored block on first access (inputs too large to hold).

    ``fill(tile tuple) -> block``; used to feed sampled runs of large problems.
    """

    def __init__(self, fill: Callable[[Tile], np.ndarray]):
        super().__init__()
        self._fill = fill

    def __missing__(self, key):
        v = np.asarray(self._fill(key), dtype=np.float64)
        self[key] = v
        return v


class BlockTensor:
    """Stored blocks of a tensor over tiled spaces, keyed by tile tuples (row-major blocks)."""

    def __init__(self, spaces: Sequence[Space], nonzero: Optional[NonZero] = None):
        self.spaces: List[Space] = list(spaces)
        self.rank = len(self.spaces)
        self.nonzero: NonZero = nonzero or _default_nonzero
        self.blocks: Dict[Tile, np.ndarray] = {}

    # -- structure -------------------------------------------------------------------------
    def all_tiles(self):
        return product(*[range(s.ntiles) for s in self.spaces])

    def is_stored(self, t: Tile) -> bool:
        spins = tuple(self.spaces[d].spins[t[d]] for d in range(self.rank))
        return bool(self.nonzero(tuple(t), spins))

    def stored_tiles(self) -> List[Tile]:
        return [tuple(t) for t in self.all_tiles() if self.is_stored(t)]

    def block_shape(self, t: Tile) -> Tuple[int, ...]:
        return tuple(self.spaces[d].sizes[t[d]] for d in range(self.rank))

    def block_slices(self, t: Tile) -> Tuple[slice, ...]:
        return tuple(
            slice(self.spaces[d].offsets[t[d]], self.spaces[d].offsets[t[d]] + self.spaces[d].sizes[t[d]])
            for d in range(self.rank)
        )

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(s.extent for s in self.spaces)

    def nnz(self) -> int:
        return sum(int(np.prod(self.block_shape(t))) for t in self.stored_tiles())

    # -- construction / conversion --------------------------------------------------------
    @classmethod
    def zeros(cls, spaces: Sequence[Space], nonzero: Optional[NonZero] = None) -> "BlockTensor":
        x = cls(spaces, nonzero)
        for t in x.stored_tiles():
            x.blocks[t] = np.zeros(x.block_shape(t))
        return x

    @classmethod
    def from_dense(cls, spaces: Sequence[Space], dense: np.ndarray, nonzero: Optional[NonZero] = None) -> "BlockTensor":
        x = cls(spaces, nonzero)
        dense = np.asarray(dense, dtype=np.float64)
        if dense.shape != x.shape:
            raise ValueError(f"dense shape {dense.shape} does not match tiled shape {x.shape}")
        for t in x.stored_tiles():
            x.blocks[t] = dense[x.block_slices(t)].copy()
        return x

    @classmethod
    def from_blocks(cls, spaces: Sequence[Space], fill: Callable[[Tile, Tuple[slice, ...]], np.ndarray],
                    nonzero: Optional[NonZero] = None) -> "BlockTensor":
        """Build from a per-block source ``fill(tile tuple, index slices) -> block``."""
        x = cls(spaces, nonzero)
        for t in x.stored_tiles():
            b = np.asarray(fill(t, x.block_slices(t)), dtype=np.float64)
            if b.shape != x.block_shape(t):
                raise ValueError("block source returned the wrong shape")
            x.blocks[t] = b
        return x

    def to_dense(self) -> np.ndarray:
        d = np.zeros(self.shape)
        for t, b in self.blocks.items():
            d[self.block_slices(t)] = b
        return d

    def copy(self) -> "BlockTensor":
        y = BlockTensor(self.spaces, self.nonzero)
        y.blocks = {t: b.copy() for t, b in self.blocks.items()}
        return y


def parse_labels(out_lbl: str, lhs_lbl: str, rhs_lbl: str):
    """Split labels into (M, N, K): out&lhs, out&rhs, lhs&rhs.  Raises ValueError otherwise."""
    for name, lbl in (("out", out_lbl), ("lhs", lhs_lbl), ("rhs", rhs_lbl)):
        if len(set(lbl)) != len(lbl):
            raise ValueError(f"repeated label in {name}: {lbl!r}")
        if not lbl.isalpha():
            raise ValueError(f"labels must be letters: {lbl!r}")
    for ch in set(out_lbl) | set(lhs_lbl) | set(rhs_lbl):
        n = (ch in out_lbl) + (ch in lhs_lbl) + (ch in rhs_lbl)
        if n != 2:
            raise ValueError(f"label {ch!r} appears in {n} tensors; a contraction label must appear in exactly two")
    m = [c for c in out_lbl if c in lhs_lbl]
    n = [c for c in out_lbl if c in rhs_lbl]
    k = [c for c in lhs_lbl if c in rhs_lbl]
    return m, n, k


def _label_spaces(out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl) -> Dict[str, Space]:
    spaces: Dict[str, Space] = {}
    for x, lbl in ((out, out_lbl), (lhs, lhs_lbl), (rhs, rhs_lbl)):
        if len(lbl) != x.rank:
            raise ValueError(f"label string {lbl!r} does not match tensor rank {x.rank}")
        for d, ch in enumerate(lbl):
            sp = x.spaces[d]
            if ch in spaces and (spaces[ch].sizes != sp.sizes or spaces[ch].spins != sp.spins):
                raise ValueError(f"label {ch!r} binds two different tiled spaces")
            spaces[ch] = sp
    return spaces


def contract(out: BlockTensor, out_lbl: str, lhs: BlockTensor, lhs_lbl: str, rhs: BlockTensor, rhs_lbl: str,
             alpha: float = 1.0, beta: float = 0.0, out_tiles=None) -> BlockTensor:
    """Return a new tensor: beta * out + alpha * (lhs contracted with rhs), on out's stored blocks.

    ``out_tiles`` restricts the work to the listed stored output blocks (sampling a large
    problem); the result then holds only those blocks.
    """
    _, _, k_lbl = parse_labels(out_lbl, lhs_lbl, rhs_lbl)
    spaces = _label_spaces(out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl)
    spec = f"{lhs_lbl},{rhs_lbl}->{out_lbl}"
    k_ranges = [range(spaces[c].ntiles) for c in k_lbl]
    result = BlockTensor(out.spaces, out.nonzero)
    todo = out.stored_tiles() if out_tiles is None else [tuple(t) for t in out_tiles]
    for ot in todo:
        if not out.is_stored(ot):
            raise ValueError(f"output block {ot} is not stored")
        acc = np.zeros(out.block_shape(ot))
        tile_of = dict(zip(out_lbl, ot))
        for kt in product(*k_ranges):
            tile_of.update(zip(k_lbl, kt))
            lt = tuple(tile_of[c] for c in lhs_lbl)
            rt = tuple(tile_of[c] for c in rhs_lbl)
            if lhs.is_stored(lt) and rhs.is_stored(rt):
                acc += np.einsum(spec, lhs.blocks[lt], rhs.blocks[rt], optimize=True)
        if beta == 0.0:
            result.blocks[ot] = alpha * acc
        else:
            result.blocks[ot] = beta * out.blocks[ot] + alpha * acc
    return result


def screen(out: BlockTensor, out_lbl: str, lhs: BlockTensor, lhs_lbl: str, rhs: BlockTensor, rhs_lbl: str) -> dict:
    """Tile-pair screening counts for one contraction.

    Returns the surviving K tile tuples of every stored output block (lexicographic), the task
    count, the useful flop count (2 * product of all label extents, summed over surviving
    tile triples), and the number of surviving pairs whose output block is not stored.
    """
    _, _, k_lbl = parse_labels(out_lbl, lhs_lbl, rhs_lbl)
    spaces = _label_spaces(out, out_lbl, lhs, lhs_lbl, rhs, rhs_lbl)
    k_ranges = [range(spaces[c].ntiles) for c in k_lbl]
    pairs: Dict[Tile, List[Tile]] = {}
    flops = 0
    dropped = 0
    for ot in out.all_tiles():
        ot = tuple(ot)
        stored = out.is_stored(ot)
        tile_of = dict(zip(out_lbl, ot))
        keep = []
        for kt in product(*k_ranges):
            tile_of.update(zip(k_lbl, kt))
            lt = tuple(tile_of[c] for c in lhs_lbl)
            rt = tuple(tile_of[c] for c in rhs_lbl)
            if lhs.is_stored(lt) and rhs.is_stored(rt):
                if stored:
                    keep.append(tuple(kt))
                    ext = 1
                    for c, t in tile_of.items():
                        ext *= spaces[c].sizes[t]
                    flops += 2 * ext
                else:
                    dropped += 1
        if stored:
            pairs[ot] = keep
    return {
        "pairs": pairs,
        "tasks": sum(len(v) for v in pairs.values()),
        "out_blocks": len(pairs),
        "useful_flops": flops,
        "dropped": dropped,
    }


def denominator_update(r: BlockTensor, e_occ: np.ndarray, e_vir: np.ndarray) -> BlockTensor:
    """New amplitudes from a residual by the orbital-energy denominator, block by block.

    Rank 4, dims (vir, vir, occ, occ):  T'[a,b,i,j] = R[a,b,i,j] / (e_i + e_j - e_a - e_b).
    Rank 2, dims (vir, occ):            T'[a,i]     = R[a,i]     / (e_i - e_a).
    The denominator is summed left to right exactly as written; the division is IEEE float64.
    """
    out = BlockTensor(r.spaces, r.nonzero)
    for t, b in r.blocks.items():
        sl = r.block_slices(t)
        if r.rank == 4:
            ea = e_vir[sl[0]][:, None, None, None]
            eb = e_vir[sl[1]][None, :, None, None]
            ei = e_occ[sl[2]][None, None, :, None]
            ej = e_occ[sl[3]][None, None, None, :]
            d = ei + ej - ea - eb
        elif r.rank == 2:
            ea = e_vir[sl[0]][:, None]
            ei = e_occ[sl[1]][None, :]
            d = ei - ea
        else:
            raise ValueError("denominator update is defined for rank 2 (vir,occ) and rank 4 (vir,vir,occ,occ)")
        out.blocks[t] = b / d
    return out
