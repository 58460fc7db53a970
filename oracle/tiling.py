"""Tiled index spaces with a spin attribute per tile (oracle side; test infrastructure only).

Follows Sec. III-A and Fig. 1 of arXiv 2201.01257: an index space is a range; a tiled index
space cuts it into tiles, either of one fixed size or from an explicit list that covers the
range; a tensor over tiled spaces is a set of blocks indexed by the Cartesian product of the
tile indices.  Spin information is attached per tile so that blocks forbidden by spin
symmetry can be left unstored.

Readings (the paper is silent on these points):

* Fixed-size tiling of a range that the tile size does not divide gives full tiles followed by
  one shorter remainder tile (Fig. 1 only shows divisible ranges).
* A spin-blocked space is the alpha sub-space followed by the beta sub-space; each is tiled on
  its own, so a tile never straddles the two, and a tile size larger than a sub-space is
  clamped to that sub-space (e.g. 20 alpha + 20 beta orbitals at tile 40 give tiles [20, 20]).
* Spin codes: alpha = 0, beta = 1.  A block of a rank-2k tensor is structurally non-zero when
  the spins of its first k indices add up to the spins of its last k indices (conservation of
  the spin projection, the spin symmetry that Sec. III-A says is used for block sparsity).
"""

from __future__ import annotations

from itertools import accumulate
from typing import List, Sequence


class Space:
    """A tiled index space: tile sizes, their start offsets, and one spin code per tile."""

    def __init__(self, tile_sizes: Sequence[int], tile_spins: Sequence[int] | None = None):
        sizes = [int(s) for s in tile_sizes]
        if not sizes or any(s <= 0 for s in sizes):
            raise ValueError("a tiled space needs at least one tile and positive tile sizes")
        spins = [0] * len(sizes) if tile_spins is None else [int(s) for s in tile_spins]
        if len(spins) != len(sizes):
            raise ValueError("one spin code per tile")
        self.sizes: List[int] = sizes
        self.spins: List[int] = spins
        self.offsets: List[int] = [0] + list(accumulate(sizes))[:-1]
        self.extent: int = sum(sizes)

    @property
    def ntiles(self) -> int:
        return len(self.sizes)

    def tile_range(self, t: int) -> range:
        return range(self.offsets[t], self.offsets[t] + self.sizes[t])

    def index_spin(self, p: int) -> int:
        """Spin code of index p (the spin of the tile that holds it)."""
        for t in range(self.ntiles):
            if self.offsets[t] <= p < self.offsets[t] + self.sizes[t]:
                return self.spins[t]
        raise IndexError(p)

    # Fig. 1: ``TiledIndexSpace tN{N, 10}`` -- one fixed tile size over a range.
    @classmethod
    def fixed(cls, extent: int, tile: int, spin: int = 0) -> "Space":
        if extent <= 0 or tile <= 0:
            raise ValueError("extent and tile must be positive")
        sizes = [tile] * (extent // tile)
        if extent % tile:
            sizes.append(extent % tile)
        return cls(sizes, [spin] * len(sizes))

    # Fig. 1: ``TiledIndexSpace tM{M, {10, 20}}`` -- explicit tile list covering the range.
    @classmethod
    def explicit(cls, extent: int, sizes: Sequence[int]) -> "Space":
        if sum(sizes) != extent:
            raise ValueError("explicit tiles must cover the whole range")
        return cls(sizes)

    @classmethod
    def spin_blocked(cls, n_alpha: int, n_beta: int, tile: int) -> "Space":
        """Alpha sub-space then beta sub-space, each tiled on its own (see module readings)."""
        sizes: List[int] = []
        spins: List[int] = []
        for n, s in ((n_alpha, 0), (n_beta, 1)):
            if n <= 0:
                continue
            sub = cls.fixed(n, min(tile, n), s)
            sizes += sub.sizes
            spins += sub.spins
        return cls(sizes, spins)

    def __repr__(self) -> str:  # pragma: no cover - debugging aid
        return f"Space(sizes={self.sizes}, spins={self.spins})"


def spin_conserving(spins: Sequence[int]) -> bool:
    """Default structural non-zero rule for a block whose tiles carry ``spins``.

    Rank 2k: the first k spins must add up to the last k spins.  Odd ranks have no such rule
    and are always stored.
    """
    r = len(spins)
    if r % 2:
        return True
    k = r // 2
    return sum(spins[:k]) == sum(spins[k:])
