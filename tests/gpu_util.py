"""Shared helpers for the GPU tests: build the same seeded inputs for the HIP path and the oracle."""

from __future__ import annotations

import numpy as np

import oracle
from oracle import LazyBlocks
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd import synth


class Problem:
    """Spin-orbital spaces + energies, with matching GPU and oracle tiled spaces."""

    def __init__(self, n_occ, n_vir, tile_occ, tile_vir, seed=synth.SEED):
        self.orb = synth.Orbitals(n_occ, n_vir, seed=seed)
        no_a, nv_a = self.orb.n_occ_alpha, self.orb.n_vir_alpha
        self.g = {"o": tm.Space.spin(no_a, n_occ - no_a, tile_occ), "v": tm.Space.spin(nv_a, n_vir - nv_a, tile_vir)}
        self.o = {"o": oracle.Space.spin_blocked(no_a, n_occ - no_a, tile_occ),
                  "v": oracle.Space.spin_blocked(nv_a, n_vir - nv_a, tile_vir)}

    def gpu_tensor(self, name, pattern, nonzero=None, fill=True):
        t = tm.Tensor([self.g[c] for c in pattern], nonzero=nonzero)
        if fill and name is not None:
            src = synth.input_name(name)
            t.fill_blocks(lambda lo, ext, out: self.orb.fill(src, pattern, lo, ext, out=out))
        return t

    def oracle_tensor(self, name, pattern, nonzero=None, lazy=False):
        spaces = [self.o[c] for c in pattern]
        src = synth.input_name(name)

        def fill(tile):
            lo = [spaces[d].offsets[tile[d]] for d in range(len(pattern))]
            ext = [spaces[d].sizes[tile[d]] for d in range(len(pattern))]
            return self.orb.fill(src, pattern, lo, ext)

        x = oracle.BlockTensor(spaces, nonzero)
        if lazy:
            x.blocks = LazyBlocks(fill)
        else:
            for t in x.stored_tiles():
                x.blocks[t] = fill(t)
        return x


def max_rel(got_blocks, ref_blocks, keys=None):
    """Parity metric over the given blocks (all of ``ref_blocks`` by default).

    Returns ``(rel, max_abs)``: ``rel`` is the larger of the relative Frobenius error
    ``||got - ref||_F / ||ref||_F`` and the element-wise error ``max |got - ref| / max |ref|``, so
    a test asserting ``rel <= tol`` bounds every single element as well as the aggregate;
    ``max_abs`` is ``max |got - ref|``.
    """
    keys = list(ref_blocks.keys()) if keys is None else keys
    num = 0.0
    den = 0.0
    mx = 0.0
    ref_mx = 0.0
    for k in keys:
        d = got_blocks[k] - ref_blocks[k]
        if not np.all(np.isfinite(got_blocks[k])):
            return float("inf"), float("inf")
        num += float(np.sum(d * d))
        den += float(np.sum(ref_blocks[k] * ref_blocks[k]))
        if d.size:
            mx = max(mx, float(np.max(np.abs(d))))
            ref_mx = max(ref_mx, float(np.max(np.abs(ref_blocks[k]))))
    frob = np.sqrt(num / den) if den > 0 else np.sqrt(num)
    elem = mx / ref_mx if ref_mx > 0 else mx
    return max(float(frob), float(elem)), mx
