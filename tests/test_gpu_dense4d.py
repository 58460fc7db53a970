"""GPU parity of the dense 4D contraction C(a,b,c,d) += A(a,b,m,n) B(m,n,c,d) (every block stored,
the comparison contraction of Sec. V) against the FP64 oracle.

* small extents with a ragged last tile (28 = 8+8+8+4), every output block, alpha/beta update;
* the benchmark's full size (n = 200, tiles of 40, 625 blocks of 2.56e6 elements per tensor) on
  sampled output blocks, in the benchmark's kernel configuration and in the plan's default.
Tolerance: relative Frobenius error <= 1e-12 (float64 products and sums in another order).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd import synth
from tests.gpu_util import max_rel

pytestmark = pytest.mark.gpu

TOL = 1e-12


def tensors(n, tile):
    orb = synth.dense4d_orbitals(n)
    sp = tm.Space.fixed(n, tile)
    osp = oracle.Space.fixed(n, tile)
    g, o = {}, {}
    for name in ("N_A4", "N_B4", "N_R"):
        g[name] = tm.Tensor([sp] * 4)
        g[name].fill_blocks(lambda lo, ext, out, nm=name: orb.fill(nm, "vvvv", lo, ext, out=out))
        x = oracle.BlockTensor([osp] * 4)
        x.blocks = oracle.LazyBlocks(
            lambda t, nm=name: orb.fill(nm, "vvvv", [osp.offsets[i] for i in t], [osp.sizes[i] for i in t]))
        o[name] = x
    return g, o


def test_dense4d_small_ragged_every_block():
    g, o = tensors(28, 8)
    C = g["N_R"]
    assert C.nblocks == 4 ** 4
    p = tm.Plan(C, "abcd", g["N_A4"], "abmn", g["N_B4"], "mncd")
    assert p.stats()["tasks"] == 4 ** 6  # every (out block, K tile pair) survives
    p.execute(0.7, -0.3)
    torch.cuda.synchronize()
    ref = oracle.contract(o["N_R"], "abcd", o["N_A4"], "abmn", o["N_B4"], "mncd", 0.7, -0.3)
    rel, mx = max_rel(C.to_blocks(), ref.blocks)
    assert rel <= TOL, (rel, mx)


@pytest.mark.parametrize("config", ["f64_m64n80k32_w4x1_o1", None])
def test_dense4d_full_size_sampled(config):
    n, tile = synth.DENSE4D["dense4d_n200_t40"]["n"], synth.DENSE4D["dense4d_n200_t40"]["tile"]
    orb = synth.dense4d_orbitals(n)
    sp = tm.Space.fixed(n, tile)
    A, B, C = tm.Tensor([sp] * 4), tm.Tensor([sp] * 4), tm.Tensor([sp] * 4)
    A.fill_blocks(lambda lo, ext, out: orb.fill("N_A4", "vvvv", lo, ext, out=out))
    B.fill_blocks(lambda lo, ext, out: orb.fill("N_B4", "vvvv", lo, ext, out=out))
    p = tm.Plan(C, "abcd", A, "abmn", B, "mncd")
    if config is not None:
        ids = [c for c in range(p.config_count()) if p.config_name(c) == config]
        p.set_config(ids[0], 1)
    p.execute(1.0, 0.0)
    torch.cuda.synchronize()
    osp = oracle.Space.fixed(n, tile)

    def ot(name):
        x = oracle.BlockTensor([osp] * 4)
        x.blocks = oracle.LazyBlocks(
            lambda t: orb.fill(name, "vvvv", [osp.offsets[i] for i in t], [osp.sizes[i] for i in t]))
        return x

    OA, OB, OC = ot("N_A4"), ot("N_B4"), oracle.BlockTensor([osp] * 4)
    tiles = OC.stored_tiles()
    rng = np.random.default_rng(7)
    pick = [tiles[i] for i in rng.choice(len(tiles), 2, replace=False)] + [tiles[-1]]
    got = C.to_blocks()
    ref = oracle.contract(OC, "abcd", OA, "abmn", OB, "mncd", 1.0, 0.0, out_tiles=pick)
    rel, mx = max_rel(got, ref.blocks, keys=pick)
    assert rel <= TOL, (rel, mx)
