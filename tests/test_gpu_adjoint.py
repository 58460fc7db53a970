"""GPU parity of the hand-written adjoint (autograd.Function) against the oracle's gradient,
central finite differences and torch.autograd.gradcheck.

L = 1/2 ||R||^2 with R = 1/2 V_vvvv[abcd] T2[cdij] + V_ovvo[mbej] T2[aeim] (ladder + ring).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd.autograd import Contraction
from tests.gpu_util import Problem, max_rel

pytestmark = pytest.mark.gpu


def setup(prob):
    V = prob.gpu_tensor("V_vvvv", "vvvv")
    Vr = prob.gpu_tensor("V_ovvo", "ovvo")
    T = prob.gpu_tensor("T2", "vvoo")
    R = prob.gpu_tensor(None, "vvoo", fill=False)
    lad = Contraction(R, "abij", V, "abcd", T, "cdij", alpha=0.5, beta=0.0)
    ring = Contraction(R, "abij", Vr, "mbej", T, "aeim", alpha=1.0, beta=1.0)
    return V, Vr, T, R, lad, ring


def forward(lad, ring, v, vr, t):
    r = lad(v, t)
    r = ring(vr, t, r)
    return r, 0.5 * (r * r).sum()


def oracle_grads(prob):
    Vo = prob.oracle_tensor("V_vvvv", "vvvv")
    Vro = prob.oracle_tensor("V_ovvo", "ovvo")
    To = prob.oracle_tensor("T2", "vvoo")
    zero = oracle.BlockTensor.zeros(To.spaces)
    R = oracle.contract(zero, "abij", Vo, "abcd", To, "cdij", 0.5, 0.0)
    R = oracle.contract(R, "abij", Vro, "mbej", To, "aeim", 1.0, 1.0)
    gV, gT1, _ = oracle.contract_vjp(R, "abij", Vo, "abcd", To, "cdij", 0.5, 0.0)
    gVr, gT2, _ = oracle.contract_vjp(R, "abij", Vro, "mbej", To, "aeim", 1.0, 1.0)
    gT = oracle.BlockTensor(To.spaces)
    gT.blocks = {k: gT1.blocks[k] + gT2.blocks[k] for k in gT1.blocks}
    return R, gV, gVr, gT


def as_blocks(struct, flat):
    out = {}
    f = flat.detach().cpu().numpy()
    for b in range(struct.nblocks):
        lo, ext = struct.block_lo_ext(b)
        off = int(struct.block_off[b])
        out[tuple(int(x) for x in struct.block_tiles[b])] = f[off:off + int(np.prod(ext))].reshape(ext)
    return out


@pytest.mark.parametrize("sizes", [(6, 16, 3, 8), (12, 40, 6, 16)])
def test_gradients_match_oracle(sizes):
    prob = Problem(*sizes)
    V, Vr, T, R, lad, ring = setup(prob)
    v = V.data[:V.numel].clone().requires_grad_(True)
    vr = Vr.data[:Vr.numel].clone().requires_grad_(True)
    t = T.data[:T.numel].clone().requires_grad_(True)
    r, L = forward(lad, ring, v, vr, t)
    L.backward()
    torch.cuda.synchronize()
    Ro, gV, gVr, gT = oracle_grads(prob)
    assert max_rel(as_blocks(R, r), Ro.blocks)[0] <= 1e-12
    assert max_rel(as_blocks(V, v.grad), gV.blocks)[0] <= 1e-12
    assert max_rel(as_blocks(Vr, vr.grad), gVr.blocks)[0] <= 1e-12
    assert max_rel(as_blocks(T, t.grad), gT.blocks)[0] <= 1e-12


def test_central_finite_differences_small():
    # O=6 -> [3a,3b], V=16 -> [8a,8b]; L is quadratic along any one element, so the central
    # difference is exact up to rounding.  Every stored element of T2 (3456), and 60 seeded
    # elements of each integral tensor
    prob = Problem(6, 16, 3, 8)
    V, Vr, T, R, lad, ring = setup(prob)
    v = V.data[:V.numel].clone().requires_grad_(True)
    vr = Vr.data[:Vr.numel].clone().requires_grad_(True)
    t = T.data[:T.numel].clone().requires_grad_(True)
    _, L = forward(lad, ring, v, vr, t)
    L.backward()
    assert t.numel() == 3456
    rng = np.random.default_rng(3)
    h = 1e-3
    with torch.no_grad():
        for x, g in ((t, t.grad), (v, v.grad), (vr, vr.grad)):
            idx = range(x.numel()) if x is t else rng.choice(x.numel(), size=min(60, x.numel()), replace=False)
            for i in idx:
                old = x[i].item()
                x[i] = old + h
                lp = forward(lad, ring, v, vr, t)[1].item()
                x[i] = old - h
                lm = forward(lad, ring, v, vr, t)[1].item()
                x[i] = old
                fd = (lp - lm) / (2 * h)
                an = g[i].item()
                assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (int(i), fd, an)


def test_gradcheck_tiny():
    prob = Problem(4, 8, 2, 4)
    V, Vr, T, R, lad, ring = setup(prob)
    v = V.data[:V.numel].clone().requires_grad_(True)
    vr = Vr.data[:Vr.numel].clone().requires_grad_(True)
    t = T.data[:T.numel].clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b, c: forward(lad, ring, a, b, c)[0], (v, vr, t), eps=1e-6, atol=1e-9,
                                    rtol=1e-7)


def test_adjoint_workload_size_sampled():
    # O=32 -> [16a,16b], V=160 -> [32,32,16]x2, tiles of 32; gradients compared on sampled blocks
    prob = Problem(32, 160, 32, 32)
    V, Vr, T, R, lad, ring = setup(prob)
    v = V.data[:V.numel].clone().requires_grad_(True)
    vr = Vr.data[:Vr.numel].clone().requires_grad_(True)
    t = T.data[:T.numel].clone().requires_grad_(True)
    r, L = forward(lad, ring, v, vr, t)
    L.backward()
    torch.cuda.synchronize()
    # oracle forward on all of R (needed by every gradient block), then sampled gradient blocks
    Vo = prob.oracle_tensor("V_vvvv", "vvvv", lazy=True)
    Vro = prob.oracle_tensor("V_ovvo", "ovvo")
    To = prob.oracle_tensor("T2", "vvoo")
    zero = oracle.BlockTensor.zeros(To.spaces)
    Ro = oracle.contract(zero, "abij", Vo, "abcd", To, "cdij", 0.5, 0.0)
    Ro = oracle.contract(Ro, "abij", Vro, "mbej", To, "aeim", 1.0, 1.0)
    assert max_rel(as_blocks(R, r), Ro.blocks)[0] <= 1e-12
    rng = np.random.default_rng(9)
    gv_got = as_blocks(V, v.grad)
    sv = Vo.stored_tiles()
    pick = [sv[i] for i in rng.choice(len(sv), size=6, replace=False)]
    gV = oracle.contract(oracle.BlockTensor(Vo.spaces), "abcd", Ro,
                         "abij", To, "cdij", 0.5, 0.0, out_tiles=pick)
    assert max_rel(gv_got, gV.blocks, keys=pick)[0] <= 1e-12
    gt_got = as_blocks(T, t.grad)
    st = To.stored_tiles()
    pickt = [st[i] for i in rng.choice(len(st), size=4, replace=False)]
    g1 = oracle.contract(oracle.BlockTensor(To.spaces), "cdij", Vo, "abcd", Ro, "abij", 0.5, 0.0, out_tiles=pickt)
    g2 = oracle.contract(oracle.BlockTensor(To.spaces), "aeim", Vro, "mbej", Ro, "abij", 1.0, 0.0, out_tiles=pickt)
    ref = {k: g1.blocks[k] + g2.blocks[k] for k in pickt}
    assert max_rel(gt_got, ref, keys=pickt)[0] <= 1e-12
