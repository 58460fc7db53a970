"""Edge cases and full-size runs of the HIP path.

* degenerate structure: every tile pair screened out (out = beta * out), an output with no stored
  block (a no-op), summed tiles of extent 1;
* a single dense block against numpy's float64 matmul (a library routine, independent of the
  oracle), and one block close to the gathers' 1 GiB addressing limit;
* the CCSD doubles workload at its full size (O=40, V=200, tiles of 40) in the launch configuration
  the bench times (autotuned), on sampled output blocks against the oracle; the mixed-precision
  workload (O=64, V=320, tiles of 64) in the aligned split at its stated error bound.

FP64 tolerance: relative Frobenius error <= 1e-12 (products and sums in float64, only the
summation order differs); exact where the result is beta * out with nothing added.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel_err(got, ref):
    num = sum(float(np.sum((got[k] - v) ** 2)) for k, v in ref.items())
    den = sum(float(np.sum(v ** 2)) for v in ref.values())
    return (num / den) ** 0.5 if den > 0 else num ** 0.5


def test_every_pair_screened_out_scales_out_by_beta():
    sp = tm.Space.fixed(12, 4)  # three tiles per label
    dense = lambda t, s: True  # noqa: E731
    rng = np.random.default_rng(11)
    out0 = rng.standard_normal((12, 12))
    out = tm.Tensor([sp, sp], nonzero=dense).from_dense(out0)
    # lhs stores only summed tile 0, rhs only summed tiles 1 and 2: no tile pair survives
    L = tm.Tensor([sp, sp], nonzero=lambda t, s: int(t[1]) == 0).from_dense(rng.standard_normal((12, 12)))
    R = tm.Tensor([sp, sp], nonzero=lambda t, s: int(t[0]) != 0).from_dense(rng.standard_normal((12, 12)))
    plan = tm.Plan(out, "ab", L, "ak", R, "kb")
    assert plan.stats()["tasks"] == 0 and plan.stats()["out_blocks"] == 9
    plan.execute(2.0, -0.75)
    torch.cuda.synchronize()
    got = out.to_blocks()
    for (i, j), blk in got.items():
        assert np.array_equal(blk, -0.75 * out0[4 * i:4 * i + 4, 4 * j:4 * j + 4])


def test_output_without_stored_blocks_is_a_no_op():
    sp = tm.Space.fixed(10, 5)
    rng = np.random.default_rng(12)
    a = rng.standard_normal((10, 10))
    L = tm.Tensor([sp, sp], nonzero=lambda t, s: True).from_dense(a)
    R = tm.Tensor([sp, sp], nonzero=lambda t, s: True).from_dense(a.T.copy())
    out = tm.Tensor([sp, sp], nonzero=lambda t, s: False)
    assert out.nblocks == 0
    plan = tm.Plan(out, "ab", L, "ak", R, "kb")
    plan.execute(1.0, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(L.to_dense(), a)


def test_summed_tiles_of_extent_one():
    one = tm.Space.fixed(7, 1)
    rows = tm.Space.fixed(33, 16)
    o_one, o_rows = oracle.Space.fixed(7, 1), oracle.Space.fixed(33, 16)
    rng = np.random.default_rng(13)
    a, b = rng.standard_normal((33, 7)), rng.standard_normal((7, 33))
    out = tm.Tensor([rows, rows])
    L = tm.Tensor([rows, one]).from_dense(a)
    R = tm.Tensor([one, rows]).from_dense(b)
    plan = tm.Plan(out, "ij", L, "ik", R, "kj")
    plan.execute(1.0, 0.0)
    torch.cuda.synchronize()
    ref = oracle.contract(oracle.BlockTensor.zeros([o_rows, o_rows]), "ij", oracle.BlockTensor.from_dense([o_rows, o_one], a),
                          "ik", oracle.BlockTensor.from_dense([o_one, o_rows], b), "kj", 1.0, 0.0)
    assert rel_err(out.to_blocks(), ref.blocks) <= TOL


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (37, 53, 29), (256, 80, 400), (300, 300, 1)])
def test_single_dense_block_matches_numpy_matmul(m, n, k):
    sm, sn, sk = tm.Space.fixed(m, m), tm.Space.fixed(n, n), tm.Space.fixed(k, k)
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    a, b = rng.standard_normal((m, k)), rng.standard_normal((k, n))
    out = tm.Tensor([sm, sn])
    plan = tm.Plan(out, "mn", tm.Tensor([sm, sk]).from_dense(a), "mk", tm.Tensor([sk, sn]).from_dense(b), "kn")
    plan.execute(1.0, 0.0)
    torch.cuda.synchronize()
    ref = a @ b
    got = out.to_dense()
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)


def test_block_near_the_gather_addressing_limit():
    # one lhs block of 8192 x 8192 elements (512 MiB): byte offsets up to 2^29 inside one buffer
    big, small = tm.Space.fixed(8192, 8192), tm.Space.fixed(16, 16)
    g = torch.Generator(device="cuda").manual_seed(14)
    L = tm.Tensor([big, big])
    L.data[:L.numel].copy_(torch.randn(L.numel, dtype=torch.float64, device="cuda", generator=g))
    R = tm.Tensor([big, small])
    R.data[:R.numel].copy_(torch.randn(R.numel, dtype=torch.float64, device="cuda", generator=g))
    out = tm.Tensor([big, small])
    tm.Plan(out, "ij", L, "ik", R, "kj").execute(1.0, 0.0)
    torch.cuda.synchronize()
    A = L.data[:L.numel].view(8192, 8192)
    B = R.data[:R.numel].view(8192, 16)
    C = out.data[:out.numel].view(8192, 16)
    rows = torch.tensor([0, 1, 4095, 8190, 8191], device="cuda")
    ref = (A[rows].cpu().numpy() @ B.cpu().numpy())
    got = C[rows].cpu().numpy()
    assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)


def _sampled_tiles(tensor_tiles, count, seed):
    rng = np.random.default_rng(seed)
    return [tensor_tiles[i] for i in rng.choice(len(tensor_tiles), size=min(count, len(tensor_tiles)), replace=False)]


@pytest.mark.slow
def test_ccsd_workload_full_size_sampled():
    import bench

    wl = synth.WORKLOADS["ccsd_doubles_o40_v200_t40"]
    orb, g, T = bench.build_inputs(torch, tm, synth, wl)
    osp = {c: bench._oracle_space(oracle, orb, c, wl["tile_occ"] if c == "o" else wl["tile_vir"]) for c in "ov"}
    for term in bench.STEP_TERMS:
        (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = synth.TERMS[term]
        lhs = T[ln]
        if ln == "W_oooo":  # the standalone input of the hole-hole ladder
            lhs = tm.Tensor([g[c] for c in lp])
            lhs.fill_blocks(lambda lo, ext, out: orb.fill(synth.input_name(ln), lp, lo, ext, out=out))
        out = tm.Tensor([g[c] for c in op])
        plan = tm.Plan(out, ol, lhs, ll, T[rn], rl)
        plan.autotune("", reps=1)  # the configuration the bench times
        plan.execute(a, 0.0)
        torch.cuda.synchronize()
        Oo = oracle.BlockTensor([osp[c] for c in op])
        pick = _sampled_tiles(Oo.stored_tiles(), 3, 2201)
        ref = oracle.contract(Oo, ol, bench._oracle_tensor(oracle, synth, orb, osp, ln, lp), ll,
                              bench._oracle_tensor(oracle, synth, orb, osp, rn, rp), rl, a, 0.0, out_tiles=pick)
        got = out.to_blocks()
        assert rel_err({t: got[t] for t in pick}, {t: ref.blocks[t] for t in pick}) <= TOL, term
