"""Mixed-precision contraction paths against the FP64 oracle (relative Frobenius error per term).

Tolerances are the stated error budgets of each scheme (no exact pin exists for them):
  bf16x4_aligned (aligned lead slice + three bfloat16 residual slices, ten products): <= 1e-8
  bf16x3 (three plain bfloat16 slices, six products):                               <= 3e-7
  f32 (float32 operands and window sums):                                           <= 1e-6
Every path promotes float32 window sums to float64 and runs a float64 epilogue.

The operand splits themselves have an exact definition: the words the library multiplies
(tamm_plan_split_operand) are compared bit for bit with the oracle's split (oracle/split.py) of
the same seeded operands, for both split layouts and both operand gather modes.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd import synth
from oracle import split as osplit
from tests.gpu_util import Problem, max_rel

pytestmark = pytest.mark.gpu

TOL = {"bf16x4_aligned": 1e-8, "bf16x3": 3e-7, "f32": 1e-6}


def run(prob, term, precision, config=None, k_splits=0, beta=0.0):
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = synth.TERMS[term]
    L = prob.gpu_tensor(ln, lp)
    R = prob.gpu_tensor(rn, rp)
    O = prob.gpu_tensor(on, op)
    plan = tm.Plan(O, ol, L, ll, R, rl, precision=precision)
    if config is not None:
        plan.set_config(config, k_splits)
    plan.execute(a, beta)
    torch.cuda.synchronize()
    ref = oracle.contract(prob.oracle_tensor(on, op), ol, prob.oracle_tensor(ln, lp), ll, prob.oracle_tensor(rn, rp), rl,
                          a, beta)
    return O.to_blocks(), ref.blocks, plan


@pytest.mark.parametrize("precision", list(TOL))
@pytest.mark.parametrize("term", ["ladder", "ring", "hh_int", "t1_o"])
def test_mixed_small(precision, term):
    prob = Problem(24, 40, 12, 16)
    got, ref, _ = run(prob, term, precision)
    rel, _ = max_rel(got, ref)
    assert rel <= TOL[precision], (precision, term, rel)


@pytest.mark.parametrize("precision", list(TOL))
@pytest.mark.parametrize("shape", [(16, 48, 8, 16), (22, 38, 11, 15)], ids=["planes", "packed"])
def test_mixed_every_config_with_splits(precision, shape):
    # every tile configuration (four and eight waves) with and without K splits, on K extents that
    # are multiples of 8 (slice-plane layout for the split paths) and on ragged ones (packed)
    prob = Problem(*shape)
    n = tm.Plan(*(lambda t: (t[0], "abij", t[1], "abcd", t[2], "cdij"))(
        [prob.gpu_tensor(None, "vvoo", fill=False), prob.gpu_tensor(None, "vvvv", fill=False),
         prob.gpu_tensor(None, "vvoo", fill=False)]), precision=precision).config_count()
    for c in range(n):
        for ks in (1, 3):
            got, ref, plan = run(prob, "ladder", precision, config=c, k_splits=ks, beta=0.0)
            rel, _ = max_rel(got, ref)
            assert rel <= TOL[precision], (precision, plan.config_name(), ks, rel)


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x4_aligned"])
@pytest.mark.parametrize("shape,planes", [((24, 40, 12, 16), True), ((22, 38, 11, 15), False)], ids=["planes", "packed"])
@pytest.mark.parametrize("term", ["ladder", "ring", "hh", "hh_int"])
def test_split_layouts(precision, shape, planes, term):
    # K extents that are multiples of 8 use the slice-plane layout, others the packed layout
    prob = Problem(*shape)
    got, ref, plan = run(prob, term, precision)
    assert bool(plan.stats()["gather_layout"] & 8) == planes
    rel, _ = max_rel(got, ref)
    assert rel <= TOL[precision], (precision, term, rel)


def test_aligned_split_windows_longer_than_one():
    # pairs whose K extent spans several 256-long windows (tiles of 32 -> K = 1024 per pair)
    prob = Problem(16, 64, 8, 32)
    got, ref, _ = run(prob, "ladder", "bf16x4_aligned")
    rel, _ = max_rel(got, ref)
    assert rel <= TOL["bf16x4_aligned"], rel


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x4_aligned"])
@pytest.mark.parametrize("shape", [(24, 40, 12, 16), (22, 38, 11, 15)], ids=["planes", "packed"])
@pytest.mark.parametrize("term", ["ladder", "ring", "hh_int", "t1_o"])
def test_operand_split_matches_oracle_bitwise(precision, shape, term):
    # the split slices have an exact definition: every word of both operands, bit for bit
    prob = Problem(*shape)
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), _ = synth.TERMS[term]
    L, R, O = prob.gpu_tensor(ln, lp), prob.gpu_tensor(rn, rp), prob.gpu_tensor(on, op, fill=False)
    plan = tm.Plan(O, ol, L, ll, R, rl, precision=precision)
    k_order = osplit.summed_label_order(ol, ll, rl)
    for which, (t, name, pattern, lbl) in enumerate([(L, ln, lp, ll), (R, rn, rp, rl)]):
        words = plan.split_operand(which)
        torch.cuda.synchronize()
        words = words.cpu().numpy().view(np.uint64)
        ot = prob.oracle_tensor(name, pattern)
        for b in range(t.nblocks):
            tile = tuple(int(x) for x in t.block_tiles[b])
            _, ext = t.block_lo_ext(b)
            off = int(t.block_off[b])
            got = words[off:off + int(np.prod(ext))].reshape(ext)
            ref = osplit.split_block(ot.blocks[tile], lbl, k_order, aligned=precision == "bf16x4_aligned")
            assert np.array_equal(got, ref), (precision, term, which, tile)


def test_split_operand_rejects_float64_plans():
    prob = Problem(16, 48, 8, 16)
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), _ = synth.TERMS["ladder"]
    plan = tm.Plan(prob.gpu_tensor(on, op, fill=False), ol, prob.gpu_tensor(ln, lp, fill=False), ll,
                   prob.gpu_tensor(rn, rp, fill=False), rl)
    with pytest.raises(tm.TammError):
        plan.split_operand(0)
