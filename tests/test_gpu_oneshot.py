"""GPU checks of the one-shot entry point tamm_contract and its plan cache.

* a sequence of residual updates (every doubles and singles term accumulated into one R with
  beta = 1) through the Python ``contract`` against the FP64 oracle, relative Frobenius error
  <= 1e-12 (float64 products and sums; only the summation order differs);
* one workspace shared by two contractions called alternately without host synchronisation:
  bitwise equal to separate plans with their own workspaces (the cache uses the same default
  kernel configuration, so the arithmetic is the same);
* each reduced precision through the cache, bitwise equal to a plan of that precision;
* a tensor destroyed and replaced: the cache drops its plans and the new tensor gets a fresh one.
"""

import ctypes

import pytest
import torch

import oracle
from paper_2201_01257_amd import _lib
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd import synth
from tests.gpu_util import Problem, max_rel

pytestmark = pytest.mark.gpu

TERMS = synth.TERMS
TOL = 1e-12
SMALL = (24, 40, 12, 16)


def inputs(prob, term, gpu=True):
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = TERMS[term]
    mk = prob.gpu_tensor if gpu else prob.oracle_tensor
    return (on, op, ol), (mk(ln, lp), ll), (mk(rn, rp), rl), a


def test_residual_update_sequence_matches_oracle():
    prob = Problem(*SMALL)
    tm.contract_cache_clear()
    R = prob.gpu_tensor("R", "vvoo")
    Ro = prob.oracle_tensor("R", "vvoo")
    seq = ["ladder", "ring", "hh", "t1_v", "t1_o", "ring"]
    for term in seq:
        (_, _, ol), (L, ll), (Rh, rl), a = inputs(prob, term)
        assert tm.contract(R, ol, L, ll, Rh, rl, a, 1.0) is R
        (_, _, _), (Lo, _), (Rho, _), _ = inputs(prob, term, gpu=False)
        Ro = oracle.contract(Ro, ol, Lo, ll, Rho, rl, a, 1.0)
    torch.cuda.synchronize()
    rel, mx = max_rel(R.to_blocks(), Ro.blocks)
    assert rel <= TOL, (rel, mx)
    # one cached plan per distinct (out, operands, labels); the repeated ring term reused its own
    # entry only if the same operand tensors were passed, which they were not (fresh tensors)
    assert tm.contract_cache_count() == len(seq)


def test_shared_workspace_alternating_contractions_bitwise():
    prob = Problem(*SMALL)
    lib = _lib.load()
    tm.contract_cache_clear()
    terms = ["ladder", "ring"]
    ops = {t: inputs(prob, t) for t in terms}
    outs = {t: prob.gpu_tensor("R", "vvoo") for t in terms}
    refs = {t: prob.gpu_tensor("R", "vvoo") for t in terms}
    sizes = []
    for t in terms:
        (_, _, ol), (L, ll), (Rh, rl), _ = ops[t]
        n = ctypes.c_size_t()
        assert lib.tamm_contract_workspace_size(outs[t]._h, ol.encode(), L._h, ll.encode(), Rh._h, rl.encode(), 0,
                                                ctypes.byref(n)) == 0
        sizes.append(n.value)
    ws_owner, ws = tm._aligned_workspace(max(sizes), outs["ladder"].data.device)
    nbytes = max(sizes)
    plans = {t: tm.Plan(refs[t], ops[t][0][2], ops[t][1][0], ops[t][1][1], ops[t][2][0], ops[t][2][1]) for t in terms}
    s = tm.current_stream_handle()
    for rep in range(3):
        for t in terms:
            (_, _, ol), (L, ll), (Rh, rl), a = ops[t]
            beta = 0.0 if rep == 0 else 1.0
            rc = lib.tamm_contract(outs[t]._h, ol.encode(), L._h, ll.encode(), Rh._h, rl.encode(), 0, a, beta,
                                   ctypes.c_void_p(ws), nbytes, s)
            assert rc == 0, lib.tamm_last_error().decode()
            plans[t].execute(a, beta)
    torch.cuda.synchronize()
    for t in terms:
        assert torch.equal(outs[t].data, refs[t].data), t
    assert tm.contract_cache_count() == 2
    del ws_owner


@pytest.mark.parametrize("precision", ["f32", "bf16x3", "bf16x4_aligned"])
def test_reduced_precision_through_the_cache_bitwise(precision):
    prob = Problem(*SMALL)
    (_, _, ol), (L, ll), (Rh, rl), a = inputs(prob, "ladder")
    O1 = prob.gpu_tensor("R", "vvoo")
    O2 = prob.gpu_tensor("R", "vvoo")
    tm.contract(O1, ol, L, ll, Rh, rl, a, 0.0, precision=precision)
    tm.Plan(O2, ol, L, ll, Rh, rl, precision=precision).execute(a, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(O1.data, O2.data)


def test_replaced_tensor_gets_a_fresh_plan():
    prob = Problem(*SMALL)
    tm.contract_cache_clear()
    (_, _, ol), (L, ll), (Rh, rl), a = inputs(prob, "ring")
    (_, _, _), (Lo, _), (Rho, _), _ = inputs(prob, "ring", gpu=False)
    ref = oracle.contract(prob.oracle_tensor("R", "vvoo"), ol, Lo, ll, Rho, rl, a, 0.0)
    for _ in range(3):
        O = prob.gpu_tensor("R", "vvoo")
        tm.contract(O, ol, L, ll, Rh, rl, a, 0.0)
        torch.cuda.synchronize()
        rel, mx = max_rel(O.to_blocks(), ref.blocks)
        assert rel <= TOL, (rel, mx)
        assert tm.contract_cache_count() == 1
        del O
        assert tm.contract_cache_count() == 0
