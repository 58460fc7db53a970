"""The closed Jacobi loop of the doubles residual on the GPU, against the oracle running the same
iterations: every iteration runs the six terms into W and R (screening + contraction each), then
T2' = R / (e_i + e_j - e_a - e_b), and the new amplitudes become the next iteration's T2.  Plans
and the denominator update are analysed once; the amplitudes move between iterations by swapping
the storage bound to the T2 and T2' tensor handles (deferred execution, Sec. III-B), so no plan
is rebuilt.  Tolerance: relative Frobenius error <= 1e-12 after each iteration.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2201_01257_amd import core as tm
from paper_2201_01257_amd import synth
from tests.gpu_util import Problem, max_rel

pytestmark = pytest.mark.gpu

TOL = 1e-12
ORDER = ["hh_int", "ladder", "ring", "hh", "t1_v", "t1_o"]
BETA = {"hh_int": 0.0, "ladder": 0.0, "ring": 1.0, "hh": 1.0, "t1_v": 1.0, "t1_o": 1.0}
OUTPUTS = ("W_oooo", "R")


def test_jacobi_iterations_match_oracle():
    prob = Problem(12, 40, 6, 10)
    G, O = {}, {}
    for term in ORDER:
        for name, pat, _ in synth.TERMS[term][:3]:
            if name in G:
                continue
            G[name] = prob.gpu_tensor(name, pat, fill=name not in OUTPUTS)
            O[name] = (oracle.BlockTensor.zeros([prob.o[c] for c in pat]) if name in OUTPUTS
                       else prob.oracle_tensor(name, pat))
    T2, T2n = G["T2"], prob.gpu_tensor(None, "vvoo", fill=False)
    plans = {}
    for term in ORDER:
        (on, _, ol), (ln, _, ll), (rn, _, rl), _ = synth.TERMS[term]
        plans[term] = tm.Plan(G[on], ol, G[ln], ll, G[rn], rl)
    e_o = torch.from_numpy(prob.orb.e_occ).cuda()
    e_v = torch.from_numpy(prob.orb.e_vir).cuda()
    den = tm.Denominator(T2n, G["R"], [e_v, e_v, e_o, e_o], [-1, -1, 1, 1])
    for it in range(3):
        for term in ORDER:
            (on, _, ol), (ln, _, ll), (rn, _, rl), alpha = synth.TERMS[term]
            plans[term].execute(alpha, BETA[term])
            O[on] = oracle.contract(O[on], ol, O[ln], ll, O[rn], rl, alpha, BETA[term])
        den.execute()
        O["T2"] = oracle.denominator_update(O["R"], prob.orb.e_occ, prob.orb.e_vir)
        a, b = T2.data, T2n.data
        T2.bind(b)   # the new amplitudes are the next iteration's input
        T2n.bind(a)  # the old storage receives the next update
        torch.cuda.synchronize()
        rel, mx = max_rel(T2.to_blocks(), O["T2"].blocks)
        assert rel <= TOL, (it, rel, mx)
        assert np.isfinite(mx)
