"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Tolerance for the FP64 path: relative Frobenius error <= 1e-12 per term (float64 products and
sums; only the summation order differs from the oracle's).  Integer results (screening pair
lists, counts) are compared exactly; the denominator update is compared bitwise.
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


def run_term(prob, term, alpha=None, beta=0.0, config=None, k_splits=0, nan_out=False):
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = TERMS[term]
    alpha = a if alpha is None else alpha
    L = prob.gpu_tensor(ln, lp)
    R = prob.gpu_tensor(rn, rp)
    O = prob.gpu_tensor(on, op)
    if nan_out:
        O.data.fill_(float("nan"))
    plan = tm.Plan(O, ol, L, ll, R, rl)
    if config is not None:
        plan.set_config(config, k_splits)
    plan.execute(alpha, beta)
    torch.cuda.synchronize()
    Lo = prob.oracle_tensor(ln, lp)
    Ro = prob.oracle_tensor(rn, rp)
    Oo = prob.oracle_tensor(on, op)
    ref = oracle.contract(Oo, ol, Lo, ll, Ro, rl, alpha, 0.0 if nan_out else beta)
    return O, plan, ref


TERMS = synth.TERMS


def test_config0_ladder_full():
    prob = Problem(10, 40, 5, 5)
    O, plan, ref = run_term(prob, "ladder")
    rel, mx = max_rel(O.to_blocks(), ref.blocks)
    assert rel <= TOL, (rel, mx)
    assert plan.stats()["tasks"] == 2560


SMALL = (24, 40, 12, 16)  # O=24 -> [12a,12b]; V=40 -> [16,4,16,4]: several macro-tiles and ragged tails
ODD = (22, 38, 11, 15)    # odd tile sizes: the gathers cannot pair table entries (8-byte loads)
N_CONFIGS = 15            # float64 kernel configurations (checked against the library below)


@pytest.mark.parametrize("term", list(TERMS))
def test_terms_small_ragged(term):
    prob = Problem(*SMALL)
    O, plan, ref = run_term(prob, term, beta=0.0)
    rel, mx = max_rel(O.to_blocks(), ref.blocks)
    assert rel <= TOL, (term, rel, mx)


@pytest.mark.parametrize("shape", [SMALL, ODD], ids=["pairs", "single"])
@pytest.mark.parametrize("term", ["ladder", "ring", "t1_o", "hh"])
@pytest.mark.parametrize("config", range(N_CONFIGS))
@pytest.mark.parametrize("k_splits", [1, 3])
def test_every_config_and_split(term, config, k_splits, shape):
    prob = Problem(*shape)
    O, plan, ref = run_term(prob, term, alpha=-0.7, beta=0.3, config=config, k_splits=k_splits)
    assert plan.config_count() == N_CONFIGS
    assert bool(plan.stats()["gather_layout"] & 4) == (shape == SMALL)
    rel, mx = max_rel(O.to_blocks(), ref.blocks)
    assert rel <= TOL, (term, config, k_splits, rel, mx)


def test_beta_zero_does_not_read_nan():
    prob = Problem(*SMALL)
    O, plan, ref = run_term(prob, "ring", nan_out=True)
    got = O.to_blocks()
    assert all(np.all(np.isfinite(b)) for b in got.values())
    rel, _ = max_rel(got, ref.blocks)
    assert rel <= TOL


def test_screen_pairs_match_oracle_exactly():
    prob = Problem(*SMALL)
    for term in TERMS:
        (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = TERMS[term]
        L = prob.gpu_tensor(ln, lp, fill=False)
        R = prob.gpu_tensor(rn, rp, fill=False)
        O = prob.gpu_tensor(on, op, fill=False)
        plan = tm.Plan(O, ol, L, ll, R, rl)
        plan.execute(1.0, 0.0)
        got = plan.screen_result()
        ref = oracle.screen(oracle.BlockTensor([prob.o[c] for c in op]), ol, oracle.BlockTensor([prob.o[c] for c in lp]),
                            ll, oracle.BlockTensor([prob.o[c] for c in rp]), rl)
        tiles = [tuple(int(x) for x in t) for t in O.block_tiles]
        assert len(got) == len(tiles)
        for b, t in enumerate(tiles):
            assert sorted(got[b]) == sorted(ref["pairs"][t]), (term, t)
        assert sum(len(x) for x in got) == ref["tasks"]


def test_user_predicate_and_dropped_pairs():
    sp = tm.Space.fixed(70, 24)  # tiles 24, 24, 22
    osp = oracle.Space.fixed(70, 24)

    def rule(seed):
        return lambda t, s: (hash((seed,) + tuple(int(x) for x in t)) % 3) != 0

    rng = np.random.default_rng(5)
    dense = [rng.standard_normal((70, 70, 70)) for _ in range(3)]
    out = tm.Tensor([sp, sp, sp], nonzero=rule(1)).from_dense(dense[0])
    L = tm.Tensor([sp, sp, sp], nonzero=rule(2)).from_dense(dense[1])
    R = tm.Tensor([sp, sp], nonzero=rule(3)).from_dense(dense[2][:, :, 0])
    plan = tm.Plan(out, "abc", L, "adc", R, "db")
    plan.execute(0.5, -1.5)
    torch.cuda.synchronize()
    Oo = oracle.BlockTensor.from_dense([osp] * 3, dense[0], rule(1))
    Lo = oracle.BlockTensor.from_dense([osp] * 3, dense[1], rule(2))
    Ro = oracle.BlockTensor.from_dense([osp] * 2, dense[2][:, :, 0], rule(3))
    ref = oracle.contract(Oo, "abc", Lo, "adc", Ro, "db", 0.5, -1.5)
    rel, _ = max_rel(out.to_blocks(), ref.blocks)
    assert rel <= TOL
    assert plan.stats()["dropped"] == oracle.screen(Oo, "abc", Lo, "adc", Ro, "db")["dropped"]


@pytest.mark.parametrize("seed", range(6))
def test_random_label_patterns(seed):
    rng = np.random.default_rng(300 + seed)
    letters = list("abcdefgh")
    rng.shuffle(letters)
    nm, nn, nk = (int(x) for x in rng.integers(1, 3, size=3))
    m, n, k = letters[:nm], letters[nm:nm + nn], letters[nm + nn:nm + nn + nk]
    ol, ll, rl = list(m + n), list(m + k), list(k + n)
    for x in (ol, ll, rl):
        rng.shuffle(x)
    ol, ll, rl = "".join(ol), "".join(ll), "".join(rl)
    dims = {}
    for c in m + n + k:
        na, nb, t = (int(x) for x in rng.integers(3, 14, size=3))
        dims[c] = (na, nb, t)
    g = {c: tm.Space.spin(*dims[c]) for c in dims}
    o = {c: oracle.Space.spin_blocked(*dims[c]) for c in dims}
    tens = []
    for lbl in (ol, ll, rl):
        shape = tuple(o[c].extent for c in lbl)
        d = rng.standard_normal(shape)
        tens.append((tm.Tensor([g[c] for c in lbl]).from_dense(d), oracle.BlockTensor.from_dense([o[c] for c in lbl], d)))
    plan = tm.Plan(tens[0][0], ol, tens[1][0], ll, tens[2][0], rl)
    plan.execute(1.25, 0.5)
    torch.cuda.synchronize()
    ref = oracle.contract(tens[0][1], ol, tens[1][1], ll, tens[2][1], rl, 1.25, 0.5)
    rel, _ = max_rel(tens[0][0].to_blocks(), ref.blocks)
    assert rel <= TOL, (ol, ll, rl, rel)


def test_bitwise_reproducible_and_order_independent():
    prob = Problem(*SMALL)
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = TERMS["ladder"]
    L = prob.gpu_tensor(ln, lp)
    R = prob.gpu_tensor(rn, rp)
    O = prob.gpu_tensor(on, op)
    plan = tm.Plan(O, ol, L, ll, R, rl)
    outs = []
    for _ in range(3):
        plan.execute(0.5, 0.0)
        torch.cuda.synchronize()
        outs.append(O.data.clone())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


@pytest.mark.parametrize("shape", [SMALL, ODD], ids=["pairs", "single"])
@pytest.mark.parametrize("term", ["ladder", "ring", "hh_int", "t1_o"])
def test_every_config_gives_the_same_bits_without_k_splits(term, shape):
    """Without K splits every tile shape sums each output element in the same order (k-steps of
    four in k order, chunk after chunk, pair after pair; padding adds exact zeros), and the edge
    tiles that deal their fragments over the waves run the same products: all configurations
    must write the same bits."""
    prob = Problem(*shape)
    (on, op, ol), (ln, lp, ll), (rn, rp, rl), a = TERMS[term]
    L = prob.gpu_tensor(ln, lp)
    R = prob.gpu_tensor(rn, rp)
    O = prob.gpu_tensor(on, op)
    plan = tm.Plan(O, ol, L, ll, R, rl)
    first = None
    for c in range(plan.config_count()):
        O.data.copy_(torch.linspace(-1.0, 1.0, O.data.numel(), dtype=torch.float64, device=O.data.device))
        plan.set_config(c, 1)
        plan.execute(-0.7, 0.3)
        torch.cuda.synchronize()
        if first is None:
            first = O.data.clone()
        else:
            assert torch.equal(O.data, first), (term, plan.config_name(c))


def test_denominator_bitwise():
    prob = Problem(*SMALL)
    R = prob.gpu_tensor("R", "vvoo")
    T = prob.gpu_tensor(None, "vvoo", fill=False)
    e_o = torch.from_numpy(prob.orb.e_occ).cuda()
    e_v = torch.from_numpy(prob.orb.e_vir).cuda()
    den = tm.Denominator(T, R, [e_v, e_v, e_o, e_o], [-1, -1, 1, 1])
    den.execute()
    torch.cuda.synchronize()
    Ro = prob.oracle_tensor("R", "vvoo")
    ref = oracle.denominator_update(Ro, prob.orb.e_occ, prob.orb.e_vir)
    got = T.to_blocks()
    for k, v in ref.blocks.items():
        assert np.array_equal(got[k], v), k
    # in place, rank 2
    T1 = prob.gpu_tensor("T1", "vo")
    ref1 = oracle.denominator_update(prob.oracle_tensor("T1", "vo"), prob.orb.e_occ, prob.orb.e_vir)
    tm.Denominator(T1, T1, [e_v, e_o], [-1, 1]).execute()
    torch.cuda.synchronize()
    got1 = T1.to_blocks()
    for k, v in ref1.blocks.items():
        assert np.array_equal(got1[k], v), k
