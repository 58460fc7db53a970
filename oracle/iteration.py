"""One Jacobi iteration of a CCSD-like doubles residual (oracle side; test infrastructure only).

The residual is the term set of the doubles equations the paper's CCSD discussion names
(Sec. IV-A-1: the particle-particle ladder, the hole-hole ladder through the intermediate of
Eqs. (cc9)-(cc11), the ring term, the terms linear in T1), with the antisymmetrisers P(ij) and
P(ab) written as additions of label-permuted tensors (the AddOp with a permutation of Fig. 3),
followed by the orbital-energy denominator update of the Jacobi step (Sec. IV-B-1):

    W[mnij]  = 1/2 V_oovv[mnef] T2[efij]
    R[abij]  = 1/2 V_vvvv[abcd] T2[cdij] + 1/2 W[mnij] T2[abmn]
    X[abij]  = V_ovvo[mbej] T2[aeim]
    Zv[abij] = V_vvvo[abej] T1[ei]
    Zo[abij] = -V_ovoo[mbij] T1[am]
    R       += P(ij) P(ab) X + P(ij) Zv + P(ab) Zo,   P(ij) Y = Y[abij] - Y[abji]
    T2'      = R / (e_i + e_j - e_a - e_b)

The factor 1/2 on W times the 1/2 on the hole-hole ladder is the 1/4 of the hole-hole ladder
term.  Executed in program order with the oracle's own operations: this is the sequential
semantics a scheduled execution of the same queue must reproduce.
"""

from __future__ import annotations

from typing import Dict

from .blocksparse import BlockTensor, contract, denominator_update
from .elementwise import add

# (output, output labels, lhs, lhs labels, rhs, rhs labels, alpha, beta) in program order
CONTRACTIONS = [
    ("W", "mnij", "V_oovv", "mnef", "T2", "efij", 0.5, 0.0),
    ("R", "abij", "V_vvvv", "abcd", "T2", "cdij", 0.5, 0.0),
    ("R", "abij", "W", "mnij", "T2", "abmn", 0.5, 1.0),
    ("X", "abij", "V_ovvo", "mbej", "T2", "aeim", 1.0, 0.0),
    ("Zv", "abij", "V_vvvo", "abej", "T1", "ei", 1.0, 0.0),
    ("Zo", "abij", "V_ovoo", "mbij", "T1", "am", -1.0, 0.0),
]
# R += alpha * Y(permuted labels), beta = 1
ANTISYMMETRISERS = [
    ("X", "abij", 1.0), ("X", "abji", -1.0), ("X", "baij", -1.0), ("X", "baji", 1.0),
    ("Zv", "abij", 1.0), ("Zv", "abji", -1.0),
    ("Zo", "abij", 1.0), ("Zo", "baij", -1.0),
]
INTERMEDIATES = {"W": "oooo", "R": "vvoo", "X": "vvoo", "Zv": "vvoo", "Zo": "vvoo"}


def doubles_iteration(t: Dict[str, BlockTensor], e_occ, e_vir) -> Dict[str, BlockTensor]:
    """Run one iteration on the tensors ``t`` (inputs V_*, T2, T1 and zero-initialised
    intermediates W, R, X, Zv, Zo); returns a new dict with the intermediates and T2 updated."""
    t = dict(t)
    for out, ol, lhs, ll, rhs, rl, alpha, beta in CONTRACTIONS:
        t[out] = contract(t[out], ol, t[lhs], ll, t[rhs], rl, alpha, beta)
    for name, lbl, sign in ANTISYMMETRISERS:
        t["R"] = add(t["R"], "abij", t[name], lbl, sign, 1.0)
    t["T2"] = denominator_update(t["R"], e_occ, e_vir)
    return t
