"""The doubles-residual iteration of CCSD as a queued schedule (argument marshalling only).

One Jacobi iteration (the doubles equations of Sec. IV-A-1 with the antisymmetrisers written as
permuted additions, Fig. 3 rules 6-8, and the denominator update of Sec. IV-B-1):

    W[mnij]  = 1/2 V_oovv[mnef] T2[efij]                          MultOp
    R[abij]  = 1/2 V_vvvv[abcd] T2[cdij]                          MultOp  \\ fused: one launch,
    R[abij] += 1/2 W[mnij] T2[abmn]                               MultOp  / shared output tiles
    X[abij]  = V_ovvo[mbej] T2[aeim]                              MultOp
    Zv[abij] = V_vvvo[abej] T1[ei]                                MultOp
    Zo[abij] = -V_ovoo[mbij] T1[am]                               MultOp
    R += X - X[abji] - X[baij] + X[baji] + Zv - Zv[abji] + Zo - Zo[baij]   AddOps
    T2[abij] = R[abij] / (e_i + e_j - e_a - e_b)                  denominator update

The scheduler fuses the two ladders, runs W, X, Zv, Zo together in the first level and leaves the
new amplitudes in T2, so that replaying the schedule (or its captured graph) runs the next
iteration.  Every operation runs in the HIP library.
"""

from __future__ import annotations

from typing import Dict

from . import core as tm

PATTERNS = {"V_vvvv": "vvvv", "V_ovvo": "ovvo", "V_oovv": "oovv", "V_vvvo": "vvvo", "V_ovoo": "ovoo",
            "T2": "vvoo", "T1": "vo", "W": "oooo", "R": "vvoo", "X": "vvoo", "Zv": "vvoo", "Zo": "vvoo"}
INPUTS = ("V_vvvv", "V_ovvo", "V_oovv", "V_vvvo", "V_ovoo", "T2", "T1")
CONTRACTIONS = [
    ("W", "mnij", "V_oovv", "mnef", "T2", "efij", 0.5, 0.0),
    ("R", "abij", "V_vvvv", "abcd", "T2", "cdij", 0.5, 0.0),
    ("R", "abij", "W", "mnij", "T2", "abmn", 0.5, 1.0),
    ("X", "abij", "V_ovvo", "mbej", "T2", "aeim", 1.0, 0.0),
    ("Zv", "abij", "V_vvvo", "abej", "T1", "ei", 1.0, 0.0),
    ("Zo", "abij", "V_ovoo", "mbij", "T1", "am", -1.0, 0.0),
]
ANTISYMMETRISERS = [
    ("X", "abij", 1.0), ("X", "abji", -1.0), ("X", "baij", -1.0), ("X", "baji", 1.0),
    ("Zv", "abij", 1.0), ("Zv", "abji", -1.0),
    ("Zo", "abij", 1.0), ("Zo", "baij", -1.0),
]


def doubles_iteration(t: Dict[str, tm.Tensor], e_occ, e_vir) -> tm.Scheduler:
    """Queue and build one iteration over the tensors ``t`` (every name of PATTERNS, on the GPU);
    ``e_occ``, ``e_vir``: float64 device tensors of the orbital energies.  Returns the built,
    bound scheduler (``execute()`` runs one iteration)."""
    s = tm.Scheduler()
    s.plans = {}
    for out, ol, lhs, ll, rhs, rl, alpha, beta in CONTRACTIONS:
        p = tm.Plan(t[out], ol, t[lhs], ll, t[rhs], rl, bind=False)
        s.plans[(out, lhs)] = p
        s.contract(p, alpha, beta)
    for name, lbl, sign in ANTISYMMETRISERS:
        s.add(tm.Add(t["R"], "abij", t[name], lbl), sign, 1.0)
    s.denominator(tm.Denominator(t["T2"], t["R"], [e_vir, e_vir, e_occ, e_occ], [-1, -1, 1, 1]))
    s.build()
    s.bind_workspace(t["R"].data.device)
    return s


__all__ = ["doubles_iteration", "PATTERNS", "INPUTS", "CONTRACTIONS", "ANTISYMMETRISERS"]
