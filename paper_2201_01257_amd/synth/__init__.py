"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and by the CPU oracle.

Holds no arithmetic of the contraction method: it only produces input values, as pure
functions of (seed, tensor name, dense index), through the C generator in ``synth.c``
(SplitMix64 counters + Box-Muller).  Values do not depend on any tiling.

Input recipe (the synthetic stand-ins for the molecular integrals of arXiv 2201.01257,
Sec. IV-A-1, which are not available here):

* spin-orbital spaces: ``n_occ`` occupied and ``n_vir`` virtual spin-orbitals, the first half
  of each alpha, the second half beta;
* orbital energies per spin-orbital, drawn independently: occupied U[-2, -0.5], virtual
  U[0.2, 3];
* two-electron-integral-like tensors ``V_<pattern>`` (pattern over o/v per dimension),
  N(0, 0.1^2) symmetrised over the subgroup of {abcd, badc, cdab, dcba} that keeps the o/v
  pattern, scaled back to unit variance, zero where spin is not conserved;
* doubles amplitudes ``T2[c,d,i,j] = w / (e_i + e_j - e_c - e_d)``, singles
  ``T1[a,i] = w / (e_i - e_a)``, with w ~ N(0, 0.1^2) and zero where spin is not conserved;
* generic tensors ``N_<name>`` are plain N(0, 0.1^2), optionally zeroed by the spin rule;
* Cholesky vectors ``B_vvx`` of the two-electron integrals, B[p,q,L] = (pq|L) over two virtual
  spin-orbitals and an auxiliary index L (pattern letter ``x``, ``n_aux`` values): zero unless p
  and q have the same spin, else one N(0, s^2) value per unordered pair of spatial orbitals and
  L (symmetric in p, q; the alpha and beta copies equal), with s^2 = 0.1 / sqrt(2 n_aux), so
  that the integrals rebuilt from them have about the spread of ``V_vvvv``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libtamm_synth.so")
_lib = None

SEED = 2201
SIGMA = 0.1
E_OCC = (-2.0, -0.5)
E_VIR = (0.2, 3.0)

KIND_NORMAL, KIND_SYMMETRIC, KIND_AMPLITUDE, KIND_CHOLESKY = 0, 1, 2, 3


def build_library(force: bool = False) -> str:
    """Compile the generator with the host C compiler (no GPU code)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_library()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_key.restype = ctypes.c_uint64
        lib.synth_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_normal_at.restype = ctypes.c_double
        lib.synth_normal_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_uniform.restype = ctypes.c_int
        lib.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        lib.synth_fill.restype = ctypes.c_int
        lib.synth_fill.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def tag(name: str) -> int:
    """64-bit FNV-1a hash of a tensor name (the stream tag)."""
    h = 0xCBF29CE484222325
    for b in name.encode():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def uniform(seed: int, name: str, n: int, a: float, b: float, first: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    rc = _load().synth_uniform(seed, tag(name), first, n, a, b, out.ctypes.data if n else None)
    if rc != 0:
        raise ValueError("synth_uniform rejected its arguments")
    return out


def normal_at(seed: int, name: str, idx: int) -> float:
    return _load().synth_normal_at(seed, tag(name), idx)


class Orbitals:
    """Occupied/virtual spin-orbital spaces (alpha half first) and their orbital energies."""

    def __init__(self, n_occ: int, n_vir: int, seed: int = SEED, n_occ_alpha: Optional[int] = None,
                 n_vir_alpha: Optional[int] = None, n_aux: int = 0):
        self.n_occ, self.n_vir, self.seed = int(n_occ), int(n_vir), int(seed)
        self.n_aux = int(n_aux)  # auxiliary (Cholesky) index extent, pattern letter "x"
        self.n_occ_alpha = self.n_occ // 2 if n_occ_alpha is None else int(n_occ_alpha)
        self.n_vir_alpha = self.n_vir // 2 if n_vir_alpha is None else int(n_vir_alpha)
        self.e_occ = uniform(self.seed, "e_occ", self.n_occ, *E_OCC)
        self.e_vir = uniform(self.seed, "e_vir", self.n_vir, *E_VIR)

    def extent(self, c: str) -> int:
        return {"o": self.n_occ, "v": self.n_vir, "x": self.n_aux}[c]

    def n_alpha(self, c: str) -> int:
        return {"o": self.n_occ_alpha, "v": self.n_vir_alpha, "x": self.n_aux}[c]

    def energy(self, c: str) -> np.ndarray:
        return self.e_occ if c == "o" else self.e_vir

    def fill(self, name: str, pattern: str, lo: Sequence[int], ext: Sequence[int],
             out: Optional[np.ndarray] = None) -> np.ndarray:
        """Values of tensor ``name`` (dims given by the o/v ``pattern``) on the box lo..lo+ext.

        ``out`` may be a C-contiguous float64 array (or a writable view into a staging buffer)
        with ext's element count; it is filled in row-major order.
        """
        rank = len(pattern)
        dims = _i64([self.extent(c) for c in pattern])
        nalpha = _i64([self.n_alpha(c) for c in pattern])
        lo_a, ext_a = _i64(lo), _i64(ext)
        if len(lo_a) != rank or len(ext_a) != rank:
            raise ValueError("box rank does not match pattern")
        if out is None:
            out = np.empty(tuple(int(e) for e in ext_a), dtype=np.float64)
        if not out.flags.c_contiguous or out.dtype != np.float64 or out.size != int(np.prod(ext_a)):
            raise ValueError("output buffer must be a C-contiguous float64 array of the box size")
        energy_ptrs = None
        esign = None
        vclass = np.ascontiguousarray(np.array([1 if c == "v" else 0 for c in pattern], dtype=np.int8))
        keep: list = []
        sigma = SIGMA
        if name == "B_vvx":
            kind = KIND_CHOLESKY
            if pattern != "vvx" or self.n_aux <= 0:
                raise ValueError("B_vvx has pattern vvx and needs n_aux > 0")
            sigma = cholesky_sigma(self.n_aux)
        elif name.startswith("V_"):
            kind = KIND_SYMMETRIC
            if name[2:] != pattern or rank != 4:
                raise ValueError("V_<pattern> tensors are rank 4 and named after their pattern")
        elif name in ("T2", "T1"):
            kind = KIND_AMPLITUDE
            want = "vvoo" if name == "T2" else "vo"
            if pattern != want:
                raise ValueError(f"{name} has pattern {want}")
            arrs = [np.ascontiguousarray(self.energy(c)) for c in pattern]
            keep += arrs
            energy_ptrs = (ctypes.c_void_p * rank)(*[a.ctypes.data for a in arrs])
            esign = np.ascontiguousarray(np.array([1 if c == "o" else -1 for c in pattern], dtype=np.int8))
        elif name.startswith("N_"):
            kind = KIND_NORMAL
        else:
            raise ValueError(f"unknown synthetic tensor {name!r}")
        if out.size == 0:
            return out
        rc = _load().synth_fill(self.seed, tag(name), kind, rank, dims.ctypes.data, nalpha.ctypes.data,
                                lo_a.ctypes.data, ext_a.ctypes.data, sigma,
                                ctypes.cast(energy_ptrs, ctypes.c_void_p) if energy_ptrs is not None else None,
                                esign.ctypes.data if esign is not None else None, vclass.ctypes.data,
                                1, out.ctypes.data)
        if rc != 0:
            raise ValueError("synth_fill rejected its arguments")
        return out

    def dense(self, name: str, pattern: str) -> np.ndarray:
        return self.fill(name, pattern, [0] * len(pattern), [self.extent(c) for c in pattern])


def cholesky_sigma(n_aux: int) -> float:
    """Spread of the synthetic Cholesky vectors for ``n_aux`` auxiliary values (see the recipe)."""
    return float(np.sqrt(SIGMA / np.sqrt(2.0 * n_aux)))


# The CCSD doubles-residual term set used as the workload (contraction shapes, spin-orbital
# form; antisymmetrisers and Fock terms are not part of it).  Each entry:
# (out name, out pattern, out labels), (lhs ...), (rhs ...), alpha.
TERMS: Dict[str, Tuple[Tuple[str, str, str], Tuple[str, str, str], Tuple[str, str, str], float]] = {
    # particle-particle ladder: R[abij] += 1/2 V[abcd] T[cdij]
    "ladder": (("R", "vvoo", "abij"), ("V_vvvv", "vvvv", "abcd"), ("T2", "vvoo", "cdij"), 0.5),
    # ring: R[abij] += V[mbej] T[aeim]
    "ring": (("R", "vvoo", "abij"), ("V_ovvo", "ovvo", "mbej"), ("T2", "vvoo", "aeim"), 1.0),
    # hole-hole intermediate of Eq. (cc10): W[mnij] = V[mnef] T[efij]
    "hh_int": (("W_oooo", "oooo", "mnij"), ("V_oovv", "oovv", "mnef"), ("T2", "vvoo", "efij"), 1.0),
    # hole-hole ladder of Eq. (cc11): R[abij] += 1/4 W[mnij] T[abmn]
    "hh": (("R", "vvoo", "abij"), ("W_oooo", "oooo", "mnij"), ("T2", "vvoo", "abmn"), 0.25),
    # terms linear in T1: R[abij] += V[abej] T1[ei];  R[abij] -= V[mbij] T1[am]
    "t1_v": (("R", "vvoo", "abij"), ("V_vvvo", "vvvo", "abej"), ("T1", "vo", "ei"), 1.0),
    "t1_o": (("R", "vvoo", "abij"), ("V_ovoo", "ovoo", "mbij"), ("T1", "vo", "am"), -1.0),
}

# Standalone inputs for tensors that a term reads but that are outputs of another term.
STANDALONE_INPUT = {"W_oooo": "N_W_oooo", "R": "N_R"}


def input_name(name: str) -> str:
    """Synthetic source of a tensor used as an input (outputs of other terms get a plain one)."""
    return STANDALONE_INPUT.get(name, name)


# Workloads: (n_occ, n_vir, occ tile, vir tile, terms).  O and V count spin-orbitals.
WORKLOADS = {
    "ladder_o10_v40_t5": dict(n_occ=10, n_vir=40, tile_occ=5, tile_vir=5, terms=["ladder"]),
    "ccsd_doubles_o40_v200_t40": dict(n_occ=40, n_vir=200, tile_occ=40, tile_vir=40,
                                      terms=["ladder", "ring", "hh_int", "hh", "t1_v", "t1_o"]),
    "adjoint_o32_v160_t32": dict(n_occ=32, n_vir=160, tile_occ=32, tile_vir=32, terms=["ladder", "ring"]),
    "adjoint_fd_o6_v16": dict(n_occ=6, n_vir=16, tile_occ=3, tile_vir=8, terms=["ladder", "ring"]),
    "mixed_o64_v320_t64": dict(n_occ=64, n_vir=320, tile_occ=64, tile_vir=64, terms=["ladder", "ring"]),
}

# The dense 4D contraction C(a,b,c,d) += A(a,b,m,n) B(m,n,c,d) of the paper's comparison with other
# tensor frameworks (Sec. V): every dimension of extent n cut into tiles of `tile`, every block
# stored, inputs N_A4 and N_B4 plain N(0, 0.1^2) over one spin (nothing zeroed).  `proxy_n` is a
# smaller extent of the output dimensions (same tiles, same summed extent) on which the kernel
# configuration is tuned.
DENSE4D = {
    "dense4d_n200_t40": dict(n=200, tile=40, proxy_n=80),
    "dense4d_n160_t40": dict(n=160, tile=40, proxy_n=80),
}


# The particle-particle ladder with V_vvvv rebuilt from Cholesky vectors, Eq. (cc12):
# V[a,b,c,d] = sum_L B[a,c,L] B[b,d,L] - B[a,d,L] B[b,c,L].  n_aux = 6.29 x the spatial orbitals
# (O + V) / 2, the ratio of the paper's aug-cc-pVDZ example (7810 vectors for 146 + 1096
# orbitals, Sec. V); the auxiliary index is one tile.
CHOLESKY = {
    "chol_ladder_o40_v200_t40": dict(n_occ=40, n_vir=200, tile_occ=40, tile_vir=40, n_aux=755, tile_aux=755),
    "chol_ladder_o64_v320_t64": dict(n_occ=64, n_vir=320, tile_occ=64, tile_vir=64, n_aux=1207, tile_aux=1207),
}


# The complex-by-real ladder of real-time coupled cluster: R(a,b,i,j) += 1/2 V(a,b,c,d) T(c,d,i,j) with
# T and R complex and V real.  A complex tensor is stored interleaved (real part, imaginary part),
# i.e. as a real tensor with one more trailing dimension of extent 2 (one tile of 2), so the
# contraction is R(a,b,i,j,z) += 1/2 V(a,b,c,d) T(c,d,i,j,z).  Real part of T: the amplitudes T2,
# imaginary part: N_T2im (plain N(0, 0.1^2), zero where spin is not conserved).
COMPLEX = {
    "tdcc_ladder_o40_v200_t40": dict(n_occ=40, n_vir=200, tile_occ=40, tile_vir=40),
}


def fill_complex(orb: "Orbitals", re_name: str, im_name: str, pattern: str, lo: Sequence[int],
                 ext: Sequence[int], out: Optional[np.ndarray] = None) -> np.ndarray:
    """Interleaved complex values of a tensor over ``pattern`` plus a trailing (re, im) dimension,
    on the box lo..lo+ext (the box covers the whole trailing dimension: lo[-1] = 0, ext[-1] = 2)."""
    if len(lo) != len(pattern) + 1 or int(lo[-1]) != 0 or int(ext[-1]) != 2:
        raise ValueError("the box must cover the whole (re, im) dimension")
    if out is None:
        out = np.empty(tuple(int(e) for e in ext), dtype=np.float64)
    out[..., 0] = orb.fill(re_name, pattern, lo[:-1], ext[:-1])
    out[..., 1] = orb.fill(im_name, pattern, lo[:-1], ext[:-1])
    return out


def dense4d_orbitals(n: int, seed: int = SEED) -> "Orbitals":
    """One-spin orbital set of extent n, so that the spin rule stores (and fills) every block."""
    return Orbitals(2, n, seed=seed, n_occ_alpha=2, n_vir_alpha=n)


def batched_problems(seed: int = SEED, count: int = 256):
    """The batched workload: ``count`` independent contractions from random index spaces.

    Per problem: O = 2*U{4..24}, V = 2*U{16..80} spin-orbitals, occupied and virtual tile sizes
    drawn independently from {16, 24, 32, 48, 64}, term type uniform over the six of TERMS.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    names = list(TERMS)
    tiles = [16, 24, 32, 48, 64]
    out = []
    for k in range(count):
        n_occ = 2 * int(rng.integers(4, 25))
        n_vir = 2 * int(rng.integers(16, 81))
        t_o = int(tiles[rng.integers(0, len(tiles))])
        t_v = int(tiles[rng.integers(0, len(tiles))])
        term = names[int(rng.integers(0, len(names)))]
        out.append(dict(index=k, n_occ=n_occ, n_vir=n_vir, tile_occ=t_o, tile_vir=t_v, term=term,
                        seed=seed * 1000 + k))
    return out
