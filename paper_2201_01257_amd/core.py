"""Python binding of the C ABI: tiled spaces, block-sparse tensors on the GPU, contraction plans.

Argument marshalling only: every step of a contraction (screening, gathers, MFMA products,
epilogue) runs in the HIP library.  PyTorch supplies device memory and the current stream.
"""

from __future__ import annotations

import ctypes
import sys
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import NONZERO_FN, PlanStats, TammError, check, load


def _destroy(obj, fname: str, _lib_mod=_lib, _sys=sys) -> None:
    """Release a library handle from ``__del__``; a no-op while the interpreter shuts down, when
    module globals and the HIP runtime may already be gone."""
    h = getattr(obj, "_h", None)
    if not h:
        return
    obj._h = None
    try:
        if _sys.is_finalizing() or _lib_mod._lib is None:
            return
        getattr(_lib_mod._lib, fname)(h)
    except Exception:  # noqa: BLE001 - destructors must not raise
        pass

PRECISIONS = {"f64": 0, "f32": 1, "bf16x3": 2, "bf16x4_aligned": 3}


def _torch():
    import torch

    return torch


def current_stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _aligned_workspace(nbytes: int, device):
    """A uint8 device buffer with a 256-byte aligned start; returns (owner, pointer)."""
    torch = _torch()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    pad = (-ptr) % 256
    return buf, ptr + pad


class Space:
    """A tiled index space (Sec. III-A, Fig. 1), owned by the C library."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        lib = load()
        n = ctypes.c_int32()
        ext = ctypes.c_int64()
        check(lib.tamm_space_info(self._h, ctypes.byref(n), ctypes.byref(ext)))
        self.ntiles = n.value
        self.extent = ext.value
        self.sizes = np.zeros(self.ntiles, dtype=np.int64)
        self.offsets = np.zeros(self.ntiles, dtype=np.int64)
        self.spins = np.zeros(self.ntiles, dtype=np.int8)
        check(lib.tamm_space_tiles(self._h, self.sizes.ctypes.data, self.offsets.ctypes.data, self.spins.ctypes.data))

    @classmethod
    def spin(cls, n_alpha: int, n_beta: int, tile: int) -> "Space":
        h = ctypes.c_void_p()
        check(load().tamm_space_create_spin(n_alpha, n_beta, tile, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def fixed(cls, extent: int, tile: int) -> "Space":
        h = ctypes.c_void_p()
        check(load().tamm_space_create_fixed(extent, tile, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def explicit(cls, sizes: Sequence[int], spins: Optional[Sequence[int]] = None) -> "Space":
        s = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
        sp = None if spins is None else np.ascontiguousarray(np.asarray(spins, dtype=np.int8))
        h = ctypes.c_void_p()
        check(load().tamm_space_create(s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       None if sp is None else sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                       len(s), ctypes.byref(h)))
        return cls(h.value)

    def __del__(self, _d=_destroy):
        _d(self, "tamm_space_destroy")


class Tensor:
    """A block-sparse float64 tensor whose stored blocks live in one device buffer.

    ``nonzero(tile_idx, tile_spins) -> bool`` overrides the spin rule.  ``device=None`` creates
    the structure only (no storage), which is enough for planning on a machine without a GPU.
    """

    def __init__(self, spaces: Sequence[Space], nonzero: Optional[Callable] = None, device="cuda"):
        lib = load()
        self.spaces = list(spaces)
        self.rank = len(self.spaces)
        self.nonzero = nonzero
        arr = (ctypes.c_void_p * self.rank)(*[s._h.value for s in self.spaces])
        h = ctypes.c_void_p()
        cb = None
        if nonzero is not None:
            def _cb(tiles, spins, rank, user):
                t = tuple(tiles[i] for i in range(rank))
                s = tuple(spins[i] for i in range(rank))
                return 1 if nonzero(t, s) else 0
            cb = NONZERO_FN(_cb)
        check(lib.tamm_tensor_create(arr, self.rank, ctypes.cast(cb, ctypes.c_void_p) if cb else None, None,
                                     ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        check(lib.tamm_tensor_numel(self._h, ctypes.byref(n)))
        self.numel = n.value
        nb = ctypes.c_int64()
        check(lib.tamm_tensor_blocks(self._h, ctypes.byref(nb), None, None))
        self.nblocks = nb.value
        self.block_tiles = np.zeros((self.nblocks, self.rank), dtype=np.int32)
        self.block_off = np.zeros(self.nblocks, dtype=np.int64)
        if self.nblocks:
            check(lib.tamm_tensor_blocks(self._h, ctypes.byref(nb), self.block_tiles.ctypes.data,
                                         self.block_off.ctypes.data))
        self.data = None
        self._contract_ws: Dict[tuple, tuple] = {}  # contract(): workspace per distinct contraction
        if device is not None:
            torch = _torch()
            self.data = torch.zeros(max(self.numel, 1), dtype=torch.float64, device=device)
            self.bind(self.data)

    def bind(self, storage):
        """Bind a float64 torch tensor with at least ``numel`` elements as the storage."""
        torch = _torch()
        if storage.dtype != torch.float64 or not storage.is_contiguous() or storage.numel() < self.numel:
            raise ValueError("storage must be a contiguous float64 tensor with at least numel elements")
        self.data = storage
        check(load().tamm_tensor_bind(self._h, ctypes.c_void_p(storage.data_ptr()), storage.numel() * 8))

    # -- block geometry -------------------------------------------------------------------
    def block_lo_ext(self, b: int) -> Tuple[Tuple[int, ...], Tuple[int, ...]]:
        t = self.block_tiles[b]
        lo = tuple(int(self.spaces[d].offsets[t[d]]) for d in range(self.rank))
        ext = tuple(int(self.spaces[d].sizes[t[d]]) for d in range(self.rank))
        return lo, ext

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(s.extent for s in self.spaces)

    # -- host <-> device ------------------------------------------------------------------
    def fill_blocks(self, fn: Callable[[Tuple[int, ...], Tuple[int, ...], np.ndarray], None],
                    chunk_bytes: int = 256 << 20):
        """Fill every stored block on the host with ``fn(lo, ext, out)`` and upload it.

        ``out`` is a C-contiguous float64 array of shape ``ext`` to be written in place.
        Blocks are staged through a pinned host buffer of at most ``chunk_bytes``.
        """
        torch = _torch()
        if self.data is None:
            raise RuntimeError("tensor has no device storage")
        if self.numel == 0:
            return
        cap = max(chunk_bytes // 8, 1)
        largest = max(int(np.prod(self.block_lo_ext(b)[1])) for b in range(self.nblocks))
        cap = max(cap, largest)
        pinned = self.data.is_cuda
        stage = torch.empty(min(cap, self.numel), dtype=torch.float64, pin_memory=pinned)
        host = stage.numpy()
        b = 0
        while b < self.nblocks:
            start = int(self.block_off[b])
            e = b
            end = start
            while e < self.nblocks:
                n = int(np.prod(self.block_lo_ext(e)[1]))
                if end + n - start > cap:
                    break
                end += n
                e += 1
            for j in range(b, e):
                lo, ext = self.block_lo_ext(j)
                off = int(self.block_off[j]) - start
                n = int(np.prod(ext))
                fn(lo, ext, host[off:off + n].reshape(ext))
            self.data[start:end].copy_(stage[:end - start], non_blocking=False)
            b = e

    def from_dense(self, dense: np.ndarray):
        dense = np.asarray(dense, dtype=np.float64)
        if dense.shape != self.shape:
            raise ValueError(f"dense shape {dense.shape} != {self.shape}")

        def fn(lo, ext, out):
            out[...] = dense[tuple(slice(l, l + e) for l, e in zip(lo, ext))]

        self.fill_blocks(fn)
        return self

    def to_host(self) -> np.ndarray:
        torch = _torch()
        torch.cuda.synchronize()
        return self.data[: self.numel].cpu().numpy()

    def to_blocks(self) -> Dict[Tuple[int, ...], np.ndarray]:
        flat = self.to_host()
        out = {}
        for b in range(self.nblocks):
            lo, ext = self.block_lo_ext(b)
            off = int(self.block_off[b])
            out[tuple(int(x) for x in self.block_tiles[b])] = flat[off:off + int(np.prod(ext))].reshape(ext)
        return out

    def to_dense(self) -> np.ndarray:
        d = np.zeros(self.shape)
        flat = self.to_host()
        for b in range(self.nblocks):
            lo, ext = self.block_lo_ext(b)
            off = int(self.block_off[b])
            d[tuple(slice(l, l + e) for l, e in zip(lo, ext))] = flat[off:off + int(np.prod(ext))].reshape(ext)
        return d

    def view_rows(self, tile_lo: int, tile_hi: int) -> "Tensor":
        """A tensor over tiles [tile_lo, tile_hi) of the first dimension sharing this tensor's
        storage (tamm_tensor_view_rows); bound to the matching slice of ``data``."""
        lib = load()
        h = ctypes.c_void_p()
        base = ctypes.c_int64()
        check(lib.tamm_tensor_view_rows(self._h, int(tile_lo), int(tile_hi), ctypes.byref(h), ctypes.byref(base)))
        v = Tensor.__new__(Tensor)
        v._h = h
        v.parent = self  # keeps the storage alive
        first = self.spaces[0]
        sl = slice(int(tile_lo), int(tile_hi))
        # the first space is a slice of this tensor's (no library handle of its own): its tiles,
        # with offsets counted from the slice's start
        v.spaces = [_SpaceSlice(first.sizes[sl], first.spins[sl])] + list(self.spaces[1:])
        v.rank = self.rank
        v.nonzero = self.nonzero
        n = ctypes.c_int64()
        check(lib.tamm_tensor_numel(h, ctypes.byref(n)))
        v.numel = n.value
        nb = ctypes.c_int64()
        check(lib.tamm_tensor_blocks(h, ctypes.byref(nb), None, None))
        v.nblocks = nb.value
        v.block_tiles = np.zeros((v.nblocks, v.rank), dtype=np.int32)
        v.block_off = np.zeros(v.nblocks, dtype=np.int64)
        if v.nblocks:
            check(lib.tamm_tensor_blocks(h, ctypes.byref(nb), v.block_tiles.ctypes.data, v.block_off.ctypes.data))
        v._contract_ws = {}
        v.view_base = base.value
        v.data = None
        if self.data is not None:
            v.bind(self.data[base.value:base.value + max(v.numel, 1)])
        return v

    def __del__(self, _d=_destroy):
        self._contract_ws = {}
        _d(self, "tamm_tensor_destroy")


class _SpaceSlice:
    """Tile geometry of a run of tiles of a Space (the first dimension of a row view)."""

    def __init__(self, sizes, spins):
        self.sizes = np.asarray(sizes, dtype=np.int64).copy()
        self.spins = np.asarray(spins, dtype=np.int8).copy()
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)[:-1]]).astype(np.int64)
        self.ntiles = len(self.sizes)
        self.extent = int(self.sizes.sum())


def spin_diagonal(tiles, spins) -> bool:
    """Non-zero check of Cholesky vectors B[p,q,L]: p and q of one spin."""
    return spins[0] == spins[1]


class Plan:
    """A contraction out(ol) = beta*out + alpha * lhs(ll) * rhs(rl), analysed once."""

    def __init__(self, out: Tensor, ol: str, lhs: Tensor, ll: str, rhs: Tensor, rl: str, precision: str = "f64",
                 bind: bool = True):
        self.out, self.lhs, self.rhs = out, lhs, rhs  # kept alive as long as the plan
        self.labels = (ol, ll, rl)
        self.precision = precision
        h = ctypes.c_void_p()
        check(load().tamm_plan_create(out._h, ol.encode(), lhs._h, ll.encode(), rhs._h, rl.encode(),
                                      PRECISIONS[precision], ctypes.byref(h)))
        self._h = h
        self._ws = None
        if bind and out.data is not None:
            self.bind_workspace()

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        check(load().tamm_plan_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def bind_workspace(self):
        device = self.out.data.device
        self._ws, ptr = _aligned_workspace(self.workspace_size(), device)
        check(load().tamm_plan_bind_workspace(self._h, ctypes.c_void_p(ptr), self.workspace_size()))

    def stats(self) -> dict:
        s = PlanStats()
        check(load().tamm_plan_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def config_count(self) -> int:
        n = ctypes.c_int32()
        check(load().tamm_plan_config_count(self._h, ctypes.byref(n)))
        return n.value

    def set_config(self, config: int, k_splits: int = 0):
        check(load().tamm_plan_set_config(self._h, config, k_splits))
        if self.out.data is not None:
            self.bind_workspace()

    def set_constant(self, which: int, constant: bool = True):
        """Declare operand ``which`` (0 = lhs, 1 = rhs) constant: its split-bfloat16 slices are made
        once and reused (tamm_plan_set_constant); call again after changing its values."""
        check(load().tamm_plan_set_constant(self._h, int(which), 1 if constant else 0))

    def set_order(self, tile_order: int = 0, chunk: int = -1):
        """Launch order: tile order (0 row by row per block, 1 grouped by B column panel) and work
        items per die chunk (0: none, -1: library default); see tamm_plan_set_order."""
        check(load().tamm_plan_set_order(self._h, int(tile_order), int(chunk)))
        if self.out.data is not None:
            self.bind_workspace()

    def autotune(self, cache_path: str = "", reps: int = 3, stream=None):
        """Measure the kernel configurations and keep the fastest (see tamm_plan_autotune)."""
        n = ctypes.c_size_t()
        check(load().tamm_plan_autotune_workspace_size(self._h, ctypes.byref(n)))
        device = self.out.data.device
        self._ws, ptr = _aligned_workspace(n.value, device)
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_plan_autotune(self._h, ctypes.c_void_p(ptr), n.value, s, cache_path.encode(), reps))

    def config_name(self, config: Optional[int] = None) -> str:
        c = self.stats()["kernel_config"] if config is None else config
        return load().tamm_config_name(PRECISIONS[self.precision], c).decode()

    def execute(self, alpha: float = 1.0, beta: float = 0.0, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_plan_execute(self._h, float(alpha), float(beta), s))

    def screen(self, stream=None):
        check(load().tamm_plan_screen(self._h, current_stream_handle() if stream is None else stream))

    def contract(self, alpha: float = 1.0, beta: float = 0.0, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_plan_contract(self._h, float(alpha), float(beta), s))

    def screen_result(self):
        """Per stored out block: list of surviving K tile tuples (K labels in lhs order)."""
        st = self.stats()
        nob = st["out_blocks"]
        counts = np.zeros(max(nob, 1), dtype=np.int32)
        ol, ll, rl = self.labels
        nk = len([c for c in ll if c not in ol])
        ktiles = np.zeros(max(st["candidates"] * max(nk, 1), 1), dtype=np.int32)
        check(load().tamm_plan_screen_result(self._h, current_stream_handle(), counts.ctypes.data, ktiles.ctypes.data))
        res = []
        w = 0
        for b in range(nob):
            lst = []
            for _ in range(int(counts[b])):
                lst.append(tuple(int(x) for x in ktiles[w:w + nk]))
                w += nk
            res.append(lst)
        return res

    def split_operand(self, which: int, stream=None):
        """The split-bfloat16 slices of operand `which` (0 = lhs, 1 = rhs) as the contraction uses
        them: one int64 word per stored element at the operand's element offsets, slice s in bits
        16s..16s+15 (see tamm_plan_split_operand)."""
        t = self.lhs if which == 0 else self.rhs
        out = _torch().empty(max(t.numel, 1), dtype=_torch().int64, device=t.data.device)
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_plan_split_operand(self._h, which, ctypes.c_void_p(out.data_ptr()), out.numel() * 8, s))
        return out[:t.numel]

    def __del__(self, _d=_destroy):
        _d(self, "tamm_plan_destroy")


def contract(out: Tensor, ol: str, lhs: Tensor, ll: str, rhs: Tensor, rl: str, alpha: float = 1.0,
             beta: float = 0.0, precision: str = "f64", stream=None) -> Tensor:
    """out(ol) = beta*out(ol) + alpha * lhs(ll) * rhs(rl) on the GPU through tamm_contract, whose
    plan cache lives in the library.  Each distinct contraction keeps its own workspace on ``out``
    (and holds ``lhs`` and ``rhs`` as long as ``out`` lives), so repeated calls stay asynchronous.
    Returns ``out``."""
    lib = load()
    key = (ol, id(lhs), ll, id(rhs), rl, precision)
    ent = out._contract_ws.get(key)
    if ent is None or ent[0] is not lhs or ent[1] is not rhs:
        n = ctypes.c_size_t()
        check(lib.tamm_contract_workspace_size(out._h, ol.encode(), lhs._h, ll.encode(), rhs._h, rl.encode(),
                                               PRECISIONS[precision], ctypes.byref(n)))
        ws, ptr = _aligned_workspace(n.value, out.data.device)
        ent = (lhs, rhs, ws, ptr, n.value)
        out._contract_ws[key] = ent
    s = current_stream_handle() if stream is None else stream
    check(lib.tamm_contract(out._h, ol.encode(), lhs._h, ll.encode(), rhs._h, rl.encode(), PRECISIONS[precision],
                            float(alpha), float(beta), ctypes.c_void_p(ent[3]), ent[4], s))
    return out


def contract_noalloc(out: Tensor, ol: str, lhs: Tensor, ll: str, rhs: Tensor, rl: str, alpha: float = 1.0,
                     beta: float = 0.0, precision: str = "f64", stream=None) -> Tensor:
    """out(ol) = beta*out(ol) + alpha * lhs(ll) * rhs(rl) through tamm_contract_noalloc: no
    workspace argument and no device allocation (the library's per-GPU scratch array).  Returns ``out``."""
    s = current_stream_handle() if stream is None else stream
    check(load().tamm_contract_noalloc(out._h, ol.encode(), lhs._h, ll.encode(), rhs._h, rl.encode(),
                                       PRECISIONS[precision], float(alpha), float(beta), s))
    return out


def contract_cache_count() -> int:
    """Number of one-shot plans in the library's cache."""
    n = ctypes.c_int64()
    check(load().tamm_contract_cache_count(ctypes.byref(n)))
    return n.value


def contract_cache_clear() -> None:
    """Drop every cached one-shot plan (and forget what each workspace holds)."""
    check(load().tamm_contract_cache_clear())


class Denominator:
    """out = in / D with D from per-dimension orbital energies (device tensors) and signs."""

    def __init__(self, out: Tensor, inp: Tensor, energies: Sequence, signs: Sequence[int]):
        torch = _torch()
        self.out, self.inp = out, inp
        self.energies = [None if e is None else e.to(dtype=torch.float64).contiguous() for e in energies]
        sg = np.ascontiguousarray(np.asarray(signs, dtype=np.int8))
        h = ctypes.c_void_p()
        check(load().tamm_denominator_create(out._h, inp._h, sg.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                             ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        check(load().tamm_denominator_workspace_size(self._h, ctypes.byref(n)))
        self.ws_bytes = n.value
        self._ws, ptr = _aligned_workspace(self.ws_bytes, out.data.device)
        check(load().tamm_denominator_bind_workspace(self._h, ctypes.c_void_p(ptr), self.ws_bytes))
        self._eptr = (ctypes.c_void_p * out.rank)(*[(0 if e is None else e.data_ptr()) for e in self.energies])

    def execute(self, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_denominator_execute(self._h, self._eptr, s))

    def __del__(self, _d=_destroy):
        _d(self, "tamm_denominator_destroy")


class CholeskyLadder:
    """R[abij] = beta R + alpha sum_cd V[abcd] T[cdij] with V rebuilt from Cholesky vectors
    B[p,q,L] by Eq. (cc12), V never formed (tamm_chol_ladder_*)."""

    def __init__(self, R: Tensor, T: Tensor, B: Tensor, strip_tiles: int = 0):
        self.R, self.T, self.B = R, T, B
        lib = load()
        h = ctypes.c_void_p()
        check(lib.tamm_chol_ladder_create(R._h, T._h, B._h, int(strip_tiles), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        check(lib.tamm_chol_ladder_workspace_size(self._h, ctypes.byref(n)))
        self.ws_bytes = n.value
        self._ws = None
        if R.data is not None:  # structure-only tensors (no device) plan without binding
            self._ws, ptr = _aligned_workspace(self.ws_bytes, R.data.device)
            check(lib.tamm_chol_ladder_bind_workspace(self._h, ctypes.c_void_p(ptr), self.ws_bytes))

    def execute(self, alpha: float = 0.5, beta: float = 0.0, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_chol_ladder_execute(self._h, float(alpha), float(beta), s))

    def autotune(self, cache_path: str = "", reps: int = 3, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_chol_ladder_autotune(self._h, s, cache_path.encode(), int(reps)))

    def stats(self) -> dict:
        bf, lf = ctypes.c_double(), ctypes.c_double()
        ns, gm, tm_ = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(load().tamm_chol_ladder_stats(self._h, ctypes.byref(bf), ctypes.byref(lf), ctypes.byref(ns),
                                            ctypes.byref(gm), ctypes.byref(tm_)))
        return {"build_flops": bf.value, "ladder_flops": lf.value, "strips": ns.value, "g_max_elements": gm.value,
                "tm_elements": tm_.value, "workspace_bytes": self.ws_bytes}

    def strip_plan_stats(self, strip: int) -> Tuple[dict, dict]:
        """Plan statistics of one strip's pair product and ladder (tamm_plan_stats)."""
        b, l = ctypes.c_void_p(), ctypes.c_void_p()
        check(load().tamm_chol_ladder_strip_plans(self._h, int(strip), ctypes.byref(b), ctypes.byref(l)))
        res = []
        for h in (b, l):
            st = PlanStats()
            check(load().tamm_plan_stats_get(h, ctypes.byref(st)))
            res.append({f: getattr(st, f) for f, _ in PlanStats._fields_})
        return res[0], res[1]

    def __del__(self, _d=_destroy):
        _d(self, "tamm_chol_ladder_destroy")


def set_value(out: Tensor, alpha: float, stream=None) -> Tensor:
    """SetOp: every stored element of ``out`` becomes ``alpha`` (tamm_set)."""
    s = current_stream_handle() if stream is None else stream
    check(load().tamm_set(out._h, float(alpha), s))
    return out


class Add:
    """AddOp with a label permutation: out(ol) = beta*out(ol) + alpha*in(il) (tamm_add_*)."""

    def __init__(self, out: Tensor, ol: str, inp: Tensor, il: str, bind: bool = True):
        self.out, self.inp = out, inp  # kept alive as long as the operation
        self.labels = (ol, il)
        h = ctypes.c_void_p()
        check(load().tamm_add_create(out._h, ol.encode(), inp._h, il.encode(), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        check(load().tamm_add_workspace_size(self._h, ctypes.byref(n)))
        self.ws_bytes = n.value
        self._ws = None
        if bind and out.data is not None:
            self.bind_workspace(out.data.device)

    def bind_workspace(self, device):
        self._ws, ptr = _aligned_workspace(self.ws_bytes, device)
        check(load().tamm_add_bind_workspace(self._h, ctypes.c_void_p(ptr), self.ws_bytes))

    def execute(self, alpha: float = 1.0, beta: float = 0.0, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_add_execute(self._h, float(alpha), float(beta), s))

    def __del__(self, _d=_destroy):
        _d(self, "tamm_add_destroy")


class Scheduler:
    """Queue of SetOp / AddOp / MultOp / denominator operations, analysed once into fused nodes and
    dataflow levels and executed level by level (tamm_sched_*).  Keeps every queued object alive."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(load().tamm_sched_create(ctypes.byref(h)))
        self._h = h
        self._keep = []
        self._ws = None
        self.n_ops = 0

    def set(self, out: Tensor, alpha: float):
        check(load().tamm_sched_set(self._h, out._h, float(alpha)))
        self._keep.append(out)
        self.n_ops += 1
        return self

    def add(self, op: "Add", alpha: float = 1.0, beta: float = 0.0):
        check(load().tamm_sched_add(self._h, op._h, float(alpha), float(beta)))
        self._keep.append(op)
        self.n_ops += 1
        return self

    def contract(self, plan: Plan, alpha: float = 1.0, beta: float = 0.0):
        check(load().tamm_sched_contract(self._h, plan._h, float(alpha), float(beta)))
        self._keep.append(plan)
        self.n_ops += 1
        return self

    def denominator(self, den: "Denominator"):
        check(load().tamm_sched_denominator(self._h, den._h, den._eptr))
        self._keep.append(den)
        self.n_ops += 1
        return self

    def build(self):
        check(load().tamm_sched_build(self._h))
        return self

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        check(load().tamm_sched_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def bind_workspace(self, device="cuda"):
        n = self.workspace_size()
        self._ws, ptr = _aligned_workspace(n, device)
        check(load().tamm_sched_bind_workspace(self._h, ctypes.c_void_p(ptr), n))
        return self

    def autotune(self, cache_path: str = "", reps: int = 2, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_sched_autotune(self._h, s, cache_path.encode(), reps))

    def execute(self, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_sched_execute(self._h, s))

    def capture(self, stream=None):
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_sched_capture(self._h, s))

    def info(self) -> dict:
        lv, nd, fu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(load().tamm_sched_info(self._h, ctypes.byref(lv), ctypes.byref(nd), ctypes.byref(fu)))
        return {"levels": lv.value, "nodes": nd.value, "fused_ops": fu.value}

    def op_info(self, i: int):
        lv, nd = ctypes.c_int32(), ctypes.c_int32()
        check(load().tamm_sched_op_info(self._h, i, ctypes.byref(lv), ctypes.byref(nd)))
        return lv.value, nd.value

    def __del__(self, _d=_destroy):
        _d(self, "tamm_sched_destroy")


class Group:
    """Independent float64 plans executed as one grouped persistent launch (optionally a hipGraph)."""

    def __init__(self, plans: Sequence[Plan]):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        check(load().tamm_group_create(arr, len(self.plans), ctypes.byref(h)))
        self._h = h
        self._ws = None
        self.device = self.plans[0].out.data.device if self.plans[0].out.data is not None else None
        if self.device is not None:
            self.bind_workspace()

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        check(load().tamm_group_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def bind_workspace(self, nbytes: Optional[int] = None):
        nbytes = self.workspace_size() if nbytes is None else nbytes
        self._ws, ptr = _aligned_workspace(nbytes, self.device)
        self._ws_bytes = nbytes
        check(load().tamm_group_bind_workspace(self._h, ctypes.c_void_p(ptr), nbytes))

    def set_config(self, config: int = -1, grid: int = 0):
        check(load().tamm_group_set_config(self._h, config, grid))
        if self.device is not None:
            self.bind_workspace()

    def stats(self) -> dict:
        c, g, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        check(load().tamm_group_stats(self._h, ctypes.byref(c), ctypes.byref(g), ctypes.byref(n)))
        return {"config": c.value, "grid": g.value, "work_items": n.value,
                "config_name": load().tamm_config_name(0, c.value).decode()}

    @staticmethod
    def _arr(vals, n):
        v = [float(x) for x in vals] if hasattr(vals, "__len__") else [float(vals)] * n
        return (ctypes.c_double * n)(*v)

    def execute(self, alpha, beta, stream=None):
        n = len(self.plans)
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_group_execute(self._h, self._arr(alpha, n), self._arr(beta, n), s))

    def capture(self, alpha, beta, stream=None):
        n = len(self.plans)
        s = current_stream_handle() if stream is None else stream
        check(load().tamm_group_capture(self._h, self._arr(alpha, n), self._arr(beta, n), s))

    def autotune(self, cache_path: str = "", reps: int = 3, stream=None):
        s = current_stream_handle() if stream is None else stream
        # the largest workspace any candidate needs: try every configuration's size
        best = self.workspace_size()
        lib = load()
        cur = self.stats()
        cnt = ctypes.c_int32()
        check(lib.tamm_plan_config_count(self.plans[0]._h, ctypes.byref(cnt)))
        for c in range(cnt.value):
            check(lib.tamm_group_set_config(self._h, c, 0))
            best = max(best, self.workspace_size())
        check(lib.tamm_group_set_config(self._h, cur["config"], cur["grid"]))
        self.bind_workspace(best)
        check(lib.tamm_group_autotune(self._h, s, cache_path.encode(), reps))

    def __del__(self, _d=_destroy):
        _d(self, "tamm_group_destroy")


__all__ = ["Space", "Tensor", "Plan", "Group", "contract", "Denominator", "Add", "set_value", "Scheduler", "TammError",
           "PRECISIONS", "CholeskyLadder", "spin_diagonal"]
