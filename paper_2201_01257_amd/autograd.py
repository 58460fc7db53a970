"""Hand-written adjoint of the block-sparse contraction, exposed as a torch.autograd.Function.

Forward: out = beta * out0 + alpha * contract(lhs, rhs).  Backward, for an upstream gradient g
on out's stored blocks:

    d lhs  = alpha * contract(g, rhs)   onto lhs's labels and stored blocks,
    d rhs  = alpha * contract(lhs, g)   onto rhs's labels and stored blocks,
    d out0 = beta * g.

Both gradients are block-sparse contractions of the same kind as the forward one and run on the
same HIP kernels (screening, gathers, MFMA, epilogue); d out0 is an AddOp of the library.  The
primal operands are re-gathered from
their storage in the backward pass (nothing permuted is saved).  The paper defines no adjoint;
this is the chain rule applied to the bilinear contraction of Sec. III-A, Fig. 3 rule 8.

Block-sparse tensors are passed as their flat storage (float64 torch tensors in the stored-block
layout of the structure ``Tensor`` objects); the structures are re-bound to whichever storage a
call uses, so one set of plans serves every call.
"""

from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import core as tm


class Contraction:
    """A contraction with fixed structure and labels, differentiable in both operands and out0."""

    def __init__(self, out: tm.Tensor, ol: str, lhs: tm.Tensor, ll: str, rhs: tm.Tensor, rl: str,
                 alpha: float = 1.0, beta: float = 0.0):
        self.ol, self.ll, self.rl = ol, ll, rl
        self.alpha, self.beta = float(alpha), float(beta)
        # private structure handles (re-bound to call storages); storage-less until bound.  Each
        # is built from the caller's spaces and non-zero check, so its stored blocks and their
        # offsets are those of the caller's tensor (checked).
        self.S_out, self.S_gout, self.S_gout0 = (_clone_structure(out) for _ in range(3))
        self.S_lhs, self.S_glhs = (_clone_structure(lhs) for _ in range(2))
        self.S_rhs, self.S_grhs = (_clone_structure(rhs) for _ in range(2))
        self._plans: Dict[str, tm.Plan] = {}
        self._scale: Optional[tm.Add] = None  # d out0 = beta * g (an AddOp in the library)

    def _plan(self, key: str) -> tm.Plan:
        p = self._plans.get(key)
        if p is None:
            if key == "fwd":
                p = tm.Plan(self.S_out, self.ol, self.S_lhs, self.ll, self.S_rhs, self.rl, bind=False)
            elif key == "dlhs":
                p = tm.Plan(self.S_glhs, self.ll, self.S_gout, self.ol, self.S_rhs, self.rl, bind=False)
            else:
                p = tm.Plan(self.S_grhs, self.rl, self.S_lhs, self.ll, self.S_gout, self.ol, bind=False)
            self._plans[key] = p
        return p

    def _run(self, key: str, alpha: float, beta: float, device):
        p = self._plan(key)
        if p._ws is None or p._ws.device != device:
            p._ws, ptr = tm._aligned_workspace(p.workspace_size(), device)
            tm.check(tm.load().tamm_plan_bind_workspace(p._h, tm.ctypes.c_void_p(ptr), p.workspace_size()))
        p.execute(alpha, beta)

    def autotune(self, cache_path: str = "", reps: int = 2):
        """Run the library's autotuner on every plan built so far (forward and, after a backward
        pass, both gradient plans) on the storages of the last call; outputs are left unchanged."""
        for p in self._plans.values():
            p.autotune(cache_path, reps=reps)

    def __call__(self, lhs_data: torch.Tensor, rhs_data: torch.Tensor, out0_data: Optional[torch.Tensor] = None):
        return _ContractFn.apply(lhs_data, rhs_data, out0_data, self)


def _clone_structure(t: tm.Tensor) -> tm.Tensor:
    """A storage-less tensor with the spaces and non-zero check of ``t``; its block table and
    block offsets must equal ``t``'s (so storage laid out for ``t`` binds to it unchanged)."""
    s = tm.Tensor(t.spaces, nonzero=t.nonzero, device=None)
    if s.numel != t.numel or not np.array_equal(s.block_tiles, t.block_tiles) or \
            not np.array_equal(s.block_off, t.block_off):
        raise ValueError("the tensor's block structure could not be reproduced from its spaces and non-zero check")
    return s


def _bind(struct: tm.Tensor, data: torch.Tensor):
    if data.dtype != torch.float64 or not data.is_contiguous() or data.numel() < struct.numel:
        raise ValueError("storage must be a contiguous float64 tensor with the structure's element count")
    tm.check(tm.load().tamm_tensor_bind(struct._h, tm.ctypes.c_void_p(data.data_ptr()), data.numel() * 8))
    struct.data = data


class _ContractFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lhs_data, rhs_data, out0_data, c: Contraction):
        dev = lhs_data.device
        out = torch.empty(max(c.S_out.numel, 1), dtype=torch.float64, device=dev)
        beta = c.beta if out0_data is not None else 0.0
        if beta != 0.0:
            out.copy_(out0_data)
        _bind(c.S_lhs, lhs_data)
        _bind(c.S_rhs, rhs_data)
        _bind(c.S_out, out)
        c._run("fwd", c.alpha, beta, dev)
        ctx.c = c
        ctx.has_out0 = out0_data is not None
        ctx.save_for_backward(lhs_data, rhs_data)
        return out

    @staticmethod
    def backward(ctx, g):
        c: Contraction = ctx.c
        lhs_data, rhs_data = ctx.saved_tensors
        dev = g.device
        g = g.contiguous()
        _bind(c.S_gout, g)
        _bind(c.S_lhs, lhs_data)
        _bind(c.S_rhs, rhs_data)
        g_lhs = g_rhs = g_out0 = None
        if ctx.needs_input_grad[0]:
            g_lhs = torch.empty(max(c.S_lhs.numel, 1), dtype=torch.float64, device=dev)
            _bind(c.S_glhs, g_lhs)
            c._run("dlhs", c.alpha, 0.0, dev)
        if ctx.needs_input_grad[1]:
            g_rhs = torch.empty(max(c.S_rhs.numel, 1), dtype=torch.float64, device=dev)
            _bind(c.S_grhs, g_rhs)
            c._run("drhs", c.alpha, 0.0, dev)
        if ctx.has_out0 and ctx.needs_input_grad[2]:
            g_out0 = torch.empty(max(c.S_out.numel, 1), dtype=torch.float64, device=dev)
            _bind(c.S_gout0, g_out0)
            if c._scale is None:
                c._scale = tm.Add(c.S_gout0, c.ol, c.S_gout, c.ol, bind=False)
            if c._scale._ws is None or c._scale._ws.device != dev:
                c._scale.bind_workspace(dev)
            c._scale.execute(c.beta, 0.0)
        return g_lhs, g_rhs, g_out0, None


__all__ = ["Contraction"]
