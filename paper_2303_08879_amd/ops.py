"""PyTorch-facing API: plan caching, device buffers from the torch allocator,
and a torch.autograd.Function whose backward is the library's reverse sweep."""
from __future__ import annotations

import torch

from . import fockdiag as F

_plans = {}


def get_plan(cutoffs, detected_mask, dtype=torch.complex128, b_mode="auto"):
    key = (tuple(int(c) for c in cutoffs), int(detected_mask), dtype, b_mode)
    p = _plans.get(key)
    if p is None:
        p = F.Plan(cutoffs, detected_mask, dtype, b_mode)
        _plans[key] = p
    return p


def _as_inputs(A, b, c, dtype, device):
    A = torch.as_tensor(A, dtype=dtype, device=device).contiguous()
    b = torch.as_tensor(b, dtype=dtype, device=device).contiguous()
    c = torch.as_tensor(c, dtype=dtype, device=device).reshape(1).contiguous()
    return A, b, c


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def fock_diag(A, b, c, cutoffs, detected_mask, dtype=torch.complex128, b_mode="auto", device="cuda"):
    """rho[k_U, l_U, n_D] (no autograd)."""
    plan = get_plan(cutoffs, detected_mask, dtype, b_mode)
    A, b, c = _as_inputs(A, b, c, dtype, device)
    ws_bytes, _ = plan.workspace(False)
    ws = _workspace(ws_bytes, device)
    rho = torch.empty(plan.out_shape, dtype=dtype, device=device)
    F.fock_diag_fwd(plan, A, b, c, rho, ws)
    return rho


def detection_probs(A, b, c, cutoffs, dtype=torch.complex128, b_mode="auto", device="cuda"):
    """p(n) for every n < cutoffs (all modes detected)."""
    mask = (1 << len(cutoffs)) - 1
    plan = get_plan(cutoffs, mask, dtype, b_mode)
    A, b, c = _as_inputs(A, b, c, dtype, device)
    ws_bytes, _ = plan.workspace(False)
    ws = _workspace(ws_bytes, device)
    probs = torch.empty(plan.out_shape, dtype=dtype, device=device)
    F.detection_probs(plan, A, b, c, probs, ws)
    return probs


def fock_diag_batch(triples, shapes, dtype=torch.complex128, b_mode="auto", device="cuda"):
    """rho of every circuit of a batch in one batched call.  ``triples`` is a
    list of (A, b, c), ``shapes`` a list of (cutoffs, detected_mask)."""
    plans = [get_plan(cut, mask, dtype, b_mode) for cut, mask in shapes]
    ins = [_as_inputs(A, b, c, dtype, device) for A, b, c in triples]
    ws = [_workspace(p.workspace(False)[0], device) for p in plans]
    rho = [torch.empty(p.out_shape, dtype=dtype, device=device) for p in plans]
    F.fock_diag_fwd_batch(plans, [x[0] for x in ins], [x[1] for x in ins], [x[2] for x in ins], rho, ws)
    return rho


_state_plans = {}


def get_state_plan(cutoffs, dtype=torch.complex128, b_mode="auto"):
    key = (tuple(int(c) for c in cutoffs), dtype, b_mode)
    p = _state_plans.get(key)
    if p is None:
        p = F.StatePlan(cutoffs, dtype, b_mode)
        _state_plans[key] = p
    return p


def state_vector(A, b, c, cutoffs, dtype=torch.complex128, b_mode="auto", device="cuda"):
    """psi[n] = <n|psi>, 0 <= n < cutoffs, of the pure state with triple
    (A: M x M, b: M, c) -- fock_state_fwd."""
    plan = get_state_plan(cutoffs, dtype, b_mode)
    A, b, c = _as_inputs(A, b, c, dtype, device)
    ws = _workspace(plan.workspace(), device)
    psi = torch.empty(plan.out_shape, dtype=dtype, device=device)
    F.fock_state_fwd(plan, A, b, c, psi, ws)
    return psi


class FockDiagFunction(torch.autograd.Function):
    """rho = fock_diag(A, b, c); backward = fock_diag_vjp with the saved
    intermediate amplitudes (PyTorch's complex-gradient convention: the
    incoming gradient g yields sum g conj(d rho / d x)); forward-mode AD with
    dual tensors (torch.autograd.forward_ad) = fock_diag_jvp (rho is
    holomorphic in A, b, c, so the tangent is sum dx d rho / d x)."""

    @staticmethod
    def forward(ctx, A, b, c, cutoffs, detected_mask, b_mode):
        dtype = A.dtype
        plan = get_plan(cutoffs, detected_mask, dtype, b_mode)
        A_, b_, c_ = A.contiguous(), b.contiguous(), c.reshape(1).contiguous()
        ws_bytes, saved_bytes = plan.workspace(True)
        ws = _workspace(ws_bytes, A.device)
        saved = _workspace(saved_bytes, A.device)
        rho = torch.empty(plan.out_shape, dtype=dtype, device=A.device)
        F.fock_diag_fwd(plan, A_, b_, c_, rho, ws, saved)
        ctx.plan = plan
        ctx.saved_buf = saved
        ctx.c_shape = c.shape
        ctx.save_for_backward(A_, b_, c_)
        ctx.save_for_forward(A_, b_, c_)
        return rho

    @staticmethod
    def jvp(ctx, dA, db, dc, *_):
        A, b, c = ctx.saved_tensors
        plan = ctx.plan
        tan = lambda t, ref: torch.zeros_like(ref) if t is None else t.reshape(ref.shape).contiguous()
        ws = _workspace(plan.jvp_workspace(), A.device)
        rho = torch.empty(plan.out_shape, dtype=A.dtype, device=A.device)
        drho = torch.empty_like(rho)
        F.fock_diag_jvp(plan, A, b, c, tan(dA, A), tan(db, b), tan(dc, c), rho, drho, ws)
        return drho

    @staticmethod
    def backward(ctx, grad_rho):
        A, b, c = ctx.saved_tensors
        plan = ctx.plan
        g = grad_rho.contiguous()
        ws_bytes, _ = plan.workspace(True)
        ws = _workspace(ws_bytes, A.device)
        dA = torch.empty_like(A)
        db = torch.empty_like(b)
        dc = torch.empty_like(c)
        F.fock_diag_vjp(plan, A, b, c, ctx.saved_buf, g, dA, db, dc, ws)
        return dA, db, dc.reshape(ctx.c_shape), None, None, None


def fock_diag_ad(A, b, c, cutoffs, detected_mask, b_mode="auto"):
    """Differentiable rho[k_U, l_U, n_D] w.r.t. (A, b, c)."""
    return FockDiagFunction.apply(A, b, c, tuple(cutoffs), int(detected_mask), b_mode)


class StateVectorFunction(torch.autograd.Function):
    """psi = state_vector(A, b, c); backward = fock_state_vjp (the cotangents
    sum_k g_k conj(d psi_k / d x), PyTorch's convention for holomorphic maps;
    A enters as its symmetric part); forward-mode AD with dual tensors
    (torch.autograd.forward_ad) = fock_state_jvp."""

    @staticmethod
    def forward(ctx, A, b, c, cutoffs, b_mode):
        dtype = A.dtype
        plan = get_state_plan(cutoffs, dtype, b_mode)
        A_, b_, c_ = A.contiguous(), b.contiguous(), c.reshape(1).contiguous()
        ws = _workspace(plan.workspace(), A.device)
        psi = torch.empty(plan.out_shape, dtype=dtype, device=A.device)
        F.fock_state_fwd(plan, A_, b_, c_, psi, ws)
        ctx.plan = plan
        ctx.c_shape = c.shape
        ctx.save_for_backward(c_, psi)
        ctx.save_for_forward(c_, psi)
        return psi

    @staticmethod
    def jvp(ctx, dA, db, dc, *_):
        c, psi = ctx.saved_tensors
        M = len(ctx.plan.cutoffs)
        tan = lambda t, shape: (torch.zeros(shape, dtype=psi.dtype, device=psi.device) if t is None
                                else t.reshape(shape).contiguous())
        dpsi = torch.empty_like(psi)
        F.fock_state_jvp(ctx.plan, c, psi, tan(dA, (M, M)), tan(db, (M,)), tan(dc, (1,)), dpsi)
        return dpsi

    @staticmethod
    def backward(ctx, grad_psi):
        c, psi = ctx.saved_tensors
        plan = ctx.plan
        ws = _workspace(plan.vjp_workspace(), psi.device)
        M = len(plan.cutoffs)
        dA = torch.empty((M, M), dtype=psi.dtype, device=psi.device)
        db = torch.empty(M, dtype=psi.dtype, device=psi.device)
        dc = torch.empty(1, dtype=psi.dtype, device=psi.device)
        F.fock_state_vjp(plan, c, psi, grad_psi.contiguous(), dA, db, dc, ws)
        return dA, db, dc.reshape(ctx.c_shape), None, None


def state_vector_ad(A, b, c, cutoffs, b_mode="auto"):
    """state_vector with autograd support (A, b, c device tensors)."""
    return StateVectorFunction.apply(A, b, c, tuple(int(x) for x in cutoffs), b_mode)

