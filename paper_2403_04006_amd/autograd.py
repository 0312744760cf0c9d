"""torch.autograd Functions over the library's kernels (argument marshalling
only): a beamsplitter mesh (angles -> U), permanents of many output patterns
(U -> perm), and the mean negative log-probability (perm -> loss).  Chained,
gradients flow from the loss to every mesh angle through the adjoint
Gray-code sweep.

This is the paper's differentiable-circuit use (Goals: machine learning
support with automatic differentiation and custom gradients; Benchmarks /
Fock-space based simulations, Differentiability: the gradient of a cost with
respect to the gate parameters of one photonic layer), with the
"Beamsplitter gate" section's cells as the parameterised gates.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import PatternSet, _lib, _check, _stream_handle, engine as _engine

__all__ = ["MeshUnitary", "PermAmp", "NegLogProb", "mesh_unitary", "perm_amp", "neg_log_prob", "mesh_loss"]


def _modes_array(cells: Sequence[tuple]):
    flat = [int(x) for pair in cells for x in pair]
    return _lib.i32_array(flat), len(cells)


class MeshUnitary(torch.autograd.Function):
    """U = B_last ... B_1 from (ncell, 2) float64 angles (theta, phi)."""

    @staticmethod
    def forward(ctx, angles: torch.Tensor, cells: tuple, m: int):
        eng = _engine(angles.device.index)
        angles = angles.detach().to(torch.float64).contiguous()
        modes, ncell = _modes_array(cells)
        U = torch.empty((m, m), dtype=torch.complex128, device=angles.device)
        _check(eng._lib.pq_mesh_unitary(eng._ctx, m, ncell, modes, angles.data_ptr(), U.data_ptr(), m,
                                        _stream_handle(angles.device)), eng._ctx)
        ctx.save_for_backward(angles)
        ctx.cells = cells
        ctx.m = m
        return U

    @staticmethod
    def backward(ctx, gU: torch.Tensor):
        (angles,) = ctx.saved_tensors
        eng = _engine(angles.device.index)
        gU = gU.to(torch.complex128).contiguous()
        modes, ncell = _modes_array(ctx.cells)
        gang = torch.empty_like(angles)
        _check(eng._lib.pq_mesh_unitary_vjp(eng._ctx, ctx.m, ncell, modes, angles.data_ptr(), gU.data_ptr(),
                                            gU.stride(0), gang.data_ptr(), _stream_handle(angles.device)),
               eng._ctx)
        return gang, None, None


def _sparse(v):
    return [(i, int(c)) for i, c in enumerate(v) if int(c) > 0]


class PermAmp(torch.autograd.Function):
    """perm(U_{T_p,S_p}) for every pattern of a PatternSet (forward:
    pq_perm_many; backward: pq_perm_grad, the adjoint sweep).  The amplitude
    is Eq. BS_prob's; its gradient, d perm / d U_ij = t_i s_j perm(U_{T-e_i,
    S-e_j}), is what the Differentiability benchmark (Fock-space based
    simulations) needs from a circuit's transition amplitudes."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, pats: PatternSet):
        eng = _engine(U.device.index)
        U = U.detach().contiguous()
        perm, _ = eng.perm_patterns(U, pats)
        ctx.save_for_backward(U)
        ctx.pats = pats
        return perm

    @staticmethod
    def backward(ctx, gperm: torch.Tensor):
        (U,) = ctx.saved_tensors
        eng = _engine(U.device.index)
        dU, _ = eng.grad_patterns(U, ctx.pats, gperm.contiguous())
        return dU, None


class NegLogProb(torch.autograd.Function):
    """-(1/N) sum_p (log|perm_p|^2 - log_norm_p)."""

    @staticmethod
    def forward(ctx, perm: torch.Tensor, log_norm: torch.Tensor | None = None):
        eng = _engine(perm.device.index)
        perm = perm.detach().contiguous()
        loss = torch.empty((), dtype=torch.float64, device=perm.device)
        ln = log_norm.detach().to(torch.float64).contiguous() if log_norm is not None else None
        _check(eng._lib.pq_neg_log_prob(eng._ctx, perm.numel(), perm.data_ptr(),
                                        ln.data_ptr() if ln is not None else None, loss.data_ptr(),
                                        _stream_handle(perm.device)), eng._ctx)
        ctx.save_for_backward(perm)
        return loss

    @staticmethod
    def backward(ctx, gloss: torch.Tensor):
        (perm,) = ctx.saved_tensors
        eng = _engine(perm.device.index)
        gl = gloss.detach().to(torch.float64).contiguous()
        gperm = torch.empty_like(perm)
        _check(eng._lib.pq_neg_log_prob_vjp(eng._ctx, perm.numel(), perm.data_ptr(), gl.data_ptr(),
                                            gperm.data_ptr(), _stream_handle(perm.device)), eng._ctx)
        return gperm, None


def mesh_unitary(angles: torch.Tensor, cells, m: int) -> torch.Tensor:
    return MeshUnitary.apply(angles, tuple(tuple(c) for c in cells), m)


def perm_amp(U: torch.Tensor, S_list, T_list=None) -> torch.Tensor:
    """Permanents of a PatternSet, or of (S_list, T_list) marshalled on the fly."""
    pats = S_list if isinstance(S_list, PatternSet) else PatternSet(S_list, T_list, U.shape[0])
    return PermAmp.apply(U, pats)


def neg_log_prob(perm: torch.Tensor, log_norm: torch.Tensor | None = None) -> torch.Tensor:
    return NegLogProb.apply(perm, log_norm)


def mesh_loss(angles: torch.Tensor, cells, m: int, S, T_list=None, log_norm: torch.Tensor | None = None):
    """Loss of output patterns T_list for input S through the mesh (or of a
    prepared PatternSet passed as S)."""
    U = mesh_unitary(angles, cells, m)
    pats = S if isinstance(S, PatternSet) else PatternSet([S] * len(T_list), T_list, m)
    perm = perm_amp(U, pats)
    return neg_log_prob(perm, log_norm)
