"""Differentiable propagation: torch.autograd.Function over gqd_propagate / gqd_adjoint.

Forward propagates psi(0) to psi(T) with the composed implicit midpoint method and
keeps only psi(T).  Backward runs the reverse sweep of the C library: every substep is
inverted exactly (time reversibility of the Cayley map), so the states are rebuilt on
the way back instead of being stored, and the sweep returns dL/dpsi*(0) and dL/dF12 on
the grid.  torch's complex gradients are 2 dL/dpsi*; the sweep is linear in the
incoming gradient, so it takes torch's gradient as is and halves the F12 part.

The torch builders below make psi(0) and F12 from parameters (centre, momentum, width;
coupling amplitude and centre) so that torch applies the chain rule to them.
"""
from __future__ import annotations

import math
from typing import Optional

import torch

from . import gqd


class PropagateFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0: torch.Tensor, F: torch.Tensor, prop: "gqd.Propagator", scheme: str,
                order: int, dt: float, nsteps: int, opts: Optional[gqd.SolverOpts]):
        Fd = F.detach().contiguous()
        prop.set_surfaces(prop.V, Fd)
        psi = psi0.detach().contiguous().clone()
        prop.propagate(psi, "midp", scheme, order, dt, nsteps, opts)
        ctx.save_for_backward(psi, Fd)
        ctx.cfg = (prop, scheme, order, dt, nsteps, opts)
        return psi

    @staticmethod
    def backward(ctx, grad_psiT: torch.Tensor):
        psiT, Fd = ctx.saved_tensors
        prop, scheme, order, dt, nsteps, opts = ctx.cfg
        prop.set_surfaces(prop.V, Fd)
        psi = psiT.clone()
        lam = grad_psiT.contiguous().to(torch.complex128).clone()
        gF = torch.zeros_like(Fd)
        prop.adjoint(psi, lam, gF, scheme, order, dt, nsteps, opts)
        ctx.reconstructed_psi0 = psi
        return lam, 0.5 * gF, None, None, None, None, None, None


def propagate(prop: "gqd.Propagator", psi0: torch.Tensor, F: torch.Tensor, scheme: str = "suzuki",
              order: int = 4, dt: float = 4.0, nsteps: int = 1,
              opts: Optional[gqd.SolverOpts] = None) -> torch.Tensor:
    """psi(T) from psi(0) and the coupling F12 (flat device tensors of the batch layout),
    differentiable with respect to both."""
    return PropagateFn.apply(psi0, F, prop, scheme, order, dt, nsteps, opts)


# ------------------------------------------------------------ differentiable inputs

def grid(n: int, qmin: float, qmax: float, device) -> torch.Tensor:
    return qmin + torch.arange(n, dtype=torch.float64, device=device) * ((qmax - qmin) / n)


def gaussian_packet(q: torch.Tensor, q0, p0, width) -> torch.Tensor:
    """(2, n) complex128: a Gaussian on surface index 0 (|psi|^2 has standard deviation
    `width`), renormalised on the grid; differentiable in q0, p0, width."""
    dq = q[1] - q[0]
    x = q - q0
    g = torch.exp(torch.complex(-(x * x) / (4.0 * width * width), p0 * x))
    g = g / torch.sqrt(dq * torch.sum(torch.abs(g) ** 2))
    return torch.stack([g, torch.zeros_like(g)])


def gaussian_packets(q: torch.Tensor, q0: torch.Tensor, p0: torch.Tensor, width: torch.Tensor) -> torch.Tensor:
    """(B, 2, n): gaussian_packet for parameter vectors of length B, built in one go."""
    dq = q[1] - q[0]
    w = width[:, None]
    x = q[None, :] - q0[:, None]
    g = torch.exp(torch.complex(-(x * x) / (4.0 * w * w), p0[:, None] * x))
    g = g / torch.sqrt(dq * torch.sum(torch.abs(g) ** 2, dim=1, keepdim=True))
    return torch.stack([g, torch.zeros_like(g)], dim=1)


def coupling(q: torch.Tensor, amp, center, cwidth: float = 0.5) -> torch.Tensor:
    """F12 = amp exp(-((q - center)/cwidth)^2), differentiable in amp and center."""
    return amp * torch.exp(-(((q - center) / cwidth) ** 2))


def couplings(q: torch.Tensor, amp: torch.Tensor, center: torch.Tensor, cwidth: float = 0.5) -> torch.Tensor:
    """(B, n): coupling for parameter vectors of length B."""
    return amp[:, None] * torch.exp(-(((q[None, :] - center[:, None]) / cwidth) ** 2))


def surface_population(psi: torch.Tensor, dq: float, surface: int = 1) -> torch.Tensor:
    """dq sum |psi_surface|^2 of one item, psi of shape (2, n) (2D: (2, n1, n2) and the
    volume element dq1 dq2)."""
    return dq * torch.sum(torch.abs(psi[surface]) ** 2)


def grid2d(n: int, qmin, qmax, device):
    """(Q1, Q2) of an n x n grid, q1 the slow index."""
    q1 = grid(n, qmin[0], qmax[0], device)
    q2 = grid(n, qmin[1], qmax[1], device)
    return torch.meshgrid(q1, q2, indexing="ij")


def coupling_2d(Q1: torch.Tensor, Q2: torch.Tensor, amp, c1, c2, w, direction=(0.8, 0.6)) -> torch.Tensor:
    """(2, n, n): F12^(d) = amp exp(-((q1 - c1)^2 + (q2 - c2)^2) / w^2) direction_d,
    differentiable in amp, c1, c2, w."""
    g = amp * torch.exp(-((Q1 - c1) ** 2 + (Q2 - c2) ** 2) / (w * w))
    return torch.stack([direction[0] * g, direction[1] * g])


def gaussian_packet_2d(Q1: torch.Tensor, Q2: torch.Tensor, q0, p0, width) -> torch.Tensor:
    """(2, n, n) complex128: a product Gaussian on surface index 0 (|psi|^2 has standard
    deviations width), renormalised on the grid."""
    dv = float((Q1[1, 0] - Q1[0, 0]) * (Q2[0, 1] - Q2[0, 0]))
    x1, x2 = Q1 - q0[0], Q2 - q0[1]
    g = torch.exp(torch.complex(-(x1 * x1) / (4.0 * width[0] ** 2) - (x2 * x2) / (4.0 * width[1] ** 2),
                                p0[0] * x1 + p0[1] * x2))
    g = g / torch.sqrt(dv * torch.sum(torch.abs(g) ** 2))
    return torch.stack([g, torch.zeros_like(g)])
