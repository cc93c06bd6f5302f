"""Differentiable ROK step with exact products, for gradient checks.

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

The step of Sec. 2.2.2, eq. (9) with the Krylov basis built by modified
Arnoldi on exact products J(y_n) v (Sec. 2.3), written with plain torch
operations so that torch's reverse-mode differentiation yields the gradient
of the computed step with respect to y_n.  Everything the step computes
depends on y_n, the basis V and the Hessenberg matrix H included, so the
gradient carries the derivative of every modified Gram-Schmidt pass and of
every product J(y_n) v_j with respect to both y_n and v_j.

The arithmetic is that of oracle.rok.rok_step with plain torch reductions
in place of the canonical summation order, so values agree with it to
rounding, which the pins check; gradients are pinned against central
differences of oracle.rok.rok_step.
"""
from __future__ import annotations

import torch

from . import fv
from .krylov import BREAKDOWN_TOL


def jvp_exact(P: fv.Problem, y: torch.Tensor, v: torch.Tensor, forward: bool = False) -> torch.Tensor:
    """J(y) v, differentiable with respect to y and v.

    forward=False: double-backward form, for reverse-mode differentiation of
    the step; forward=True: forward-mode product, which nests inside an outer
    forward-mode derivative (directional derivatives of whole trajectories).
    """
    if forward:
        return fv.jvp_exact(P, y, v)
    _, t = torch.autograd.functional.jvp(lambda z: fv.residual(P, z), y, v, create_graph=True)
    return t


def arnoldi(P: fv.Problem, y: torch.Tensor, f0: torch.Tensor, M: int, tol: float = BREAKDOWN_TOL,
            forward: bool = False):
    """Modified Gram-Schmidt Arnoldi on K_M(J(y), f0); returns (V N x m, H m x m, m).

    The breakdown decision (h_{j+1,j} <= tol ||(h_1j..h_{j+1,j})||) is taken
    on values; it selects m and is not differentiated.
    """
    N = f0.numel()
    M = min(M, N)
    beta = torch.sqrt(torch.dot(f0, f0))
    if M == 0 or float(beta.detach()) == 0.0:
        return f0.new_zeros(N, 0), f0.new_zeros(0, 0), 0
    zero = f0.new_zeros(())
    H = [[zero] * M for _ in range(M + 1)]
    cols = [f0 / beta]
    m = M
    for j in range(M):
        w = jvp_exact(P, y, cols[j], forward)
        for i in range(j + 1):
            hij = torch.dot(cols[i], w)
            H[i][j] = hij
            w = w - hij * cols[i]
        if j + 1 == M:
            break
        hn = torch.sqrt(torch.dot(w, w))
        H[j + 1][j] = hn
        colnorm = sum(float(H[i][j].detach()) ** 2 for i in range(j + 2)) ** 0.5
        if float(hn.detach()) <= tol * colnorm:
            m = j + 1
            break
        cols.append(w / hn)
    V = torch.stack(cols[:m], dim=1)
    Hm = torch.stack([torch.stack(H[i][:m]) for i in range(m)])
    return V, Hm, m


def rok_step(P: fv.Problem, tab: dict, M: int, h: float, y: torch.Tensor, frozen_basis: bool = False,
             forward: bool = False):
    """One ROK step (eq. 9) with exact products, differentiable in y.

    frozen_basis=True detaches V and H from y: the gradient then misses the
    dependence of the Krylov approximation on the state.  It exists only so
    that a test can show the gradient pins detect that omission.
    forward=True: for use under an outer forward-mode derivative.
    """
    s = tab["s"]
    alpha, gam, b, gamma = tab["alpha"], tab["gam"], tab["b"], tab["gamma"]
    F1 = fv.residual(P, y)
    V, H, m = arnoldi(P, y, F1, M, forward=forward)
    if frozen_basis:
        V, H = V.detach(), H.detach()
    if m > 0:
        A = torch.eye(m, dtype=y.dtype) - (h * gamma) * H
    ks, lams = [], []
    for i in range(s):
        if i == 0:
            Fi = F1
        else:
            Y = y
            for j in range(i):
                if alpha[i][j] != 0.0:
                    Y = Y + alpha[i][j] * ks[j]
            Fi = fv.residual(P, Y)
        if m > 0:
            phi = V.T @ Fi
            g = torch.zeros(m, dtype=y.dtype)
            for j in range(i):
                if gam[i][j] != 0.0:
                    g = g + gam[i][j] * lams[j]
            lam = torch.linalg.solve(A, h * phi + h * (H @ g))
            ki = V @ lam + h * (Fi - V @ phi)
        else:
            lam = y.new_zeros(0)
            ki = h * Fi
        ks.append(ki)
        lams.append(lam)
    yn = y
    for i in range(s):
        if b[i] != 0.0:
            yn = yn + b[i] * ks[i]
    return yn


def trajectory(P: fv.Problem, tab: dict, M: int, h: float, y0: torch.Tensor, nsteps: int, forward: bool = False):
    y = y0
    for _ in range(nsteps):
        y = rok_step(P, tab, M, h, y, forward=forward)
    return y


def kinetic_energy(P: fv.Problem, y: torch.Tensor) -> torch.Tensor:
    """Integrated kinetic energy sum_cells |m|^2 / (2 rho) dV (a scalar tensor)."""
    U = y.reshape(P.shape)
    rho = U[0]
    ke = U[1] * U[1]
    for d in range(1, P.ndim):
        ke = ke + U[1 + d] * U[1 + d]
    dV = 1.0
    for d in range(P.ndim):
        dV = dV * P.dx(d)
    return (0.5 * ke / rho).sum() * dV


def directional_derivative(fn, y: torch.Tensor, d: torch.Tensor) -> float:
    """<grad fn(y), d> by forward-mode differentiation (fn built with forward=True)."""
    _, t = torch.func.jvp(fn, (y,), (d,))
    return float(t)


def gradient(fn, y: torch.Tensor) -> torch.Tensor:
    """d fn(y) / d y by reverse-mode differentiation (fn returns a scalar tensor)."""
    z = y.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(fn(z), z)
    return g
