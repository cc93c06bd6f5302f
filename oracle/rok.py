"""One step of the Rosenbrock-Krylov (ROK) method, and trajectories.

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

Sec. 2.2.2, eq. (9): with V, H from modified Arnoldi on K_M(J_n, f(y_n)),

    F_i      = f(y_n + sum_{j<i} alpha_ij k_j)
    phi_i    = V^T F_i
    lambda_i = (I_M - h gamma H)^{-1} (h phi_i + h H sum_{j<i} gamma_ij lambda_j)
    k_i      = V lambda_i + h (F_i - V phi_i)
    y_{n+1}  = y_n + sum_i b_i k_i

For M = 0 the step is the explicit Runge-Kutta method with coefficients
(alpha, b) acting on k_i = h F_i (stated right after eq. 9).

A tableau is a dict with keys s, alpha (s x s, strictly lower), gam (s x s,
strictly lower), gamma and b (length s).
"""
from __future__ import annotations

import math

import torch

from . import fv
from .krylov import arnoldi, dot, lu_factor, lu_solve, matvec_cols

JVP_FD = "fd"
JVP_EXACT = "exact"


def rok_step(f, matvec_at, tab: dict, M: int, h: float, y: torch.Tensor, record: dict | None = None):
    """One ROK step.

    f(y)              right-hand side
    matvec_at(y, fy)  returns a function v -> J(y) v (exact or finite-difference)
    record            optional dict that receives V, H, M_eff, F, phi, lam, k
    """
    s = tab["s"]
    alpha, gam, b, gamma = tab["alpha"], tab["gam"], tab["b"], tab["gamma"]
    F1 = f(y)
    V, H, m = arnoldi(matvec_at(y, F1), F1, M)
    if m > 0:
        hg = h * gamma
        Hl = H.tolist()
        A = torch.tensor([[(1.0 if i == j else 0.0) - hg * Hl[i][j] for j in range(m)] for i in range(m)],
                         dtype=torch.float64)
        LU, perm = lu_factor(A)
    Fs, ks, lams, phis = [], [], [], []
    for i in range(s):
        if i == 0:
            Fi = F1
        else:
            Y = y
            for j in range(i):
                if alpha[i][j] != 0.0:
                    Y = Y + alpha[i][j] * ks[j]
            Fi = f(Y)
        if m > 0:
            phi = torch.tensor([dot(V[:, c], Fi) for c in range(m)], dtype=torch.float64)
            g = torch.zeros(m, dtype=torch.float64)
            for j in range(i):
                if gam[i][j] != 0.0:
                    g = g + gam[i][j] * lams[j]
            Hg = torch.tensor([float(matvec_cols(H[r:r + 1, :], g)[0]) for r in range(m)], dtype=torch.float64)
            rhs = h * phi + h * Hg
            lam = lu_solve(LU, perm, rhs)
            ki = matvec_cols(V, lam) + h * (Fi - matvec_cols(V, phi))
        else:
            phi = lam = torch.zeros(0, dtype=torch.float64)
            ki = h * Fi
        Fs.append(Fi)
        ks.append(ki)
        lams.append(lam)
        phis.append(phi)
    yn = y
    for i in range(s):
        if b[i] != 0.0:
            yn = yn + b[i] * ks[i]
    if record is not None:
        record.update(V=V, H=H, M_eff=m, F=Fs, phi=phis, lam=lams, k=ks)
    return yn


def fv_system(P: fv.Problem, mode: str = JVP_FD, eps: float | None = None):
    """(f, matvec_at) for the finite-volume right-hand side.

    mode 'fd': finite-difference products with eps = sqrt((1 + ||y_n||) eps_mach)
    (fv.fd_epsilon for unit Arnoldi vectors), or the given eps; mode 'exact':
    exact products.
    """
    def f(y):
        return fv.residual(P, y)

    def matvec_at(y, fy):
        if mode == JVP_EXACT:
            return lambda v: fv.jvp_exact(P, y, v)
        e = eps if eps is not None else math.sqrt((1.0 + math.sqrt(dot(y, y))) * fv.EPS_MACH)
        return lambda v: fv.jvp_fd(P, y, fy, v, e)

    return f, matvec_at


def trajectory(f, matvec_at, tab, M, h, y0, nsteps: int, keep: bool = False):
    y = y0
    ys = [y0] if keep else None
    for _ in range(nsteps):
        y = rok_step(f, matvec_at, tab, M, h, y)
        if keep:
            ys.append(y)
    return ys if keep else y
