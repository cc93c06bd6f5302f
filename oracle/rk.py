"""Explicit Runge-Kutta methods (Sec. 2.1, eq. 2) and the Lorenz-96 model (Appendix).

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

Used as independent checks of the ROK oracle: with M = 0, ROK reduces to the
explicit method with coefficients (alpha, b) (Sec. 2.2.2), and the Appendix
confirms temporal orders on Lorenz-96 with n = 40 and forcing F = 8.
"""
from __future__ import annotations

import torch

RK4_A = [[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]]
RK4_B = [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]


def erk_step(f, a, b, h, y):
    """k_i = f(y + h sum_j a_ij k_j), y_{n+1} = y + h sum_j b_j k_j (eq. 2, explicit)."""
    s = len(b)
    ks = []
    for i in range(s):
        acc = torch.zeros_like(y)
        for j in range(i):
            if a[i][j] != 0.0:
                acc = acc + a[i][j] * ks[j]
        ks.append(f(y + h * acc))
    acc = torch.zeros_like(y)
    for j in range(s):
        acc = acc + b[j] * ks[j]
    return y + h * acc


def lorenz96(u: torch.Tensor, forcing: float = 8.0) -> torch.Tensor:
    """du_i/dt = (u_{i+1} - u_{i-2}) u_{i-1} - u_i + F, periodic in i (Appendix)."""
    up1 = torch.roll(u, -1)
    um1 = torch.roll(u, 1)
    um2 = torch.roll(u, 2)
    return (up1 - um2) * um1 - u + forcing
