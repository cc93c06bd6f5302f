"""Pins for the oracle's Jacobian eigenvalues (no GPU).

At a uniform state the first-order Rusanov residual on a periodic grid is
translation invariant, so J is block circulant and its spectrum is the union
over the grid's Fourier modes (theta_d = 2 pi k_d / n_d) of the eigenvalues
of the symbol

    S(theta) = sum_d [ -i sin(theta_d) A_d - a_d (1 - cos(theta_d)) I ] / dx_d,

A_d the Jacobian of the physical flux along d and a_d = |u_d| + c the
Rusanov speed (von Neumann analysis of the scheme; the speed's own
derivative multiplies a zero jump).  Each S is a small matrix whose
eigenvalues are taken separately from the dense J's, so a wrong Jacobian,
assembly sign, or spectrum routine fails the comparison.  Also: J at a
general state is real, so its spectrum is closed under conjugation, and the
trace of J equals the sum of the eigenvalues.
"""
import math

import numpy as np
import torch

import rok_inputs as ri
from oracle import eigen, fv
from tests._util import oracle_problem, t64


def _flux(U, d, g=1.4):
    """Physical Euler flux along d of one conserved state (2-D)."""
    r, m, E = U[0], U[1:3], U[3]
    u = m / r
    p = (g - 1.0) * (E - 0.5 * r * (u * u).sum())
    F = torch.stack([m[d], m[0] * u[d] + (p if d == 0 else 0.0), m[1] * u[d] + (p if d == 1 else 0.0),
                     (E + p) * u[d]])
    return F


def test_uniform_state_spectrum_is_the_fourier_symbol():
    n = (6, 5)
    pb = ri.problem(n, (0.0, 0.0), (1.2, 0.7), "euler", "first")
    P = oracle_problem(pb)
    rho, vel, p = 1.3, [0.4, -0.25], 0.9
    y = t64(ri.uniform_state(pb, rho=rho, vel=vel, p=p))
    U0 = torch.tensor([rho, rho * vel[0], rho * vel[1], p / 0.4 + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2)],
                      dtype=torch.float64)
    A = [torch.func.jacfwd(lambda U: _flux(U, d))(U0).numpy() for d in range(2)]
    c = math.sqrt(1.4 * p / rho)
    a = [abs(vel[d]) + c for d in range(2)]
    dx = [1.2 / n[0], 0.7 / n[1]]
    want = []
    for kx in range(n[0]):
        for ky in range(n[1]):
            th = [2 * math.pi * kx / n[0], 2 * math.pi * ky / n[1]]
            S = sum((-1j * math.sin(th[d]) * A[d] - a[d] * (1 - math.cos(th[d])) * np.eye(4)) / dx[d]
                    for d in range(2))
            want.extend(np.linalg.eigvals(S))
    got = eigen.eigenvalues(P, y)
    want = np.array(want)
    scale = np.abs(want).max()
    # match as multisets: every computed eigenvalue has a symbol eigenvalue nearby and vice versa
    dist = np.abs(got[:, None] - want[None, :])
    assert dist.min(axis=1).max() <= 1e-9 * scale
    assert dist.min(axis=0).max() <= 1e-9 * scale
    assert len(got) == len(want)


def test_conjugate_closed_and_trace():
    pb = ri.problem((5, 4), (0.0, 0.0), (1.0, 1.1), "ns", "muscl", mu=0.05)
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=3, amplitude=0.2))
    ev = eigen.eigenvalues(P, y)
    J = eigen.dense_jacobian(P, y).numpy()
    assert abs(ev.sum().real - np.trace(J)) <= 1e-9 * np.abs(ev).sum()
    assert abs(ev.sum().imag) <= 1e-9 * np.abs(ev).sum()
    d = np.abs(ev[:, None] - np.conj(ev)[None, :]).min(axis=1)
    assert d.max() <= 1e-8 * np.abs(ev).max()
    top = eigen.largest(P, y, 4)
    assert np.all(np.abs(top) >= np.abs(ev[4]) - 1e-12)
