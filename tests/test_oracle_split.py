"""Pins for the split residual output (inviscid / viscous parts) of the oracle.

* The inviscid part is exactly the residual of the same problem with Euler
  physics (same operations, bit for bit); the viscous part of an Euler
  problem is zero.
* The two parts add up to f (to rounding: one addition per element).
* The viscous part on one-dimensional waves is the discrete Laplacian of
  Stokes' stress / Fourier's law (mu v_xx for a shear wave, kappa T_xx for a
  temperature wave).
"""
import math

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64

CASES = [
    ri.problem((7, 6), (0.0, 0.0), (1.0, 1.3), "ns", "muscl", mu=0.05),
    ri.problem((7, 6), (0.0, 0.0), (1.0, 1.3), "ns", "first", mu=0.05, flux="roe", sutherland=0.4),
    ri.problem((5, 4, 3), (0.0,) * 3, (1.0, 0.9, 1.2), "ns", "muscl", mu=0.05),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_split_parts(k):
    pb = CASES[k]
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=k, amplitude=0.2))
    Fi = fv.residual(P, y, "inviscid")
    Fv = fv.residual(P, y, "viscous")
    assert torch.equal(Fi, fv.residual(oracle_problem(dict(pb, physics="euler", mu=0.0, sutherland=0.0)), y))
    F = fv.residual(P, y)
    assert float(torch.abs(Fi + Fv - F).max()) <= 4 * 2.0 ** -52 * float(torch.abs(Fi).max() + torch.abs(Fv).max())
    Pe = oracle_problem(dict(pb, physics="euler", mu=0.0, sutherland=0.0))
    assert torch.count_nonzero(fv.residual(Pe, y, "viscous")) == 0


def test_viscous_part_on_waves():
    n, mu = 16, 0.07
    pb = ri.problem((n, 4), (0.0, 0.0), (2.0, 1.0), "ns", "muscl", mu=mu)
    P = oracle_problem(pb)
    x = ri._centres(pb, 0)[None, :] * np.ones((4, 1))
    dx = 2.0 / n
    s = np.sin(math.pi * x)
    one = np.ones_like(x)
    lap = lambda a: (np.roll(a, -1, axis=-1) - 2 * a + np.roll(a, 1, axis=-1)) / dx**2
    y = t64(ri._pack(pb, one, [0 * x, 0.3 * s], one))
    got = fv.residual(P, y, "viscous").reshape(4, 4, n)[2].numpy()
    assert np.abs(got - mu * lap(0.3 * s)).max() <= 1e-9 * np.abs(mu * lap(0.3 * s)).max()
    y = t64(ri._pack(pb, one, [0 * x, 0 * x], one + 0.3 * s))
    kappa = mu * 1.4 / (0.4 * 0.72)
    got = fv.residual(P, y, "viscous").reshape(4, 4, n)[3].numpy()
    want = kappa * lap(one + 0.3 * s)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
