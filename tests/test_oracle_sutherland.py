"""Pins for Sutherland's viscosity law in the oracle's viscous terms (no GPU).

* The law itself against tabulated air viscosities (White, Viscous Fluid
  Flow: 1.846e-5 Pa s at 300 K, 2.286e-5 at 400 K, with the usual constants
  mu_ref = 1.716e-5 Pa s at 273.15 K and S = 110.4 K).
* At a uniform temperature the viscous terms are those of a constant viscosity
  mu(T0) (a shear wave at T0 = T_ref and at 2 T_ref).
* Heat conduction with a temperature wave is the conservative discrete
  operator d/dx (kappa(T_face) dT/dx), kappa at the mean of the two cell
  temperatures (the reading of where mu is evaluated).
* Conservation and the brute-force Jacobian with a temperature-dependent mu.
"""
import math

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64


def test_tabulated_air_viscosity():
    P = fv.Problem(n=(4, 4), lo=(0.0, 0.0), hi=(1.0, 1.0), physics="ns", mu=1.716e-5,
                   sutherland=110.4 / 273.15, t_ref=273.15)
    for T, mu in ((300.0, 1.846e-5), (400.0, 2.286e-5), (273.15, 1.716e-5)):
        got = float(fv.sutherland_mu(P, torch.tensor([T], dtype=torch.float64))[0])
        assert abs(got - mu) <= 1e-3 * mu, (T, got, mu)


def _viscous(pb, y):
    P = oracle_problem(pb)
    Pe = oracle_problem(dict(pb, physics="euler", mu=0.0, sutherland=0.0))
    return fv.residual(P, y) - fv.residual(Pe, y)


@pytest.mark.parametrize("theta", [1.0, 2.0])
def test_uniform_temperature_is_constant_viscosity(theta):
    n, mu, s, tref = 16, 0.07, 0.4, 1.3
    pb = ri.problem((n, 4), (0.0, 0.0), (2.0, 1.0), "ns", "muscl", mu=mu, sutherland=s, t_ref=tref)
    x = ri._centres(pb, 0)[None, :] * np.ones((4, 1))
    one = np.ones_like(x)
    rho = 1.0 + 0.2 * np.cos(math.pi * x)
    y = t64(ri._pack(pb, rho, [0.1 * np.sin(math.pi * x), 0.3 * np.sin(math.pi * x)], rho * theta * tref))
    mu_t = mu * theta * math.sqrt(theta) * (1.0 + s) / (theta + s)
    want = _viscous(dict(pb, mu=mu_t, sutherland=0.0), y)
    assert relerr(_viscous(pb, y), want) <= 1e-13


def test_heat_conduction_variable_kappa():
    n, mu, s = 32, 0.05, 0.5
    pb = ri.problem((n, 4), (0.0, 0.0), (2.0, 1.0), "ns", "muscl", mu=mu, sutherland=s, t_ref=1.0)
    x = ri._centres(pb, 0)[None, :] * np.ones((4, 1))
    one = np.ones_like(x)
    T = 1.0 + 0.5 * np.sin(math.pi * x)
    y = t64(ri._pack(pb, one, [0 * x, 0 * x], T))        # rho = 1: p = T
    dx = 2.0 / n
    Tf = 0.5 * (T + np.roll(T, -1, axis=-1))
    muf = mu * Tf ** 1.5 * (1.0 + s) / (Tf + s)
    kf = muf * 1.4 / (0.4 * 0.72)
    q = kf * (np.roll(T, -1, axis=-1) - T) / dx
    want = (q - np.roll(q, 1, axis=-1)) / dx
    got = _viscous(pb, y).reshape(4, 4, n)[3].numpy()
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


TINY = [
    ("ns_muscl", ri.problem((5, 4), (0.0, 0.0), (1.0, 1.1), "ns", "muscl", mu=0.05, sutherland=0.4)),
    ("ns3d_fo", ri.problem((4, 3, 4), (0.0,) * 3, (1.0, 0.9, 1.1), "ns", "first", mu=0.05, sutherland=0.4,
                           t_ref=0.8)),
]


@pytest.mark.parametrize("name,pb", TINY)
def test_conservation_and_bruteforce_jacobian(name, pb):
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=5, amplitude=0.2))
    F = fv.residual(P, y).reshape(P.nvar, -1)
    assert float(torch.abs(F.sum(dim=1)).max()) <= 1e-13 * float(torch.abs(F).sum(dim=1).max())
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    assert relerr(fv.jvp_exact(P, y, v), J @ v) <= 1e-7
