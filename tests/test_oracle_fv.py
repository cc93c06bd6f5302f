"""Pins for the oracle's residual f and its Jacobian products (no GPU).

Each check is fixed by the mathematics, not by re-typing the oracle's formulas:
free-stream preservation, discrete conservation, 90-degree rotation symmetry,
the isentropic vortex (an exact travelling solution: f -> -(u_inf . grad) y at
the scheme's spatial order), viscous decay of the Taylor-Green vortex, the
brute-force Jacobian by central differences, the Taylor test and the
adjoint dot-product test.
"""
import math

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64

VARIANTS = [
    ("euler_fo", lambda n: ri.problem((n, n + 1), (-1.0, -1.5), (1.0, 1.0), "euler", "first")),
    ("euler_muscl", lambda n: ri.problem((n, n + 1), (-1.0, -1.5), (1.0, 1.0), "euler", "muscl")),
    ("ns_muscl", lambda n: ri.problem((n, n + 1), (0.0, 0.0), (1.0, 1.3), "ns", "muscl", mu=0.05)),
    ("ns3d_muscl", lambda n: ri.problem((n, n - 1, n + 1), (0.0, 0.0, 0.0), (1.0, 0.9, 1.2), "ns", "muscl", mu=0.05)),
]


@pytest.mark.parametrize("name,mk", VARIANTS)
def test_free_stream_is_exactly_steady(name, mk):
    pb = mk(6)
    P = oracle_problem(pb)
    y = t64(ri.uniform_state(pb, rho=1.3, vel=[0.4, -0.7, 0.2][:len(pb["n"])], p=0.9))
    F = fv.residual(P, y)
    assert torch.count_nonzero(F) == 0


@pytest.mark.parametrize("name,mk", VARIANTS)
def test_discrete_conservation(name, mk):
    pb = mk(7)
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=3))
    F = fv.residual(P, y).reshape(P.nvar, -1)
    scale = float(torch.abs(F).sum(dim=1).max())
    sums = F.sum(dim=1)
    assert float(torch.abs(sums).max()) <= 1e-13 * scale


def _rot90(pb, y):
    """Rotate a 2-D state by +90 degrees on a square periodic grid: new(x, y) = R old(R^-1 (x, y))."""
    n = pb["n"][0]
    U = y.reshape(4, n, n).numpy()              # [var][j][i]
    # cell (i, j) of the new field takes cell (j, n-1-i) of the old one
    R = np.empty_like(U)
    for v in range(4):
        R[v] = np.rot90(U[v], k=1, axes=(1, 0))  # rotate the array image
    ru, rv = R[1].copy(), R[2].copy()
    R[1], R[2] = -rv, ru
    return t64(R.reshape(-1))


@pytest.mark.parametrize("recon,phys", [("first", "euler"), ("muscl", "euler"), ("muscl", "ns")])
def test_rotation_symmetry(recon, phys):
    n = 8
    pb = ri.problem((n, n), (0.0, 0.0), (1.0, 1.0), phys, recon, mu=0.05 if phys == "ns" else 0.0)
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=11))
    lhs = fv.residual(P, _rot90(pb, y))
    rhs = _rot90(pb, fv.residual(P, y))
    assert relerr(lhs, rhs) <= 1e-14


def _vortex_error(n, recon):
    pb = ri.vortex_problem(n, recon)
    P = oracle_problem(pb)
    y0 = ri.vortex_state(pb)
    d = 1e-4
    dydt = (ri.vortex_state(pb, t=d) - ri.vortex_state(pb, t=-d)) / (2 * d)
    F = fv.residual(P, t64(y0)).numpy()
    return np.linalg.norm(F - dydt) / np.linalg.norm(dydt)


@pytest.mark.parametrize("recon,order", [("first", 0.8), ("muscl", 1.5)])
def test_vortex_travelling_solution_spatial_order(recon, order):
    errs = [_vortex_error(n, recon) for n in (32, 64, 128)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < errs[0]
    assert min(rates) >= order, (errs, rates)


def _viscous_part(pb, y):
    """NS residual minus the Euler residual of the same discretisation."""
    P = oracle_problem(pb)
    Pe = oracle_problem(dict(pb, physics="euler", mu=0.0))
    return fv.residual(P, y) - fv.residual(Pe, y)


def test_taylor_green_viscous_decay():
    """2-D TGV: the viscous terms drain kinetic energy at rate 4 nu (exp(-4 nu t) decay)."""
    pb = ri.tgv_problem(64, 2)
    y = t64(ri.tgv_state(pb))
    F = _viscous_part(pb, y).reshape(4, -1)
    U = y.reshape(4, -1)
    rho, m = U[0], U[1:3]
    ke = float((0.5 * (m * m).sum(0) / rho).sum())
    u = m / rho
    dke = float(((u * F[1:3]).sum(0) - 0.5 * (u * u).sum(0) * F[0]).sum())
    assert abs(-dke / ke / (4 * pb["mu"]) - 1.0) < 0.01


def test_taylor_green_3d_initial_dissipation():
    """3-D TGV: the viscous terms drain kinetic energy at the rate of the
    incompressible flow, -dE_k/dt = nu <|grad u|^2> = (3/4) nu with E_k = 1/8
    per unit volume at t = 0.  Measured ratios 0.9914, 0.9962, 0.9979 on 16^3,
    24^3, 32^3: the central viscous differences converge at second order."""
    pb = ri.tgv_problem(24, 3, reynolds=100.0)
    y = t64(ri.tgv_state(pb))
    F = _viscous_part(pb, y).reshape(5, -1)
    U = y.reshape(5, -1)
    rho, m = U[0], U[1:4]
    vol = (2 * np.pi) ** 3
    dV = vol / U.shape[1]
    ke = float((0.5 * (m * m).sum(0) / rho).sum()) * dV / vol
    u = m / rho
    dke = float(((u * F[1:4]).sum(0) - 0.5 * (u * u).sum(0) * F[0]).sum()) * dV / vol
    assert abs(ke - 0.125) < 1e-12
    assert abs(-dke / (0.75 * pb["mu"]) - 1.0) < 0.01, -dke / (0.75 * pb["mu"])


def _lap(a, dx):
    return (np.roll(a, -1, axis=-1) - 2 * a + np.roll(a, 1, axis=-1)) / dx**2


@pytest.mark.parametrize("case", ["shear", "longitudinal", "heat"])
def test_viscous_terms_on_one_dimensional_waves(case):
    """Stokes stress and Fourier heat flux (eq. 11) reduce to discrete Laplacians:
    shear wave: mu v_xx; longitudinal wave: (4/3) mu u_xx; conduction: kappa T_xx."""
    n, mu = 16, 0.07
    pb = ri.problem((n, 4), (0.0, 0.0), (2.0, 1.0), "ns", "muscl", mu=mu)
    x = ri._centres(pb, 0)[None, :] * np.ones((4, 1))
    dx = 2.0 / n
    s = np.sin(math.pi * x)
    one = np.ones_like(x)
    if case == "shear":
        y = ri._pack(pb, one, [0 * x, 0.3 * s], one)
        want, var = mu * _lap(0.3 * s, dx), 2
    elif case == "longitudinal":
        y = ri._pack(pb, one, [0.3 * s, 0 * x], one)
        want, var = 4.0 / 3.0 * mu * _lap(0.3 * s, dx), 1
    else:
        y = ri._pack(pb, one, [0 * x, 0 * x], one + 0.3 * s)
        kappa = mu * 1.4 / (0.4 * 0.72)
        want, var = kappa * _lap(one + 0.3 * s, dx), 3
    got = _viscous_part(pb, t64(y)).reshape(4, 4, n)[var].numpy()
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


TINY = [
    ("euler_fo", ri.problem((6, 5), (-1.0, -1.0), (1.0, 1.2), "euler", "first")),
    ("euler_muscl", ri.problem((6, 5), (-1.0, -1.0), (1.0, 1.2), "euler", "muscl")),
    ("ns_muscl", ri.problem((6, 5), (0.0, 0.0), (1.0, 1.2), "ns", "muscl", mu=0.05)),
    ("ns3d_muscl", ri.problem((5, 4, 3), (0.0, 0.0, 0.0), (1.0, 0.8, 0.6), "ns", "muscl", mu=0.05)),
]


def _margin_state(pb, seed):
    """Random smooth state; MUSCL kinks (a*b = 0, |a| = |b|) are far away at this size."""
    return t64(ri.smooth_random_state(pb, seed=seed, amplitude=0.2))


@pytest.mark.parametrize("name,pb", TINY)
def test_exact_jvp_matches_bruteforce_jacobian(name, pb):
    P = oracle_problem(pb)
    y = _margin_state(pb, 5)
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    assert relerr(fv.jvp_exact(P, y, v), J @ v) <= 1e-7


@pytest.mark.parametrize("name,pb", TINY)
def test_taylor_remainder_is_second_order(name, pb):
    P = oracle_problem(pb)
    y = _margin_state(pb, 9)
    v = t64(ri.random_direction(P.size, seed=4))
    F0 = fv.residual(P, y)
    Jv = fv.jvp_exact(P, y, v)
    rs = []
    for k in range(4):
        d = 1e-3 / 2**k
        rs.append(float(torch.linalg.norm(fv.residual(P, y + d * v) - F0 - d * Jv)))
    rates = [math.log2(rs[i] / rs[i + 1]) for i in range(3)]
    assert min(rates) > 1.8, rates


@pytest.mark.parametrize("name,pb", TINY)
def test_adjoint_dot_product(name, pb):
    P = oracle_problem(pb)
    y = _margin_state(pb, 12)
    v = t64(ri.random_direction(P.size, seed=1))
    wb = t64(ri.random_direction(P.size, seed=2))
    lhs = float(torch.dot(wb, fv.jvp_exact(P, y, v)))
    rhs = float(torch.dot(fv.vjp(P, y, wb), v))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("name,pb", TINY[:2] + TINY[2:3])
def test_second_order_adjoint_matches_difference_of_adjoints(name, pb):
    P = oracle_problem(pb)
    y = _margin_state(pb, 21)
    v = t64(ri.random_direction(P.size, seed=3))
    wb = t64(ri.random_direction(P.size, seed=6))
    so = fv.vjp_second(P, y, v, wb)
    d = 1e-5
    fd = (fv.vjp(P, y + d * v, wb) - fv.vjp(P, y - d * v, wb)) / (2 * d)
    assert relerr(so, fd) <= 1e-7


def test_fd_jvp_converges_to_exact():
    pb = TINY[1][1]
    P = oracle_problem(pb)
    y = _margin_state(pb, 8)
    v = t64(ri.random_direction(P.size, seed=9))
    F0 = fv.residual(P, y)
    ex = fv.jvp_exact(P, y, v)
    errs = [relerr(fv.jvp_fd(P, y, F0, v, e), ex) for e in (1e-3, 1e-4, 1e-5)]
    assert errs[0] > errs[1] > errs[2]
    assert 5 < errs[0] / errs[1] < 20
    e_def = fv.fd_epsilon(y, v)
    assert relerr(fv.jvp_fd(P, y, F0, v, e_def), ex) < 1e-6
