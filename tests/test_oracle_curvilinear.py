"""Pins for the oracle's residual on 2-D curvilinear periodic grids (no GPU).

* Metric identities: every cell's outward face vectors sum to zero (the
  geometric conservation law) and the cell areas add up to the box's area.
* On the Cartesian nodes the curvilinear residual is the Cartesian one (to
  rounding), for both fluxes and reconstructions.
* On a warped grid: a uniform flow is steady (free-stream preservation),
  area-weighted residuals sum to zero (conservation), and the travelling
  vortex's exact time derivative is approached at the scheme's order as the
  grid is refined.
"""
import math

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64


def _P(pb, nodes):
    P = oracle_problem(pb)
    P.nodes = nodes
    return P


def test_metric_identities():
    pb = ri.problem((12, 9), (-1.0, 0.0), (2.0, 1.5), "euler", "first")
    P = _P(pb, ri.warped_nodes(pb, 0.06))
    sxe, sye, sxn, syn, inva = (a.numpy() for a in fv.metrics(P)[:5])
    gx = sxe - np.roll(sxe, 1, axis=1) + sxn - np.roll(sxn, 1, axis=0)
    gy = sye - np.roll(sye, 1, axis=1) + syn - np.roll(syn, 1, axis=0)
    assert np.abs(gx).max() <= 1e-14 and np.abs(gy).max() <= 1e-14
    assert abs((1.0 / inva).sum() - 3.0 * 1.5) <= 1e-12
    assert (inva > 0).all()


@pytest.mark.parametrize("recon", ["first", "muscl"])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_cartesian_nodes_reduce_to_the_cartesian_residual(recon, flux):
    pb = ri.problem((10, 7), (-1.0, 0.0), (2.0, 1.4), "euler", recon, flux=flux)
    y = t64(ri.smooth_random_state(pb, seed=2, amplitude=0.2))
    assert relerr(fv.residual(_P(pb, ri.cartesian_nodes(pb)), y), fv.residual(oracle_problem(pb), y)) <= 1e-13


@pytest.mark.parametrize("recon", ["first", "muscl"])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_free_stream_and_conservation_on_a_warped_grid(recon, flux):
    pb = ri.problem((12, 10), (-1.0, 0.0), (2.0, 1.4), "euler", recon, flux=flux)
    P = _P(pb, ri.warped_nodes(pb, 0.06))
    y = t64(ri.uniform_state(pb, rho=1.3, vel=[0.4, -0.7], p=0.9))
    F = fv.residual(P, y)
    scale = float(torch.abs(fv.residual(oracle_problem(pb), t64(ri.smooth_random_state(pb, seed=1)))).max())
    assert float(torch.abs(F).max()) <= 1e-12 * max(scale, 1.0)
    y = t64(ri.smooth_random_state(pb, seed=3, amplitude=0.2))
    F = fv.residual(P, y).reshape(4, -1)
    area = (1.0 / fv.metrics(P)[4]).reshape(-1)
    sums = (F * area).sum(dim=1)
    assert float(torch.abs(sums).max()) <= 1e-13 * float((torch.abs(F) * area).sum(dim=1).max())


@pytest.mark.parametrize("recon,order", [("first", 0.8), ("muscl", 1.5)])
def test_vortex_on_a_warped_grid_converges(recon, order):
    errs = []
    for n in (32, 64, 128):
        pb = ri.vortex_problem(n, recon)
        nodes = ri.warped_nodes(pb, 0.06)
        c = ri.node_centres(pb, *nodes)
        d = 1e-4
        dydt = (ri.vortex_state(pb, t=d, centres=c) - ri.vortex_state(pb, t=-d, centres=c)) / (2 * d)
        F = fv.residual(_P(pb, nodes), t64(ri.vortex_state(pb, centres=c))).numpy()
        errs.append(np.linalg.norm(F - dydt) / np.linalg.norm(dydt))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= order, (errs, rates)


def test_warped_jacobian_bruteforce():
    pb = ri.problem((5, 4), (0.0, 0.0), (1.0, 0.8), "euler", "muscl", flux="roe")
    P = _P(pb, ri.warped_nodes(pb, 0.06))
    y = t64(ri.smooth_random_state(pb, seed=5, amplitude=0.2))
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    assert relerr(fv.jvp_exact(P, y, v), J @ v) <= 1e-7


@pytest.mark.parametrize("recon", ["first", "muscl"])
@pytest.mark.parametrize("suth", [0.0, 0.4])
def test_ns_cartesian_nodes_reduce_to_the_cartesian_residual(recon, suth):
    """Viscous terms through the chain rule reduce to the Cartesian face
    gradients on Cartesian nodes (to rounding)."""
    pb = ri.problem((10, 7), (-1.0, 0.0), (2.0, 1.4), "ns", recon, mu=0.05, sutherland=suth, t_ref=0.8)
    y = t64(ri.smooth_random_state(pb, seed=2, amplitude=0.2))
    assert relerr(fv.residual(_P(pb, ri.cartesian_nodes(pb)), y), fv.residual(oracle_problem(pb), y)) <= 1e-13


def test_ns_conservation_on_a_warped_grid():
    pb = ri.problem((12, 10), (-1.0, 0.0), (2.0, 1.4), "ns", "muscl", mu=0.05, flux="roe", sutherland=0.4)
    P = _P(pb, ri.warped_nodes(pb, 0.06))
    y = t64(ri.uniform_state(pb, rho=1.3, vel=[0.4, -0.7], p=0.9))
    scale = float(torch.abs(fv.residual(oracle_problem(pb), t64(ri.smooth_random_state(pb, seed=1)))).max())
    assert float(torch.abs(fv.residual(P, y)).max()) <= 1e-12 * max(scale, 1.0)
    y = t64(ri.smooth_random_state(pb, seed=3, amplitude=0.2))
    F = fv.residual(P, y).reshape(4, -1)
    area = (1.0 / fv.metrics(P)[4]).reshape(-1)
    assert float(torch.abs((F * area).sum(dim=1)).max()) <= 1e-13 * float((torch.abs(F) * area).sum(dim=1).max())


def test_ns_shear_wave_on_a_warped_grid_converges():
    """Viscous part of the y-momentum residual for v = 0.3 sin(2 pi x / Lx) (rho,
    p uniform) on warped grids: converges to mu v_xx at first order or better."""
    errs = []
    for n in (16, 32, 64):
        pb = ri.problem((n, n), (0.0, 0.0), (2.0, 2.0), "ns", "muscl", mu=0.07)
        nodes = ri.warped_nodes(pb, 0.05)
        xc, yc = ri.node_centres(pb, *nodes)
        one = np.ones_like(xc)
        v = 0.3 * np.sin(math.pi * xc)
        y = t64(ri._pack(pb, one, [0 * xc, v], one))
        Pn, Pe = _P(pb, nodes), _P(dict(pb, physics="euler", mu=0.0), nodes)
        visc = (fv.residual(Pn, y) - fv.residual(Pe, y)).reshape(4, n, n)[2].numpy()
        want = -0.07 * math.pi ** 2 * v
        errs.append(np.sqrt(((visc - want) ** 2).mean()) / np.sqrt((want ** 2).mean()))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.05 and min(rates) >= 0.9, (errs, rates)


def test_ns_warped_jacobian_bruteforce():
    pb = ri.problem((5, 4), (0.0, 0.0), (1.0, 0.8), "ns", "muscl", mu=0.05, flux="roe", sutherland=0.4)
    P = _P(pb, ri.warped_nodes(pb, 0.06))
    y = t64(ri.smooth_random_state(pb, seed=5, amplitude=0.2))
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    assert relerr(fv.jvp_exact(P, y, v), J @ v) <= 1e-7
