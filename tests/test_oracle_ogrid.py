"""Pins for the oracle's O-grid residual: a cylinder with a slip wall and a
far-field boundary (no GPU).

* Gas at rest matching the far field is steady: every face carries only
  p S, and the face vectors of each cell, wall faces included, close.
* Mirror symmetry: with the free stream along x, a state symmetric under
  y -> -y (rho, u, p even, v odd) has a residual with the same symmetry
  (the grid maps cell i to cell nx - 1 - i).
* The brute-force Jacobian on a generic (seeded, symmetry-breaking) state.
"""
import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64


def _P(nx, ny, recon, flux, fs):
    pb, nodes = ri.cylinder_ogrid(nx, ny, recon=recon, flux=flux)
    P = oracle_problem(pb)
    P.nodes, P.farfield = nodes, fs
    return pb, P, nodes


def _state(pb, nodes, seed, fs):
    """The free stream plus a smooth, seeded perturbation in the cell centres."""
    xc, yc = ri.ogrid_centres(*nodes)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, 4)
    bump = np.exp(-((xc - 1.0) ** 2 + yc ** 2) / 2.0)
    rho = fs[0] * (1.0 + 0.1 * a[0] * bump)
    u = fs[1] / fs[0] * (1.0 + 0.2 * a[1] * bump)
    v = 0.2 * a[2] * yc * bump
    p0 = (1.4 - 1.0) * (fs[3] - 0.5 * (fs[1] ** 2 + fs[2] ** 2) / fs[0])
    p = p0 * (1.0 + 0.1 * a[3] * bump)
    return ri._pack(pb, rho, [u, v], p)


@pytest.mark.parametrize("recon", ["first", "muscl"])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_gas_at_rest_is_steady(recon, flux):
    fs = (1.2, 0.0, 0.0, 0.9 / 0.4)
    pb, P, nodes = _P(16, 10, recon, flux, fs)
    y = t64(ri.uniform_state(pb, rho=1.2, vel=[0.0, 0.0], p=0.9))
    F = fv.residual(P, y)
    scale = 0.9 * float(fv.ogrid_metrics(P)[4].max()) * float(torch.sqrt(fv.ogrid_metrics(P)[0] ** 2).max())
    assert float(torch.abs(F).max()) <= 1e-13 * scale


@pytest.mark.parametrize("recon", ["first", "muscl"])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_mirror_symmetry(recon, flux):
    fs = ri.freestream(mach=0.3)
    nx, ny = 16, 10
    pb, P, nodes = _P(nx, ny, recon, flux, fs)
    y = t64(_state(pb, nodes, 3, fs)).reshape(4, ny, nx)
    mirror = lambda U: torch.stack([U[0], U[1], -U[2], U[3]])[:, :, list(range(nx - 1, -1, -1))]
    # the state is symmetric: cell i at y <-> cell nx-1-i at -y
    assert relerr(mirror(y), y) <= 1e-14
    F = fv.residual(P, y.reshape(-1)).reshape(4, ny, nx)
    assert relerr(mirror(F), F) <= 1e-12


@pytest.mark.parametrize("recon", ["first", "muscl"])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_bruteforce_jacobian(recon, flux):
    """On a generic state: the symmetric one sits on ties of the wave-speed maximum
    and of minmod, where f has kinks and differences straddle them."""
    fs = ri.freestream(mach=0.3)
    pb, P, nodes = _P(6, 4, recon, flux, fs)
    y0 = _state(pb, nodes, 5, fs)
    y = t64(y0 + 1e-2 * np.random.default_rng(9).uniform(-1.0, 1.0, y0.size))   # v = 0 on the x axis breaks too
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    assert relerr(fv.jvp_exact(P, y, v), J @ v) <= 1e-7


def _manufactured(xc, yc):
    rho = 1.0 + 0.1 * torch.sin(xc) * torch.cos(yc)
    u = 0.3 + 0.1 * torch.cos(xc)
    v = 0.2 + 0.1 * torch.sin(yc)
    p = 1.0 + 0.1 * torch.cos(xc + yc)
    return rho, u, v, p


def _exact_divergence(xc, yc):
    """-div F of the manufactured fields at the points (x, y), by forward-mode differentiation."""
    def flux(x, y, d):
        rho, u, v, p = _manufactured(x, y)
        E = p / 0.4 + 0.5 * rho * (u * u + v * v)
        un = u if d == 0 else v
        return torch.stack([rho * un, rho * u * un + (p if d == 0 else 0.0), rho * v * un + (p if d == 1 else 0.0),
                            (E + p) * un])
    one = torch.ones_like(xc)
    _, dfx = torch.func.jvp(lambda x: flux(x, yc, 0), (xc,), (one,))
    _, dfy = torch.func.jvp(lambda y: flux(xc, y, 1), (yc,), (one,))
    return -(dfx + dfy)


@pytest.mark.parametrize("recon,order", [("first", 0.8), ("muscl", 1.35)])
def test_interior_consistency_order(recon, order):
    """Away from the boundaries (two rows each side) the residual of a smooth
    manufactured state converges to the exact -div F at the scheme's order
    (measured: first order 0.9-1.0, MUSCL 1.44 then 1.52 on the stretched grid)."""
    errs = []
    for nx, ny in ((32, 16), (64, 32), (128, 64)):
        pb, nodes = ri.cylinder_ogrid(nx, ny, radius=1.0, far=3.0, recon=recon, flux="roe")
        P = oracle_problem(pb)
        P.nodes, P.farfield = nodes, ri.freestream(mach=0.3)
        xc, yc = (torch.from_numpy(a) for a in ri.ogrid_centres(*nodes))
        rho, u, v, p = _manufactured(xc, yc)
        y = t64(ri._pack(pb, rho.numpy(), [u.numpy(), v.numpy()], p.numpy()))
        F = fv.residual(P, y).reshape(4, ny, nx)[:, 2:-2]
        ex = _exact_divergence(xc, yc)[:, 2:-2]
        errs.append(float(torch.sqrt(((F - ex) ** 2).mean()) / torch.sqrt((ex ** 2).mean())))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= order, (errs, rates)


def _Pns(nx, ny, recon, flux, fs, t_wall, suth=0.0):
    pb, nodes = ri.cylinder_ogrid(nx, ny, recon=recon, flux=flux)
    pb = dict(pb, physics="ns", mu=0.02, sutherland=suth, t_ref=0.9)
    P = oracle_problem(pb)
    P.nodes, P.farfield, P.t_wall = nodes, fs, t_wall
    return pb, P, nodes


@pytest.mark.parametrize("recon", ["first", "muscl"])
def test_ns_gas_at_rest_at_the_wall_temperature_is_steady(recon):
    fs = (1.2, 0.0, 0.0, 0.9 / 0.4)
    pb, P, nodes = _Pns(16, 10, recon, "roe", fs, t_wall=0.9 / 1.2, suth=0.4)
    y = t64(ri.uniform_state(pb, rho=1.2, vel=[0.0, 0.0], p=0.9))
    F = fv.residual(P, y)
    scale = 0.9 * float(fv.ogrid_metrics(P)[4].max()) * float(torch.abs(fv.ogrid_metrics(P)[0]).max())
    assert float(torch.abs(F).max()) <= 1e-13 * scale


def test_ns_hot_wall_heats_only_the_first_row():
    """Gas at rest at T0 with a wall at Tw > T0: only the energy of the wall cells
    changes, and it grows (heat flows in through the wall)."""
    fs = (1.2, 0.0, 0.0, 0.9 / 0.4)
    pb, P, nodes = _Pns(16, 10, "muscl", "rusanov", fs, t_wall=1.5)
    y = t64(ri.uniform_state(pb, rho=1.2, vel=[0.0, 0.0], p=0.9))
    F = fv.residual(P, y).reshape(4, 10, 16)
    scale = float(torch.abs(F).max())
    assert (F[3, 0] > 0).all()
    rest = torch.cat([F[:3].reshape(-1), F[3, 1:].reshape(-1)])
    assert float(torch.abs(rest).max()) <= 1e-12 * scale


@pytest.mark.parametrize("recon", ["first", "muscl"])
def test_ns_mirror_symmetry(recon):
    fs = ri.freestream(mach=0.3)
    nx, ny = 16, 10
    pb, P, nodes = _Pns(nx, ny, recon, "roe", fs, t_wall=1.1, suth=0.4)
    y = t64(_state(pb, nodes, 3, fs)).reshape(4, ny, nx)
    mirror = lambda U: torch.stack([U[0], U[1], -U[2], U[3]])[:, :, list(range(nx - 1, -1, -1))]
    F = fv.residual(P, y.reshape(-1)).reshape(4, ny, nx)
    assert relerr(mirror(F), F) <= 1e-12


def test_ns_bruteforce_jacobian():
    fs = ri.freestream(mach=0.3)
    pb, P, nodes = _Pns(6, 4, "muscl", "roe", fs, t_wall=1.1, suth=0.4)
    y0 = _state(pb, nodes, 5, fs)
    y = t64(y0 + 1e-2 * np.random.default_rng(9).uniform(-1.0, 1.0, y0.size))
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    assert relerr(fv.jvp_exact(P, y, v), J @ v) <= 1e-7
