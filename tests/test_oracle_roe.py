"""Pins for the oracle's Roe flux (no GPU).

Fixed by the mathematics of Roe's linearisation, not by re-typing it:
* consistency: Fhat(U, U) = F(U) exactly;
* Roe's property F(U_R) - F(U_L) = A(U_L, U_R)(U_R - U_L): when every wave
  speed of the averaged state is positive (beyond the entropy-fix band) the
  flux is the left physical flux F(U_L), and the right one when all are
  negative.  A wrong eigenvector, strength, average or sign breaks this;
* a stationary contact (u = 0, equal pressure) carries no mass flux;
* Harten's fix is continuous at its threshold and gives delta / 2 at a sonic
  point;
* at the residual level: free-stream preservation, discrete conservation,
  90-degree rotation symmetry, the travelling vortex at the scheme's order,
  the brute-force Jacobian and the Taylor remainder.
"""
import math

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64


def _P(D=2, flux="roe"):
    n = (4,) * D
    return fv.Problem(n=n, lo=(0.0,) * D, hi=(1.0,) * D, flux=flux)


def _states(P, r, vel, p):
    r = torch.as_tensor(np.asarray(r, dtype=np.float64))
    vel = [torch.as_tensor(np.asarray(v, dtype=np.float64)) for v in vel]
    p = torch.as_tensor(np.asarray(p, dtype=np.float64))
    return fv.conserved(P, r, vel, p), r, vel, p


def _flux(P, L, R, d):
    (UL, rL, vL, pL), (UR, rR, vR, pR) = L, R
    return torch.stack(fv.face_flux(P, UL, rL, vL, pL, UR, rR, vR, pR, d))


def _phys(P, S, d):
    U, r, vel, p = S
    return torch.stack(fv._euler_flux(P, U, vel, p, d))


def _random_side(P, rng, n, un_range, d):
    D = P.ndim
    r = rng.uniform(0.5, 2.0, n)
    p = rng.uniform(0.5, 2.0, n)
    vel = [rng.uniform(-0.5, 0.5, n) for _ in range(D)]
    vel[d] = rng.uniform(*un_range, n)
    return _states(P, r, vel, p)


@pytest.mark.parametrize("D", [2, 3])
def test_consistency(D):
    P = _P(D)
    rng = np.random.default_rng(1)
    for d in range(D):
        S = _random_side(P, rng, 64, (-2.0, 2.0), d)
        assert torch.equal(_flux(P, S, S, d), _phys(P, S, d))


@pytest.mark.parametrize("D", [2, 3])
def test_supersonic_upwinding_roe_property(D):
    """u_n >= 4 with c <= sqrt(1.4 * 2 / 0.5) = 2.37: every averaged wave speed
    exceeds the fix band, so Fhat = F(U_L) (u_n > 0) or F(U_R) (u_n < 0)."""
    P = _P(D)
    rng = np.random.default_rng(2)
    for d in range(D):
        L = _random_side(P, rng, 200, (4.0, 6.0), d)
        R = _random_side(P, rng, 200, (4.0, 6.0), d)
        F = _flux(P, L, R, d)
        FL = _phys(P, L, d)
        assert float(torch.abs(F - FL).max()) <= 1e-12 * float(torch.abs(FL).max())
        L = _random_side(P, rng, 200, (-6.0, -4.0), d)
        R = _random_side(P, rng, 200, (-6.0, -4.0), d)
        F = _flux(P, L, R, d)
        FR = _phys(P, R, d)
        assert float(torch.abs(F - FR).max()) <= 1e-12 * float(torch.abs(FR).max())
    # Rusanov is not upwind there: the same check must fail for it
    Pr = _P(D, "rusanov")
    L = _random_side(Pr, rng, 50, (4.0, 6.0), 0)
    R = _random_side(Pr, rng, 50, (4.0, 6.0), 0)
    assert float(torch.abs(_flux(Pr, L, R, 0) - _phys(Pr, L, 0)).max()) > 1e-3


def test_stationary_contact():
    P = _P(2)
    zero = np.zeros(16)
    L = _states(P, np.linspace(0.5, 1.0, 16), [zero, np.linspace(-0.3, 0.3, 16)], np.full(16, 0.9))
    R = _states(P, np.linspace(1.5, 3.0, 16), [zero, np.linspace(0.2, 0.4, 16)], np.full(16, 0.9))
    F = _flux(P, L, R, 0)
    assert torch.count_nonzero(F[0]) == 0          # no mass through the contact
    assert torch.equal(F[1], torch.full((16,), 0.9, dtype=torch.float64))


def test_entropy_fix_continuity_and_sonic_value():
    """A pure left-moving acoustic jump whose averaged wave speed u - c passes
    through the band |u - c| < c/8: the flux is continuous in the state, and
    with u - c = 0 the acoustic wave is damped by delta/2 = c/16."""
    P = _P(2)
    c = math.sqrt(1.4)                    # rho = p = 1
    fl = []
    for k, un in enumerate(np.linspace(c - c / 8 - 1e-3, c - c / 8 + 1e-3, 5)):
        L = _states(P, [1.0], [[un], [0.0]], [1.0])
        R = _states(P, [1.0 + 1e-9], [[un], [0.0]], [1.0 + 1.4e-9])
        fl.append(float(_flux(P, L, R, 0)[0]))
    jumps = np.abs(np.diff(fl))
    assert jumps.max() < 1e-3 * abs(fl[0])
    # sonic point: only the 1-wave is excited and |lambda_1| -> delta / 2
    L = _states(P, [1.0], [[c], [0.0]], [1.0])
    eps = 1e-7
    R = _states(P, [1.0 + eps], [[c - eps * c], [0.0]], [1.0 + 1.4 * eps])   # dp = c^2 drho, du = -c drho
    F = _flux(P, L, R, 0)
    central = 0.5 * (_phys(P, L, 0) + _phys(P, R, 0))
    diss = 2.0 * (central - F)                  # = |lambda_1| alpha_1 r_1 (+ O(eps^2))
    alpha1 = (1.4 * eps + c * c * eps) / (2 * 1.4)
    assert abs(float(diss[0]) / alpha1 - (c / 8) / 2) < 1e-6


ROE_VARIANTS = [
    ("euler_fo", lambda n: ri.problem((n, n + 1), (-1.0, -1.5), (1.0, 1.0), "euler", "first", flux="roe")),
    ("euler_muscl", lambda n: ri.problem((n, n + 1), (-1.0, -1.5), (1.0, 1.0), "euler", "muscl", flux="roe")),
    ("ns_muscl", lambda n: ri.problem((n, n + 1), (0.0, 0.0), (1.0, 1.3), "ns", "muscl", mu=0.05, flux="roe")),
    ("euler3d_muscl", lambda n: ri.problem((n, n - 1, n + 1), (0.0,) * 3, (1.0, 0.9, 1.2), "euler", "muscl",
                                           flux="roe")),
]


@pytest.mark.parametrize("name,mk", ROE_VARIANTS)
def test_free_stream_and_conservation(name, mk):
    pb = mk(6)
    P = oracle_problem(pb)
    y = t64(ri.uniform_state(pb, rho=1.3, vel=[0.4, -0.7, 0.2][:len(pb["n"])], p=0.9))
    assert torch.count_nonzero(fv.residual(P, y)) == 0
    y = t64(ri.smooth_random_state(pb, seed=3))
    F = fv.residual(P, y).reshape(P.nvar, -1)
    assert float(torch.abs(F.sum(dim=1)).max()) <= 1e-13 * float(torch.abs(F).sum(dim=1).max())


@pytest.mark.parametrize("recon", ["first", "muscl"])
def test_rotation_symmetry(recon):
    from tests.test_oracle_fv import _rot90
    n = 8
    pb = ri.problem((n, n), (0.0, 0.0), (1.0, 1.0), "euler", recon, flux="roe")
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=11))
    assert relerr(fv.residual(P, _rot90(pb, y)), _rot90(pb, fv.residual(P, y))) <= 1e-14


@pytest.mark.parametrize("recon,order", [("first", 0.8), ("muscl", 1.5)])
def test_vortex_travelling_solution_spatial_order(recon, order):
    errs = []
    for n in (32, 64, 128):
        pb = dict(ri.vortex_problem(n, recon), flux="roe")
        P = oracle_problem(pb)
        d = 1e-4
        dydt = (ri.vortex_state(pb, t=d) - ri.vortex_state(pb, t=-d)) / (2 * d)
        F = fv.residual(P, t64(ri.vortex_state(pb))).numpy()
        errs.append(np.linalg.norm(F - dydt) / np.linalg.norm(dydt))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= order, (errs, rates)


def test_roe_less_dissipative_than_rusanov_on_the_vortex():
    """Upwinding each wave by its own speed: the first-order Roe residual of the
    travelling vortex is closer to the exact time derivative than Rusanov's."""
    errs = {}
    for flux in ("rusanov", "roe"):
        pb = dict(ri.vortex_problem(64, "first"), flux=flux)
        P = oracle_problem(pb)
        d = 1e-4
        dydt = (ri.vortex_state(pb, t=d) - ri.vortex_state(pb, t=-d)) / (2 * d)
        F = fv.residual(P, t64(ri.vortex_state(pb))).numpy()
        errs[flux] = np.linalg.norm(F - dydt) / np.linalg.norm(dydt)
    assert errs["roe"] < 0.8 * errs["rusanov"], errs


TINY = [
    ("euler_fo", ri.problem((4, 3), (0.0, 0.0), (1.0, 0.8), "euler", "first", flux="roe")),
    ("ns_muscl", ri.problem((5, 4), (0.0, 0.0), (1.0, 1.1), "ns", "muscl", mu=0.05, flux="roe")),
    ("euler3d_muscl", ri.problem((4, 3, 4), (0.0,) * 3, (1.0, 0.9, 1.1), "euler", "muscl", flux="roe")),
]


@pytest.mark.parametrize("name,pb", TINY)
def test_exact_jvp_bruteforce_and_taylor(name, pb):
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=5, amplitude=0.2))
    J = fv.dense_jacobian_fd(P, y, delta=1e-6)
    v = t64(ri.random_direction(P.size, seed=7))
    Jv = fv.jvp_exact(P, y, v)
    assert relerr(Jv, J @ v) <= 1e-7
    F0 = fv.residual(P, y)
    rs = [float(torch.linalg.norm(fv.residual(P, y + (1e-3 / 2**k) * v) - F0 - (1e-3 / 2**k) * Jv))
          for k in range(4)]
    assert min(math.log2(rs[i] / rs[i + 1]) for i in range(3)) > 1.8
