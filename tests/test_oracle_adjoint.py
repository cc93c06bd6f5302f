"""Pins of the differentiable ROK step (oracle.rok_ad) against independent facts.

- its value is the step of oracle.rok.rok_step (exact products) to rounding;
- its gradient matches central differences of oracle.rok.rok_step (a separate
  implementation with its own summation order), directionally and, on a tiny
  grid, in every component;
- dropping the dependence of the Krylov basis on the state (a plausible
  mistake in a hand adjoint) fails the difference check by orders of
  magnitude, so the check has the power to see it.

The base states avoid the kinks of f: the Rusanov wave-speed maximum ties on
the symmetry lines of the unperturbed vortex, and minmod ties on symmetric
slopes.  At a tie the exact-product step is discontinuous (J jumps), so a
difference quotient measures the jump, not a derivative.
"""
import warnings

import pytest
import torch

from oracle import rok as orok
from oracle import rok_ad
from rok_inputs import (cfl_step, perturb_density, random_direction, rok4_tableau, smooth_random_state,
                        vortex_problem, vortex_state)
from tests._util import oracle_problem, relerr, t64

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _case(kind, n=8):
    if kind == "fo":
        pb = vortex_problem(n, "first")
        y = perturb_density(pb, vortex_state(pb))
    else:
        pb = vortex_problem(n, "muscl")
        y = smooth_random_state(pb, seed=11)
    return pb, oracle_problem(pb), y


def _fd_directional(L, y, d, rels=(1e-5, 1e-6, 1e-7)):
    """Central differences (L(y + t d) - L(y - t d)) / 2t at relative steps t ||d|| / ||y||."""
    out = []
    for rel in rels:
        t = rel * float(torch.linalg.norm(y)) / float(torch.linalg.norm(d))
        out.append((L(y + t * d) - L(y - t * d)) / (2 * t))
    return out


@pytest.mark.parametrize("kind", ["fo", "muscl"])
def test_value_is_the_oracle_step(torch64, kind):
    pb, P, y0 = _case(kind)
    y = t64(y0)
    tab = rok4_tableau()
    h = cfl_step(pb, y0, 2.0)
    f, mv = orok.fv_system(P, "exact")
    ref = orok.rok_step(f, mv, tab, 6, h, y)
    got = rok_ad.rok_step(P, tab, 6, h, y).detach()
    assert relerr(got, ref) <= 1e-13


@pytest.mark.parametrize("kind,M", [("fo", 6), ("muscl", 6), ("fo", 0)])
def test_step_gradient_matches_central_differences(torch64, kind, M):
    pb, P, y0 = _case(kind)
    y = t64(y0)
    tab = rok4_tableau()
    h = cfl_step(pb, y0, 2.0 if M else 0.5)
    c = t64(random_direction(y.numel(), 5))
    d = t64(random_direction(y.numel(), 6))
    g = rok_ad.gradient(lambda z: torch.dot(c, rok_ad.rok_step(P, tab, M, h, z)), y)
    gd = float(torch.dot(g, d))
    f, mv = orok.fv_system(P, "exact")
    fds = _fd_directional(lambda z: float(torch.dot(c, orok.rok_step(f, mv, tab, M, h, z))), y, d)
    best = min(abs(fd - gd) for fd in fds) / abs(gd)
    assert best <= 1e-6, (gd, fds)


def test_frozen_basis_gradient_is_caught(torch64):
    pb, P, y0 = _case("fo")
    y = t64(y0)
    tab = rok4_tableau()
    h = cfl_step(pb, y0, 2.0)
    c = t64(random_direction(y.numel(), 5))
    d = t64(random_direction(y.numel(), 6))
    gf = rok_ad.gradient(lambda z: torch.dot(c, rok_ad.rok_step(P, tab, 6, h, z, frozen_basis=True)), y)
    gd = float(torch.dot(gf, d))
    f, mv = orok.fv_system(P, "exact")
    fds = _fd_directional(lambda z: float(torch.dot(c, orok.rok_step(f, mv, tab, 6, h, z))), y, d)
    assert min(abs(fd - gd) for fd in fds) / abs(fds[1]) > 1e-3


def test_full_gradient_on_tiny_grid(torch64):
    """Every component of the gradient of KE(step(y)) on a 4 x 4 grid (N = 64) against central differences."""
    pb, P, y0 = _case("fo", n=4)
    y = t64(y0)
    tab = rok4_tableau()
    h = cfl_step(pb, y0, 1.0)
    g = rok_ad.gradient(lambda z: rok_ad.kinetic_energy(P, rok_ad.rok_step(P, tab, 4, h, z)), y)
    f, mv = orok.fv_system(P, "exact")

    def L(z):
        return float(rok_ad.kinetic_energy(P, orok.rok_step(f, mv, tab, 4, h, z)))

    t = 1e-6
    fd = torch.empty_like(y)
    for k in range(y.numel()):
        e = torch.zeros_like(y)
        e[k] = t * max(1.0, abs(float(y[k])))
        fd[k] = (L(y + e) - L(y - e)) / (2 * float(e[k]))
    assert relerr(g, fd) <= 1e-6


def test_trajectory_gradient_of_kinetic_energy(torch64):
    pb, P, y0 = _case("fo")
    y = t64(y0)
    tab = rok4_tableau()
    h = cfl_step(pb, y0, 2.0)
    d = t64(random_direction(y.numel(), 7))
    g = rok_ad.gradient(lambda z: rok_ad.kinetic_energy(P, rok_ad.trajectory(P, tab, 6, h, z, 3)), y)
    gd = float(torch.dot(g, d))
    f, mv = orok.fv_system(P, "exact")

    def L(z):
        return float(rok_ad.kinetic_energy(P, orok.trajectory(f, mv, tab, 6, h, z, 3)))

    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        fds = _fd_directional(L, y, d)
    assert min(abs(fd - gd) for fd in fds) / abs(gd) <= 1e-6, (gd, fds)


def test_kinetic_energy_closed_form(torch64):
    """KE of a uniform flow is rho |u|^2 / 2 times the domain area."""
    from rok_inputs import uniform_state
    pb = vortex_problem(6, "first")
    P = oracle_problem(pb)
    y = t64(uniform_state(pb, rho=1.3, vel=(0.4, -0.7), p=2.0))
    area = (pb["hi"][0] - pb["lo"][0]) * (pb["hi"][1] - pb["lo"][1])
    ke = float(rok_ad.kinetic_energy(P, y))
    assert abs(ke - 0.5 * 1.3 * (0.4 ** 2 + 0.7 ** 2) * area) <= 1e-12 * ke
