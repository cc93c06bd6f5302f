"""The 3-D FP64 MUSCL residual and FD product on grids whose sizes take the
column-marching kernel (columns of 16 x 16 cells walking up z: n0 and n1
multiples of 16, any n2), against the oracle bit for bit.

The other 3-D parity tests use grids that take the tile kernel; these cover
the marching form: its three staged planes and the plane read ahead into
registers, the z face carried from one plane to the next, ranges of planes of
unequal length, periodic wrap at the ends of a range (down to grids of one, two
and three planes), the edge faces exchanged through LDS, and every flux variant
(Rusanov, Roe, constant viscosity, Sutherland's law, the split into inviscid
and viscous parts).
"""
import sys

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv, rok
from tests._util import oracle_problem, relerr, t64

pytestmark = pytest.mark.gpu

NONFINITE, NONPHYSICAL = 1, 16


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1607_06834_amd import load_library
    load_library()
    return torch.device("cuda", 0)


def gpu(pb, precision="fp64", mgs="auto"):
    from paper_1607_06834_amd import Rok
    return Rok(pb, precision, mgs)


def _pb(shape, physics, flux="rusanov", suth=0.0):
    return ri.problem(shape, (0.0, 0.0, 0.0), (1.0, 0.9, 1.2), physics, "muscl", mu=0.05 if physics == "ns" else 0.0,
                      flux=flux, sutherland=suth, t_ref=0.8)


CASES = [((32, 32, 32), "ns", "rusanov", 0.0), ((48, 16, 64), "ns", "roe", 0.0), ((16, 32, 37), "ns", "rusanov", 0.4),
         ((32, 16, 20), "euler", "rusanov", 0.0), ((16, 16, 64), "euler", "roe", 0.0), ((16, 16, 3), "ns", "rusanov", 0.0),
         ((16, 48, 5), "ns", "roe", 0.4), ((32, 16, 2), "euler", "rusanov", 0.0), ((16, 16, 1), "ns", "rusanov", 0.0)]


@pytest.mark.parametrize("shape,physics,flux,suth", CASES)
def test_column_residual_and_fd_product_bitwise(dev, shape, physics, flux, suth):
    say("column residual / fd", shape, physics, flux, suth)
    pb = _pb(shape, physics, flux, suth)
    P = oracle_problem(pb)
    g = gpu(pb)
    y = t64(ri.smooth_random_state(pb, seed=4, amplitude=0.2))
    F = fv.residual(P, y)
    out = g.residual(y.to(dev)).cpu()
    assert torch.equal(out, F), relerr(out, F)
    v = t64(ri.random_direction(P.size, seed=5))
    eps = 1.7e-7
    out = g.jvp(y.to(dev), v.to(dev), "fd", fy=F.to(dev), eps=eps).cpu()
    ref = fv.jvp_fd(P, y, F, v, eps)
    assert torch.equal(out, ref), relerr(out, ref)
    if physics == "ns":
        Fi, Fv = g.residual_split(y.to(dev))
        assert torch.equal(Fi.cpu(), fv.residual(P, y, "inviscid"))
        assert torch.equal(Fv.cpu(), fv.residual(P, y, "viscous"))


@pytest.mark.parametrize("mgs", ["auto", "one_reduce"])
def test_column_step_bitwise(dev, mgs):
    """A whole FD step on a marching-size grid: bitwise against the oracle's
    (every stage residual and Krylov product goes through the marching kernel;
    the one-reduce form passes the basis scale to the product)."""
    say("column step", mgs)
    pb = _pb((32, 16, 32), "ns", "rusanov", 0.0)
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=6, amplitude=0.2))
    h = ri.cfl_step(pb, y.numpy(), 2.0)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "fd")
    ref = rok.rok_step(f, mv, tab, 6, h, y)
    out = gpu(pb, mgs=mgs).step(y.to(dev), h, tab, 6, "fd").cpu()
    assert relerr(out, ref) <= 1e-12
    if mgs == "auto":
        assert torch.equal(out, ref)


def test_column_exact_step(dev):
    """An exact-product step on a marching-size grid: the stage residuals go
    through the marching kernel and the tangent products through the tile
    kernel's dual-number form; within 1e-12 of the oracle's step."""
    say("column exact step")
    pb = _pb((16, 32, 32), "ns", "roe", 0.4)
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=7, amplitude=0.2))
    h = ri.cfl_step(pb, y.numpy(), 2.0)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "exact")
    ref = rok.rok_step(f, mv, tab, 6, h, y)
    out = gpu(pb).step(y.to(dev), h, tab, 6, "exact").cpu()
    assert relerr(out, ref) <= 1e-12


def test_column_flags(dev):
    """A negative pressure in the top plane of a chunk (staged by the chunk
    above as its lower halo too) sets NONPHYSICAL and, through the NaN sound
    speed, NONFINITE; the unperturbed state sets neither."""
    from paper_1607_06834_amd import Rok
    pb = ri.tgv_problem(32, 3)
    y = ri.tgv_state(pb)
    n = 32
    cell = (n - 1) * n * n + 5 * n + 7
    bad = y.copy().reshape(5, -1)
    rho = bad[0, cell]
    ke = 0.5 * sum(bad[1 + d, cell] ** 2 for d in range(3)) / rho
    g_ = pb["gamma"]
    p = (g_ - 1.0) * (bad[4, cell] - ke)
    bad[4, cell] = ke + (-0.1 * p) / (g_ - 1.0)
    bad = bad.reshape(-1)
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y, 2.0)
    g = Rok(pb, "fp64")
    for state, want in ((y, 0), (bad, NONPHYSICAL | NONFINITE)):
        g.step(torch.tensor(state, device=dev), h, tab, 4, "fd")
        f = g.last_status()[0]
        say("column flags", want, f)
        assert f & (NONPHYSICAL | NONFINITE) == want, f
