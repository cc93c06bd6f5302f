"""Roe flux on the GPU against the oracle (ROK_ROE).

Same bars as the Rusanov path: FP64 residual and FD products bit for bit
(one operation order on both sides, correctly rounded / and sqrt), exact
(tangent) products and exact-product steps to 1e-12, FD steps and the 32^2
vortex trajectory bit for bit, FP32 residual/tangent within 2e-6 of the FP64
oracle on smooth states.  A transonic state puts many faces inside the
entropy-fix band of the acoustic waves, so both branches are compared.  The
adjoint products (FP64) against the oracle's reverse mode to 1e-12,
the step adjoint to 1e-10.
"""
import math
import sys

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv, rok
from tests._util import oracle_problem, relerr, t64

pytestmark = pytest.mark.gpu


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


def gpu(pb, precision="fp64"):
    from paper_1607_06834_amd import Rok
    return Rok(pb, precision)


VARIANTS = {
    "euler_fo": lambda n: ri.problem(n, (-1.0, -1.5), (1.0, 1.0), "euler", "first", flux="roe"),
    "euler_muscl": lambda n: ri.problem(n, (-1.0, -1.5), (1.0, 1.0), "euler", "muscl", flux="roe"),
    "ns_fo": lambda n: ri.problem(n, (0.0, 0.0), (1.0, 1.3), "ns", "first", mu=0.05, flux="roe"),
    "ns_muscl": lambda n: ri.problem(n, (0.0, 0.0), (1.0, 1.3), "ns", "muscl", mu=0.05, flux="roe"),
    "euler3d_fo": lambda n: ri.problem(n, (0.0,) * 3, (1.0, 0.9, 1.2), "euler", "first", flux="roe"),
    "euler3d_muscl": lambda n: ri.problem(n, (0.0,) * 3, (1.0, 0.9, 1.2), "euler", "muscl", flux="roe"),
    "ns3d_muscl": lambda n: ri.problem(n, (0.0,) * 3, (1.0, 0.9, 1.2), "ns", "muscl", mu=0.05, flux="roe"),
}
SHAPES_2D = [(6, 5), (37, 21), (70, 33)]
SHAPES_3D = [(5, 4, 3), (19, 9, 7)]
CASES = [(k, s) for k in VARIANTS if "3d" not in k for s in SHAPES_2D] + \
        [(k, s) for k in VARIANTS if "3d" in k for s in SHAPES_3D]


def _transonic(pb, seed):
    """u ~ c (1 +- 10 %) along x: the averaged u - c crosses the band |u - c| < c/8."""
    rng = np.random.default_rng(seed)
    X = ri._mesh(pb)
    D = len(pb["n"])
    L = [pb["hi"][d] - pb["lo"][d] for d in range(D)]
    ph = rng.uniform(0, 2 * math.pi, 4)
    s = [np.sin(2 * math.pi * (X[0] - pb["lo"][0]) / L[0] + ph[k]) for k in range(4)]
    c = math.sqrt(pb["gamma"])
    rho = 1.0 + 0.1 * s[0]
    p = 1.0 + 0.1 * s[1]
    vel = [c * (1.0 + 0.1 * s[2])] + [0.1 * s[3] * (e + 1) for e in range(D - 1)]
    return ri._pack(pb, rho, vel, p)


def _states(pb, seed):
    return [("smooth", ri.smooth_random_state(pb, seed=seed, amplitude=0.2)), ("transonic", _transonic(pb, seed))]


@pytest.mark.parametrize("name,shape", CASES)
def test_roe_residual_fd_tangent(dev, name, shape):
    pb = VARIANTS[name](shape)
    P = oracle_problem(pb)
    g = gpu(pb)
    for kind, y0 in _states(pb, 1):
        say("roe", name, shape, kind)
        y = t64(y0)
        ref = fv.residual(P, y)
        out = g.residual(y.to(dev)).cpu()
        assert torch.equal(out, ref), (kind, relerr(out, ref))
        v = t64(ri.random_direction(P.size, seed=3))
        eps = 1.7e-7
        fd = g.jvp(y.to(dev), v.to(dev), "fd", fy=ref.to(dev), eps=eps).cpu()
        assert torch.equal(fd, fv.jvp_fd(P, y, ref, v, eps)), kind
        tg = g.jvp(y.to(dev), v.to(dev), "exact").cpu()
        assert relerr(tg, fv.jvp_exact(P, y, v)) <= 1e-12, kind


@pytest.mark.parametrize("name", ["euler_fo", "euler_muscl", "ns_muscl", "euler3d_muscl", "ns3d_muscl"])
def test_roe_fp32_error_vs_fp64_oracle(dev, name):
    shape = (37, 21) if "3d" not in name else (19, 9, 7)
    pb = VARIANTS[name](shape)
    P = oracle_problem(pb)
    g = gpu(pb, "fp32")
    for kind, y0 in _states(pb, 8):
        y = t64(y0)
        v = t64(ri.random_direction(P.size, seed=9))
        eF = relerr(g.residual(y.to(dev)).cpu().double(), fv.residual(P, y))
        ew = relerr(g.jvp(y.to(dev), v.to(dev), "exact").cpu().double(), fv.jvp_exact(P, y, v))
        say("roe fp32", name, kind, eF, ew)
        assert eF <= 2e-6 and ew <= 2e-6


def test_roe_fp32_low_mach_taylor_green(dev):
    """Mach 0.1 Taylor-Green at 128^2: the reference-state form keeps the Roe
    residual's digits (p ~ 71 against flux differences ~ 1e-3)."""
    pb = dict(ri.tgv_problem(128, 2), flux="roe")
    P = oracle_problem(pb)
    y = t64(ri.tgv_state(pb))
    eF = relerr(gpu(pb, "fp32").residual(y.to(dev)).cpu().double(), fv.residual(P, y))
    say("roe fp32 tgv128", eF)
    assert eF <= 1e-3


@pytest.mark.parametrize("mode,recon,M", [("fd", "muscl", 8), ("exact", "muscl", 8), ("fd", "first", 6),
                                          ("exact", "first", 0), ("fd", "muscl", 4)])
def test_roe_step_parity(dev, mode, recon, M):
    say("roe step", mode, recon, M)
    pb = dict(ri.vortex_problem(24, recon), flux="roe")
    pb["n"] = (24, 20)
    P = oracle_problem(pb)
    y = t64(ri.perturb_density(pb, ri.vortex_state(pb), 0.01, seed=12))
    h = ri.cfl_step(pb, y.numpy(), 2.0)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, mode)
    ref = rok.rok_step(f, mv, tab, M, h, y)
    g = gpu(pb)
    out = g.step(y.to(dev), h, tab, M, "fd" if mode == "fd" else "exact").cpu()
    flags, meff = g.last_status()
    assert meff == M and flags == 0
    assert relerr(out, ref) <= 1e-12
    if mode == "fd":
        assert torch.equal(out, ref)


def test_roe_vortex32_trajectory(dev):
    """32^2 first-order vortex with the Roe flux, FD products, M = 8, 10 steps at CFL 5, bit for bit."""
    pb, y0, w = ri.workload("vortex32_fo")
    pb = dict(pb, flux="roe")
    P = oracle_problem(pb)
    h = ri.cfl_step(pb, y0, w["cfl"])
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "fd")
    g = gpu(pb)
    yr = t64(y0)
    yg = torch.tensor(y0, device=dev)
    for n in range(w["steps"]):
        yr = rok.rok_step(f, mv, tab, w["M"], h, yr)
        yg = g.step(yg, h, tab, w["M"], "fd")
        assert torch.equal(yg.cpu(), yr), (n, relerr(yg.cpu(), yr))


ADJ_CASES = [("euler_fo", (37, 21)), ("euler_muscl", (6, 5)), ("euler_muscl", (37, 21)), ("euler3d_fo", (5, 4, 3)),
             ("euler3d_muscl", (11, 7, 6))]


@pytest.mark.parametrize("name,shape", ADJ_CASES)
def test_roe_vjp_matches_oracle(dev, name, shape):
    """J(y)^T wbar and d/dt [J(y + t v)^T wbar] of the Roe residual against
    the oracle's reverse-mode products, 1e-12 normwise."""
    pb = VARIANTS[name](shape)
    # first order also on the transonic state (entropy-fix branch); MUSCL's
    # minmod would meet zero transverse slopes there, a kink
    states = _states(pb, 3) if "fo" in name else _states(pb, 3)[:1]
    for kind, y in states:
        _roe_vjp_case(dev, pb, name, shape, kind, y)


def _roe_vjp_case(dev, pb, name, shape, kind, y):
    say("roe vjp", name, shape, kind)
    v, w = ri.random_direction(y.size, 103), ri.random_direction(y.size, 203)
    P = oracle_problem(pb)
    ref1 = fv.vjp(P, t64(y), t64(w))
    ref2 = fv.vjp_second(P, t64(y), t64(v), t64(w))
    g = gpu(pb)
    yd, vd, wd = (torch.tensor(a, device=dev) for a in (y, v, w))
    got = g.vjp(yd, wd).cpu()
    e1 = relerr(got, ref1)
    g1, g2 = g.vjp(yd, wd, v=vd)
    e2 = relerr(g2.cpu(), ref2)
    say("  relerr", e1, e2)
    assert e1 <= 1e-12
    assert torch.equal(g1.cpu(), got)
    assert e2 <= 1e-12
    # <J v, w> = <v, J^T w> with the GPU tangent and adjoint kernels
    jv = g.jvp(yd, vd, mode="tangent")
    a, b = float(torch.dot(jv, wd)), float(torch.dot(vd, g1))
    assert abs(a - b) <= 1e-13 * float(torch.linalg.norm(jv) * torch.linalg.norm(wd))


@pytest.mark.parametrize("recon,n,M", [("first", 8, 6), ("muscl", 12, 8), ("first", 8, 0)])
def test_roe_step_vjp_matches_oracle_gradient(dev, recon, n, M):
    """Gradient of c . y_{n+1} through one exact-product ROK4 step with Roe's
    flux, against the oracle's reverse-mode differentiation of the step, 1e-10."""
    from oracle import rok_ad
    say("roe step vjp", recon, n, M)
    pb = dict(ri.vortex_problem(n, recon), flux="roe")
    y0 = ri.smooth_random_state(pb, seed=11)
    P = oracle_problem(pb)
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y0, 2.0 if M else 0.5)
    c = ri.random_direction(y0.size, 5)
    ref = rok_ad.gradient(lambda z: torch.dot(t64(c), rok_ad.rok_step(P, tab, M, h, z)), t64(y0))
    g = gpu(pb)
    yd, cd = torch.tensor(y0, device=dev), torch.tensor(c, device=dev)
    y1 = torch.empty_like(yd)
    gr = g.step_vjp(yd, cd, h, tab, M, y_next_out=y1).cpu()
    err = relerr(gr, ref)
    say("  relerr", err)
    assert err <= 1e-10
    assert torch.equal(y1, g.step(yd, h, tab, M, mode="tangent"))


def test_roe_adjoint_refused_in_fp32(dev):
    from paper_1607_06834_amd.rok import RokError
    pe = VARIANTS["euler_fo"]((8, 8))
    ye = torch.tensor(ri.smooth_random_state(pe, seed=1), device=dev)
    with pytest.raises(RokError):
        gpu(pe, precision="fp32").vjp(ye, torch.ones_like(ye))
    with pytest.raises(RokError):
        gpu(pe, precision="fp32").step_vjp(ye, torch.ones_like(ye), 1e-3, ri.rok4_tableau(), 4)
