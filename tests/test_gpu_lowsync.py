"""One-reduce Gram-Schmidt for the Arnoldi columns (ROK_MGS_ONE_REDUCE, the
inverse compact WY form of modified Gram-Schmidt) against the oracle's modified
Gram-Schmidt (Sec. 2.2.2), through the C-ABI.

With exact products the two compute the same coefficients in exact arithmetic
and round differently: V, H and ROK steps within 1e-12 of the oracle.  With
finite-difference products the quotient multiplies the last-bit differences
of the basis by 1/eps, so that path stays on modified Gram-Schmidt (bit for
bit); forcing the one-reduce form there is measured and stated.  Also: M up
to 24, ragged and multi-block sizes, 3-D and the FP32 form, breakdown and a
zero right-hand side, the automatic choice at large N, and the step adjoint
(which keeps modified Gram-Schmidt)."""
import sys

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv, krylov, rok
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


def gpu(pb, precision="fp64", mgs="one_reduce"):
    from paper_1607_06834_amd import Rok
    return Rok(pb, precision, mgs)


CASES = {
    "vortex_muscl_24x20": lambda: dict(ri.vortex_problem(24, "muscl"), n=(24, 20)),
    "vortex_fo_130x67": lambda: dict(ri.vortex_problem(130, "first"), n=(130, 67)),
    "tgv2d_64": lambda: ri.tgv_problem(64, 2),
    "tgv3d_11x9x7": lambda: dict(ri.tgv_problem(11, 3), n=(11, 9, 7)),
}


def _state(pb, seed=11):
    y0 = ri.tgv_state(pb) if pb["physics"] == "ns" else ri.vortex_state(pb)
    return t64(ri.perturb_generic(pb, y0, seed=ri.PERTURB_SEED + seed))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("M", [1, 3, 8, 16, 20, 24])
def test_arnoldi_one_reduce_vs_oracle(dev, name, M):
    pb = CASES[name]()
    P = oracle_problem(pb)
    y = _state(pb)
    F = fv.residual(P, y)
    V, H, m = krylov.arnoldi(lambda v: fv.jvp_exact(P, y, v), F, M)
    Vg, Hg, mg = gpu(pb).arnoldi(y.to(dev), F.to(dev), M, "exact")
    eH, eV = relerr(Hg.cpu(), H), relerr(Vg.cpu().T, V)
    orth = float(torch.linalg.matrix_norm(Vg @ Vg.T - torch.eye(mg, dtype=torch.float64, device=dev)))
    say(f"arnoldi one-reduce {name} N {ri.size(pb)} M {M}: H {eH:.2e}, V {eV:.2e}, ||V^T V - I|| {orth:.1e}")
    assert mg == m
    assert eH <= 1e-12 and eV <= 1e-12 and orth <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("M", [4, 16, 20])
def test_step_one_reduce_vs_oracle(dev, name, M):
    pb = CASES[name]()
    P = oracle_problem(pb)
    y = _state(pb, 12)
    h = ri.cfl_step(pb, y.numpy(), 2.0)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "exact")
    ref = rok.rok_step(f, mv, tab, M, h, y)
    g = gpu(pb)
    out = g.step(y.to(dev), h, tab, M, "exact").cpu()
    flags, meff = g.last_status()
    e, ei = relerr(out, ref), relerr(out - y, ref - y)
    say(f"step one-reduce {name} M {M}: {e:.2e} (increment {ei:.2e})")
    assert meff == M and flags == 0
    assert e <= 1e-12 and ei <= 1e-10


def test_fp32_form_one_reduce(dev):
    """The FP32 form with the one-reduce basis: the step from a generic state
    against the oracle's exact-product step, within the FP32 bound 1e-5, and
    against the same form with modified Gram-Schmidt within 1e-9 (the two
    bases differ in their last bits, which the FP32 products can round apart
    by one FP32 unit in an element now and then)."""
    pb = ri.tgv_problem(48, 2)
    P = oracle_problem(pb)
    y = _state(pb, 13)
    h = ri.cfl_step(pb, y.numpy(), 2.5)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "exact")
    ref = rok.rok_step(f, mv, tab, 16, h, y)
    a = gpu(pb, "fp32").step(y.to(dev), h, tab, 16, "exact").cpu()
    b = gpu(pb, "fp32", "pass").step(y.to(dev), h, tab, 16, "exact").cpu()
    say(f"fp32 one-reduce: vs oracle {relerr(a, ref):.2e}, vs fp32 modified Gram-Schmidt {relerr(a, b):.2e}")
    assert relerr(a, ref) <= 1e-5 and relerr(a, b) <= 1e-9


def test_fd_products_forced_one_reduce(dev):
    """Finite-difference products with the one-reduce basis forced at a size
    where the automatic choice is the resident modified Gram-Schmidt (bit for
    bit): the measured deviation from the oracle's step is stated, 1e-12."""
    pb = CASES["vortex_muscl_24x20"]()
    P = oracle_problem(pb)
    y = _state(pb, 14)
    h = ri.cfl_step(pb, y.numpy(), 2.0)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "fd")
    ref = rok.rok_step(f, mv, tab, 8, h, y)
    out = gpu(pb).step(y.to(dev), h, tab, 8, "fd").cpu()
    auto = gpu(pb, mgs="auto").step(y.to(dev), h, tab, 8, "fd").cpu()
    e = relerr(out, ref)
    say(f"fd products, one-reduce forced: {e:.2e} against the oracle; automatic path bit for bit: "
        f"{torch.equal(auto, ref)}")
    assert torch.equal(auto, ref)
    assert e <= 1e-12


def test_zero_rhs_and_breakdown_one_reduce(dev):
    # zero right-hand side: M_eff = 0 and the step is the identity, bit for bit
    pb = ri.vortex_problem(40, "muscl")
    y = torch.tensor(ri.uniform_state(pb, 1.0, [0.3, 0.2], 1.0), device=dev)
    g = gpu(pb)
    y1 = g.step(y, 0.01, ri.rok4_tableau(), 8, "exact")
    flags, meff = g.last_status()
    assert meff == 0 and flags & 4 and not flags & 1
    assert torch.equal(y1, y)
    # 2 x 2 grid (N = 16), M = 16: the basis stops at an invariant subspace; columns past it take no part
    pb = ri.vortex_problem(2, "first")
    y0 = ri.smooth_random_state(pb, seed=3)
    P = oracle_problem(pb)
    _, _, m = krylov.arnoldi(lambda v: fv.jvp_exact(P, t64(y0), v), fv.residual(P, t64(y0)), 16)
    h = ri.cfl_step(pb, y0, 1.0)
    g = gpu(pb)
    yd = torch.tensor(y0, device=dev)
    a = g.step(yd, h, ri.rok4_tableau(), 16, "exact").clone()
    flags, meff = g.last_status()
    b = g.step(yd, h, ri.rok4_tableau(), meff, "exact")
    say(f"breakdown one-reduce: M_eff {meff} (oracle {m}), flags {flags}")
    assert meff == m < 16 and flags == 2
    assert torch.equal(a, b)


def test_automatic_choice_at_large_n(dev):
    """Above 4194304 unknowns (no room on chip for the work vector) the
    automatic path orthogonalises the columns by the one-reduce form: the same
    bits as forcing it; within 1e-12 of modified Gram-Schmidt with exact
    products and with FD products (state; the increment within 1e-10)."""
    pb = ri.vortex_problem(1100, "first")
    pb["n"] = (1100, 960)                       # N = 4 224 000
    y = torch.tensor(ri.perturb_density(pb, ri.vortex_state(pb), 0.01, seed=15), device=dev)
    h = ri.cfl_step(pb, y.cpu().numpy(), 2.0)
    tab = ri.rok4_tableau()
    auto, one, mgs = gpu(pb, mgs="auto"), gpu(pb), gpu(pb, mgs="pass")
    a = auto.step(y, h, tab, 12, "exact").clone()
    b = one.step(y, h, tab, 12, "exact").clone()
    c = mgs.step(y, h, tab, 12, "exact").clone()
    say(f"large N exact: auto == one-reduce {torch.equal(a, b)}, vs modified Gram-Schmidt {relerr(a, c):.2e}")
    assert torch.equal(a, b) and relerr(a, c) <= 1e-12
    fa = auto.step(y, h, tab, 12, "fd").clone()
    fb = one.step(y, h, tab, 12, "fd").clone()
    fc = mgs.step(y, h, tab, 12, "fd").clone()
    ei = relerr(fa - y, fc - y)
    say(f"large N fd: auto == one-reduce {torch.equal(fa, fb)}, vs modified Gram-Schmidt {relerr(fa, fc):.2e} "
        f"(increment {ei:.2e})")
    assert torch.equal(fa, fb) and relerr(fa, fc) <= 1e-12 and ei <= 1e-10


def test_step_adjoint_keeps_modified_gram_schmidt(dev):
    """rok_step_vjp recomputes its forward with modified Gram-Schmidt whatever
    the path (its reverse is that of modified Gram-Schmidt): the same bits with
    the one-reduce path selected; rok_step_vjp_stored refuses a forward that
    rok_step took with the one-reduce form."""
    from paper_1607_06834_amd import RokError
    pb = dict(ri.vortex_problem(24, "first"), n=(24, 20))
    y = _state(pb, 16).to(dev)
    yb = torch.tensor(ri.random_direction(y.numel(), 6), device=dev)
    h = ri.cfl_step(pb, y.cpu().numpy(), 2.0)
    tab = ri.rok4_tableau()
    a = gpu(pb).step_vjp(y, yb, h, tab, 8)
    b = gpu(pb, mgs="pass").step_vjp(y, yb, h, tab, 8)
    assert torch.equal(a, b)
    g = gpu(pb)
    _, rec = g.step_keep(y, h, tab, 8)
    with pytest.raises(RokError):
        g.step_vjp_stored(rec, yb)
