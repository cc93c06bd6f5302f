"""Status word of a step (rok_read_status through the C-ABI): non-physical and
non-finite states.

The gas law has no positivity fix (Sec. 3.2: ideal gas): a stage residual or
product that stages a cell with rho <= 0 or p <= 0 sets ROK_FLAG_NONPHYSICAL,
and the arithmetic goes on (the sound speed of a negative pressure is NaN,
which then sets ROK_FLAG_NONFINITE through the residual's output).  A NaN in
y_n reaches F_1 = f(y_n) and sets ROK_FLAG_NONFINITE only (a NaN compares
false, so it is not reported as non-physical).  Every state here is built on
the host; every kernel runs to completion.
"""
import sys

import numpy as np
import pytest
import torch

import rok_inputs as ri

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


CASES = {
    "euler2d_muscl": (lambda: ri.vortex_problem(24, "muscl"), "fp64"),
    "euler2d_fo": (lambda: ri.vortex_problem(20, "first"), "fp64"),
    "ns2d_muscl": (lambda: ri.tgv_problem(24, 2), "fp64"),
    "ns3d_muscl": (lambda: ri.tgv_problem(12, 3), "fp64"),
    "ns2d_muscl_fp32": (lambda: ri.tgv_problem(24, 2), "fp32"),
    "ns3d_muscl_fp32": (lambda: ri.tgv_problem(12, 3), "fp32"),
}


def _initial(pb):
    return ri.tgv_state(pb) if pb["physics"] == "ns" else ri.vortex_state(pb)


def _cell_view(pb, y):
    D = len(pb["n"])
    return y.reshape((D + 2, -1))


def _negative_pressure(pb, y, cell):
    """Lower the energy of one cell until p = -0.1 p_old (rho and momentum kept)."""
    g = pb["gamma"]
    U = _cell_view(pb, y.copy())
    D = len(pb["n"])
    rho = U[0, cell]
    ke = 0.5 * sum(U[1 + d, cell] ** 2 for d in range(D)) / rho
    p = (g - 1.0) * (U[D + 1, cell] - ke)
    U[D + 1, cell] = ke + (-0.1 * p) / (g - 1.0)
    assert (g - 1.0) * (U[D + 1, cell] - ke) < 0.0
    return U.reshape(-1)


def _negative_density(pb, y, cell):
    """Flip the sign of one cell's density (momentum and energy kept: p stays positive)."""
    U = _cell_view(pb, y.copy())
    U[0, cell] = -U[0, cell]
    return U.reshape(-1)


def _nan(pb, y, cell):
    U = _cell_view(pb, y.copy())
    U[1, cell] = np.nan
    return U.reshape(-1)


def _flags(dev, pb, precision, y, M, mode, mgs="auto"):
    from paper_1607_06834_amd import Rok
    g = Rok(pb, precision, mgs)
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, _initial(pb), 2.0)
    g.step(torch.tensor(y, device=dev), h, tab, M, mode)
    flags, _ = g.last_status()
    return flags


def _modes(precision):
    return [("exact", 6), ("exact", 0)] if precision == "fp32" else [("fd", 6), ("exact", 6), ("fd", 0)]


@pytest.mark.parametrize("name", list(CASES))
def test_physical_state_sets_no_flag(dev, name):
    make, prec = CASES[name]
    pb = make()
    y = _initial(pb)
    for mode, M in _modes(prec):
        say("physical", name, mode, M)
        f = _flags(dev, pb, prec, y, M, mode)
        assert f & (NONFINITE | NONPHYSICAL) == 0, f


@pytest.mark.parametrize("name", list(CASES))
def test_negative_pressure_sets_nonphysical(dev, name):
    make, prec = CASES[name]
    pb = make()
    ncell = int(np.prod(pb["n"]))
    y = _negative_pressure(pb, _initial(pb), ncell // 3)
    for mode, M in _modes(prec):
        say("negative pressure", name, mode, M)
        f = _flags(dev, pb, prec, y, M, mode)
        assert f & NONPHYSICAL, f
        # the sound speed of a negative pressure is NaN: the residual's output is not finite
        assert f & NONFINITE, f


@pytest.mark.parametrize("name", ["euler2d_muscl", "ns3d_muscl", "ns2d_muscl_fp32"])
def test_negative_density_sets_nonphysical(dev, name):
    make, prec = CASES[name]
    pb = make()
    ncell = int(np.prod(pb["n"]))
    y = _negative_density(pb, _initial(pb), ncell // 2 + 1)
    for mode, M in _modes(prec)[:1]:
        say("negative density", name, mode, M)
        f = _flags(dev, pb, prec, y, M, mode)
        assert f & NONPHYSICAL, f


@pytest.mark.parametrize("name", list(CASES))
def test_nan_state_sets_nonfinite_only(dev, name):
    make, prec = CASES[name]
    pb = make()
    ncell = int(np.prod(pb["n"]))
    y = _nan(pb, _initial(pb), ncell // 5)
    for mode, M in _modes(prec):
        say("nan", name, mode, M)
        f = _flags(dev, pb, prec, y, M, mode)
        assert f & NONFINITE, f
        assert not (f & NONPHYSICAL), f


@pytest.mark.parametrize("name", ["euler2d_muscl", "ns3d_muscl", "ns2d_muscl_fp32", "ns3d_muscl_fp32"])
def test_flags_same_on_every_gram_schmidt_form(dev, name):
    """The status word does not depend on how the basis is orthogonalised: the
    one-reduce form (whose columns rok_step keeps unnormalised, with their scales
    on the device) and the pass-by-pass form report the flags of the resident
    form, for a physical state, a negative pressure and a NaN."""
    make, prec = CASES[name]
    pb = make()
    ncell = int(np.prod(pb["n"]))
    y0 = _initial(pb)
    states = [("physical", y0), ("negative pressure", _negative_pressure(pb, y0, ncell // 3)),
              ("nan", _nan(pb, y0, ncell // 5))]
    for label, y in states:
        for mode, M in _modes(prec):
            if M == 0:
                continue   # no basis
            ref = _flags(dev, pb, prec, y, M, mode)
            for mgs in ("one_reduce", "pass"):
                f = _flags(dev, pb, prec, y, M, mode, mgs)
                say(label, name, mode, M, mgs, f, "resident:", ref)
                assert f == ref


def test_flags_cleared_by_next_step(dev):
    """The status word belongs to the last call: a physical step after a
    non-physical one on the same workspace reports nothing."""
    from paper_1607_06834_amd import Rok
    pb = ri.vortex_problem(24, "muscl")
    y = ri.vortex_state(pb)
    bad = _negative_pressure(pb, y, 100)
    g = Rok(pb, "fp64")
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y, 2.0)
    say("cleared by next step")
    g.step(torch.tensor(bad, device=dev), h, tab, 6, "fd")
    assert g.last_status()[0] & NONPHYSICAL
    g.step(torch.tensor(y, device=dev), h, tab, 6, "fd")
    assert g.last_status()[0] & (NONFINITE | NONPHYSICAL) == 0


def test_arnoldi_reports_products(dev):
    """rok_arnoldi's status word reports the products: a negative pressure in y
    is staged by every J v_j."""
    from paper_1607_06834_amd import Rok
    pb = ri.tgv_problem(16, 2)
    y = ri.tgv_state(pb)
    g = Rok(pb, "fp64")
    say("arnoldi flags")
    for state, want in ((y, 0), (_negative_pressure(pb, y, 40), NONPHYSICAL)):
        yt = torch.tensor(state, device=dev)
        F = torch.tensor(ri.smooth_random_state(pb, seed=3, amplitude=0.2), device=dev)
        g.arnoldi(yt, F, 4, "exact")
        f = g.last_arnoldi_flags()
        assert (f & NONPHYSICAL) == want, f
