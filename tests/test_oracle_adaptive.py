"""Pins for the oracle's adaptive step-size control (no GPU).

* The step-doubling estimate is the local error of the two-half-step result
  to leading order (Richardson): on Lorenz-96 (Appendix) the ratio of the
  estimate to the true local error tends to 1 as the step shrinks, for the
  explicit RK4 method and for ROK4 with exact products.
* Tighter tolerances give smaller global errors (Lorenz-96).
* On a stiff linear system the explicit method's accepted steps stay at its
  stability limit whatever the tolerance while ROK's follow the tolerance:
  the behaviour Sec. 4.2 reports for the cylinder problems.
"""
import math

import numpy as np
import torch

import rok_inputs as ri
from oracle import adaptive, rk, rok


def _l96_state():
    g = torch.Generator().manual_seed(3)
    return 8.0 + torch.randn(40, generator=g, dtype=torch.float64)


def _rok_l96(M):
    f = rk.lorenz96

    def mv(y, fy):
        J = torch.func.jacfwd(f)(y)
        return lambda v: J @ v

    return lambda y, h: rok.rok_step(f, mv, ri.rok4_tableau(), M, h, y)


def _erk(f):
    return lambda y, h: rk.erk_step(f, rk.RK4_A, rk.RK4_B, h, y)


def test_step_doubling_estimate_is_the_local_error():
    y0 = _l96_state()
    ref_step = _erk(rk.lorenz96)
    for name, step in (("erk4", _erk(rk.lorenz96)), ("rok4", _rok_l96(8))):
        ratios = []
        for H in (0.02, 0.01, 0.005):
            y_full = step(y0, H)
            y_half = step(step(y0, 0.5 * H), 0.5 * H)
            est = float(torch.linalg.norm(y_half - y_full)) / 15.0
            y_ref = y0
            for _ in range(256):
                y_ref = ref_step(y_ref, H / 256)
            true = float(torch.linalg.norm(y_half - y_ref))
            ratios.append(est / true)
        assert abs(ratios[-1] - 1.0) < 0.1, (name, ratios)
        assert abs(ratios[-1] - 1.0) <= abs(ratios[0] - 1.0) + 1e-3, (name, ratios)


def test_tighter_tolerance_smaller_error():
    y0 = _l96_state()
    step = _rok_l96(8)
    T = 0.5
    yr = y0
    for _ in range(2000):
        yr = rk.erk_step(rk.lorenz96, rk.RK4_A, rk.RK4_B, T / 2000, yr)
    errs = []
    for tol in (1e-4, 1e-6, 1e-8):
        y, rec = adaptive.integrate(step, y0, T, 0.01, tol, tol)
        assert rec["accepted"][-1][0] + rec["accepted"][-1][1] == T or abs(
            rec["accepted"][-1][0] + rec["accepted"][-1][1] - T) < 1e-15
        errs.append(float(torch.linalg.norm(y - yr)) / float(torch.linalg.norm(yr)))
    assert errs[0] > 20 * errs[1] > 400 * errs[2], errs


def test_stiff_system_explicit_steps_bound_by_stability():
    """y' = L y + g: a fast mode (-2000) and slow oscillators; RK4 is stable
    for h <= 2.785 / 2000.  The explicit method's mean accepted step stays at
    that limit for every tolerance, with many rejections (the controller
    probes past the limit and the growing fast mode throws it back); ROK with M = N (the Rosenbrock method with the
    exact Jacobian) takes steps set by the tolerance, far above it."""
    N = 6
    L = torch.zeros(N, N, dtype=torch.float64)
    L[0, 0] = -2000.0
    L[1, 2], L[2, 1] = 1.0, -1.0
    L[3, 4], L[4, 3] = 2.0, -2.0
    L[5, 5] = -0.5
    f = lambda y: L @ y + 0.1
    mv = lambda y, fy: (lambda v: L @ v)
    y0 = torch.ones(N, dtype=torch.float64)
    T = 2.0
    mean = {}
    for tol in (1e-4, 1e-8):
        _, re = adaptive.integrate(_erk(f), y0, T, 1e-3, tol, tol)
        _, rr = adaptive.integrate(lambda y, h: rok.rok_step(f, mv, ri.rok4_tableau(), N, h, y), y0, T, 1e-3,
                                   tol, tol)
        he = [H for _, H, _ in re["accepted"]]
        hr = [H for _, H, _ in rr["accepted"]]
        mean[tol] = (T / len(he), T / len(hr))
        # a macro step is two stable steps of H/2: the mean sits at the limit
        assert T / len(he) <= 1.1 * 2 * 2.785 / 2000
        assert len(re["rejected"]) > 0.2 * len(he)
    # explicit: the step count hardly changes with the tolerance; ROK: it follows the tolerance
    assert mean[1e-8][0] > 0.5 * mean[1e-4][0]
    assert mean[1e-4][1] > 20 * mean[1e-4][0]
    assert mean[1e-4][1] > 4 * mean[1e-8][1]


def test_controller_step_factor():
    assert adaptive.next_step(1.0, 1.0, 4, False) == 0.9
    assert adaptive.next_step(1.0, 1e-12, 4, False) == 4.0
    assert adaptive.next_step(1.0, 1e-12, 4, True) == 1.0
    assert adaptive.next_step(1.0, 1e6, 4, True) == 0.2
    assert math.isclose(adaptive.next_step(2.0, 32.0, 4, True), 2.0 * 0.9 * 32.0 ** -0.2)


def test_error_sum_by_hand():
    """sc = atol + rtol*max(|y_n|, |y_half|), q = (y_half - y_full)/((2^p-1) sc),
    worked by hand on two components."""
    yn = torch.tensor([1.0, -2.0], dtype=torch.float64)
    yh = torch.tensor([3.0, 1.0], dtype=torch.float64)
    yf = torch.tensor([0.0, 2.0], dtype=torch.float64)
    # sc = (2.5, 2.0); differences (3, -1)
    assert math.isclose(adaptive.error_sum(yn, yh, yf, 0.5, 1.0, order=1), 1.2 ** 2 + 0.5 ** 2, rel_tol=1e-15)
    assert math.isclose(adaptive.error_sum(yn, yh, yf, 0.5, 1.0, order=4),
                        (3.0 / 37.5) ** 2 + (1.0 / 30.0) ** 2, rel_tol=1e-15)


def test_accepted_steps_cover_the_interval():
    y0 = _l96_state()
    _, rec = adaptive.integrate(_erk(rk.lorenz96), y0, 0.3, 0.05, 1e-5, 1e-5)
    t = 0.0
    for t0, H, err in rec["accepted"]:
        assert t0 == t and err <= 1.0
        t = t0 + H
    assert abs(t - 0.3) < 1e-15 and all(e > 1.0 for _, _, e in rec["rejected"])


def test_rok4_has_no_embedded_order3_weights():
    """Why step doubling: the four order-3 conditions (the first four rows of
    the ROK conditions) are linear in the weights; for the four-stage ROK4
    tableau their matrix is nonsingular, so the only order-3 weights are b
    itself and an embedded pair would estimate zero."""
    tab = ri.rok4_tableau()
    s = tab["s"]
    al = np.array(tab["alpha"], dtype=np.float64).reshape(s, s)
    ga = np.array(tab["gam"], dtype=np.float64).reshape(s, s)
    g = float(tab["gamma"])
    be = al + ga
    a, bp = al.sum(axis=1), be.sum(axis=1)
    A = np.stack([np.ones(s), bp, a ** 2, be @ bp])
    rhs = np.array([1.0, 0.5 - g, 1.0 / 3.0, 1.0 / 6.0 - g + g * g])
    assert np.linalg.cond(A) < 1e6
    bhat = np.linalg.solve(A, rhs)
    assert np.allclose(bhat, np.array(tab["b"], dtype=np.float64), rtol=0, atol=1e-12)
