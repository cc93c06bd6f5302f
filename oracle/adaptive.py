"""Adaptive step-size control by step doubling (Sec. 4.2 reading).

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

The paper compares the adaptive step sizes of fourth-order explicit
Runge-Kutta and of ROK (Sec. 4.2, the cylinder step-size figures) with its
integrator library's controller, whose estimator it does not state, and no
embedded ROK4 coefficients exist (the four order-3 conditions fix the
weights of a four-stage method uniquely, to b itself).  Reading: the local
error of an order-p one-step method is estimated by step doubling.  A macro
step of size H is attempted as one step of H and two steps of H/2; with

    sc_i  = atol + rtol * max(|y_n,i|, |y_half,i|)
    q_i   = (y_half,i - y_full,i) / ((2^p - 1) * sc_i)
    err   = sqrt( sum_i q_i^2 / N )        (canonical sum)

the step is accepted when err <= 1 and the integration continues from the
two-half-step result; the next macro step is H * min(fmax, max(fmin,
safety * err^(-1/(p+1)))) with safety 0.9, fmin 0.2, fmax 4 (fmax 1 right
after a rejection), and the last step is shortened to end at T.
"""
from __future__ import annotations

import math

import torch

from .krylov import canonical_sum

SAFETY, FMIN, FMAX = 0.9, 0.2, 4.0


def error_sum(y_n: torch.Tensor, y_half: torch.Tensor, y_full: torch.Tensor, rtol: float, atol: float,
              order: int = 4) -> float:
    """sum_i q_i^2 of the estimate above (element by element, then the canonical sum)."""
    c = float(2 ** order - 1)
    sc = atol + rtol * torch.maximum(torch.abs(y_n), torch.abs(y_half))
    q = (y_half - y_full) / (c * sc)
    return canonical_sum((q * q).numpy())


def next_step(H: float, err: float, order: int, after_reject: bool) -> float:
    """The controller's next macro step from the current one and its error."""
    fmax = 1.0 if after_reject else FMAX
    if err == 0.0:
        fac = fmax
    else:
        fac = min(fmax, max(FMIN, SAFETY * err ** (-1.0 / (order + 1))))
    return H * fac


def integrate(step, y0: torch.Tensor, T: float, H0: float, rtol: float, atol: float, order: int = 4,
              max_steps: int = 100000):
    """Integrate to T with step(y, h) -> y_next under step-doubling control.

    Returns (y_T, record) with record = {"accepted": [(t, H, err)], "rejected": [(t, H, err)]}.
    """
    y, t, H = y0, 0.0, float(H0)
    rec = {"accepted": [], "rejected": []}
    after_reject = False
    n = y0.numel()
    for _ in range(max_steps):
        if t >= T:
            break
        last = t + H >= T
        if last:
            H = T - t
        y_full = step(y, H)
        y_mid = step(y, 0.5 * H)
        y_half = step(y_mid, 0.5 * H)
        err = math.sqrt(error_sum(y, y_half, y_full, rtol, atol, order) / n)
        if not math.isfinite(err):
            err = math.inf
        if err <= 1.0:
            rec["accepted"].append((t, H, err))
            t = T if last else t + H
            y = y_half
            H_next = next_step(H, err, order, after_reject)
            after_reject = False
        else:
            rec["rejected"].append((t, H, err))
            H_next = next_step(H, err, order, True) if math.isfinite(err) else H * FMIN
            after_reject = True
        H = H_next
    return y, rec
