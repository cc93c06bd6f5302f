"""Pins for the oracle's Arnoldi, reduced solve and ROK step (no GPU).

Checked against what the mathematics fixes: orthonormality and V^T J V = H
against a brute-force Jacobian, V H V^T = J when M = N, the breakdown cases,
LU against a library solve, the explicit limit M = 0 against an independently
written Runge-Kutta step, the linear-problem identities (ROK with M = N is
the Rosenbrock method with the exact Jacobian), free-stream and conservation
invariants, and observed temporal order on Lorenz-96 (Appendix, Table 4) and
on the vortex.
"""
import math

import numpy as np
import pytest
import torch

import rok_inputs as ri
from oracle import fv, krylov, rk, rok
from tests._util import oracle_problem, relerr, t64


def _tiny():
    pb = ri.problem((5, 4), (-1.0, -1.0), (1.0, 1.0), "euler", "muscl")
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=2, amplitude=0.2))
    return P, y


@pytest.mark.parametrize("n", [1, 255, 257, 4099, 262147, 600001])
def test_canonical_sum_is_a_faithful_sum(n):
    """The canonical-order sum is within the classical recursive-summation
    bound of the exactly rounded sum (math.fsum) and exact on integers."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-5, 5, n))
    s = krylov.canonical_sum(x)
    depth = -(-n // krylov.RED_LANES) + 8 + 2 + 8
    bound = depth * 2.0**-53 * float(np.abs(x).sum())
    assert abs(s - math.fsum(x)) <= bound
    xi = rng.integers(-1000, 1000, n).astype(np.float64)
    assert krylov.canonical_sum(xi) == float(xi.sum())


def test_arnoldi_invariants_against_bruteforce_jacobian():
    P, y = _tiny()
    J = fv.dense_jacobian_fd(P, y, 1e-6)
    F = fv.residual(P, y)
    V, H, m = krylov.arnoldi(lambda v: fv.jvp_exact(P, y, v), F, 8)
    assert m == 8
    assert float(torch.abs(V.T @ V - torch.eye(m)).max()) <= 1e-12
    assert relerr(V.T @ J @ V, H) <= 1e-7            # J itself is a 1e-8 brute force
    assert float(torch.abs(torch.tril(H, -2)).max()) == 0.0
    assert bool((torch.diagonal(H, -1) > 0).all())
    assert relerr(V[:, 0], F / torch.linalg.norm(F)) <= 1e-15


def test_arnoldi_full_space_reproduces_operator():
    """M = N: V H V^T = J (exact in exact arithmetic; MGS keeps V orthonormal
    for a well-conditioned Krylov basis, so a small random operator is used)."""
    rng = np.random.default_rng(5)
    N = 12
    J = torch.tensor(rng.standard_normal((N, N)))
    f = torch.tensor(rng.standard_normal(N))
    V, H, m = krylov.arnoldi(lambda v: J @ v, f, N)
    assert m == N
    assert relerr(V @ H @ V.T, J) <= 1e-11


def test_arnoldi_breakdowns():
    N = 12
    z = torch.zeros(N)
    V, H, m = krylov.arnoldi(lambda v: v, z, 5)
    assert m == 0 and V.shape == (N, 0)
    # f is an eigenvector of the operator: the Krylov space is invariant after one vector
    L = torch.diag(torch.arange(1.0, N + 1))
    f = torch.zeros(N)
    f[3] = 2.0
    V, H, m = krylov.arnoldi(lambda v: L @ v, f, 5)
    assert m == 1 and abs(H[0, 0].item() - 4.0) < 1e-15
    # M larger than N is clamped
    g = torch.linspace(1, 2, N)
    V, H, m = krylov.arnoldi(lambda v: L @ v, g, 50)
    assert m <= N


def test_lu_solve_matches_library():
    rng = np.random.default_rng(0)
    for n in (1, 3, 8, 20):
        A = torch.tensor(rng.standard_normal((n, n)) + n * np.eye(n) * rng.uniform(0, 1))
        if n > 1:
            A[0, 0] = 0.0  # forces a pivot
        b = torch.tensor(rng.standard_normal(n))
        LU, perm = krylov.lu_factor(A)
        x = krylov.lu_solve(LU, perm, b)
        ref = torch.tensor(np.linalg.solve(A.numpy(), b.numpy()))
        assert relerr(x, ref) <= 1e-12 * np.linalg.cond(A.numpy())


def test_m0_is_the_explicit_method():
    pb = ri.vortex_problem(16, "muscl")
    P = oracle_problem(pb)
    y = t64(ri.vortex_state(pb))
    h = ri.cfl_step(pb, y.numpy(), 0.5)
    f, mv = rok.fv_system(P)
    y1 = rok.rok_step(f, mv, ri.rk4_tableau(), 0, h, y)
    y2 = rk.erk_step(f, rk.RK4_A, rk.RK4_B, h, y)
    assert relerr(y1, y2) <= 1e-14
    # the derived ROK4 table has the classical RK4 (alpha, b)
    y3 = rok.rok_step(f, mv, ri.rok4_tableau(), 0, h, y)
    assert relerr(y3, y2) <= 1e-14


@pytest.mark.parametrize("gamma", [1.0, 0.5])
def test_linear_problem_full_space_is_rosenbrock(gamma):
    """f = L y, M = N, s = 1: y1 = (I - h gamma L)^{-1} (I + h (1 - gamma) L) y0."""
    rng = np.random.default_rng(4)
    N = 10
    L = torch.tensor(rng.standard_normal((N, N)) - 3 * np.eye(N))
    y0 = torch.tensor(rng.standard_normal(N))
    h = 0.3
    tab = {"s": 1, "alpha": [[0.0]], "gam": [[0.0]], "gamma": gamma, "b": [1.0]}
    y1 = rok.rok_step(lambda y: L @ y, lambda y, fy: (lambda v: L @ v), tab, N, h, y0)
    I = torch.eye(N)
    ref = torch.linalg.solve(I - h * gamma * L, (I + h * (1 - gamma) * L) @ y0)
    assert relerr(y1, ref) <= 1e-13


def test_free_stream_step_is_bitwise_identity():
    pb = ri.vortex_problem(8, "muscl")
    P = oracle_problem(pb)
    y = t64(ri.uniform_state(pb, 1.0, [0.3, 0.2], 1.0))
    f, mv = rok.fv_system(P)
    rec = {}
    y1 = rok.rok_step(f, mv, ri.rok4_tableau(), 6, 0.1, y, rec)
    assert rec["M_eff"] == 0
    assert torch.equal(y1, y)


@pytest.mark.parametrize("mode", ["fd", "exact"])
def test_step_conserves_totals(mode):
    pb = ri.problem((12, 10), (-1.0, -1.0), (1.0, 1.0), "euler", "muscl")
    P = oracle_problem(pb)
    y = t64(ri.smooth_random_state(pb, seed=8))
    f, mv = rok.fv_system(P, mode)
    h = ri.cfl_step(pb, y.numpy(), 2.0)
    y1 = rok.rok_step(f, mv, ri.rok4_tableau(), 8, h, y)
    s0 = y.reshape(4, -1).sum(1)
    s1 = y1.reshape(4, -1).sum(1)
    assert float(torch.abs(s1 - s0).max()) <= 1e-12 * float(torch.abs(y).sum())


def _l96_orders(tab, M, T=0.2, h0=0.02, levels=3, seed=3):
    f = rk.lorenz96

    def mv(y, fy):
        J = torch.func.jacfwd(f)(y)          # exact Jacobian of the 40-variable model
        return lambda v: J @ v

    g = torch.Generator().manual_seed(seed)
    u0 = 8.0 + torch.randn(40, generator=g, dtype=torch.float64)
    yr = u0
    hr = h0 / 2 ** (levels + 5)
    for _ in range(round(T / hr)):
        yr = rk.erk_step(f, rk.RK4_A, rk.RK4_B, hr, yr)
    errs = []
    for k in range(levels):
        h = h0 / 2**k
        y = u0
        for _ in range(round(T / h)):
            y = rok.rok_step(f, mv, tab, M, h, y)
        errs.append(float(torch.linalg.norm(y - yr)))
    return [math.log2(errs[i] / errs[i + 1]) for i in range(levels - 1)]


def test_rok4_order_on_lorenz96():
    """Appendix, Table 4: ROK keeps (close to) its full order 4 on Lorenz-96."""
    orders = _l96_orders(ri.rok4_tableau(), 4)
    assert min(orders) >= 3.8, orders


def test_split_condition_matters_only_for_small_krylov_space():
    """A table satisfying only the classical Rosenbrock conditions loses order
    when M = 4 < N, but not when the Krylov space is the whole space."""
    o_small = _l96_orders(ri.ros4_only_tableau(), 4, levels=4, h0=0.01)
    o_full = _l96_orders(ri.ros4_only_tableau(), 40, levels=4, h0=0.01)
    assert o_full[-1] > 3.9
    assert o_small[-1] < o_full[-1] - 0.15, (o_small, o_full)


def test_rok4_order_on_the_vortex():
    """Temporal order on the semi-discrete vortex (32^2 first-order Rusanov,
    density-perturbed, exact products, M = 8): four steps at CFL 2 and eight at
    CFL 1 against a reference at CFL 1/8.  Measured rate 3.99.  At smaller
    steps the rate falls (2.96, then 1.91): the wave-speed maximum and |u| of
    the Rusanov flux make f only piecewise smooth, and a step that crosses one
    of its switches has a local error of lower order, so the asymptotic order
    is pinned on the smooth Lorenz-96 system above."""
    pb = ri.vortex_problem(32, "first")
    y0 = t64(ri.perturb_density(pb, ri.vortex_state(pb)))
    P = oracle_problem(pb)
    f, mv = rok.fv_system(P, "exact")
    tab = ri.rok4_tableau()
    h0 = ri.cfl_step(pb, y0.numpy(), 2.0)

    def run(h, k):
        y = y0
        for _ in range(k):
            y = rok.rok_step(f, mv, tab, 8, h, y)
        return y

    ref = run(h0 / 16, 64)
    e0 = float(torch.linalg.norm(run(h0, 4) - ref))
    e1 = float(torch.linalg.norm(run(h0 / 2, 8) - ref))
    assert math.log2(e0 / e1) >= 3.7, (e0, e1)


@pytest.mark.parametrize("recon,rate", [("first", 0.75), ("muscl", 1.5)])
def test_vortex_trajectory_converges_to_the_travelling_solution(recon, rate):
    """ROK4 (FD products, M = 8, CFL 2) integrates the isentropic vortex to
    t = 1; its distance to the closed-form translated vortex shrinks at the
    scheme's spatial order under refinement 32^2 -> 64^2 -> 128^2 (measured
    rates 0.68, 0.82 first order; 1.60, 1.67 MUSCL, whose minmod limiter clips
    the extrema)."""
    errs = []
    for n in (64, 128):
        pb = ri.vortex_problem(n, recon)
        P = oracle_problem(pb)
        y0 = ri.vortex_state(pb)
        h = ri.cfl_step(pb, y0, 2.0)
        K = math.ceil(1.0 / h)
        f, mv = rok.fv_system(P, "fd")
        y = t64(y0)
        for _ in range(K):
            y = rok.rok_step(f, mv, ri.rok4_tableau(), 8, 1.0 / K, y)
        errs.append(float(torch.linalg.norm(y - t64(ri.vortex_state(pb, t=1.0)))) / math.sqrt(y.numel()))
    assert math.log2(errs[0] / errs[1]) >= rate, errs
