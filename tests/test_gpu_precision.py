"""Precision form on the GPU: residual and tangent products in FP32, Arnoldi,
reduced solve and accumulation in FP64; every result against the FP64 oracle.

The FP32 residual and tangent carry perturbations about a reference state, so
their own rounding error is about 1e-7 of f and J v on generic states, and a
step from a given state is within ~1e-7 of the oracle's step from that state.
Beyond that, f is piecewise smooth (minmod, |u_n|, the wave-speed maximum):
the exact-product step jumps where J does, and two states 1e-8 apart can lie
on either side of a switch.  The oracle reports every branch decision of f
with its distance from the switch (oracle.fv.branches), so the tests say
where that happens instead of widening the bound: generic states are held to
1e-5 (the benchmark spec's tolerance for FP32-residual states) step by step from
the same input, and along the whole trajectory until the oracle's decisions
at the two trajectories' states differ (reported on a line of its own); the
analytic initial states sit exactly on switches (mirror symmetry) and are
bounded by the plain FP64 method with finite-difference products.

Full size (2048^2 and 256^3 Taylor-Green): F and J v element by element
against the oracle, the FP64 residual bit for bit, and one step against the
oracle's step stored at sampled indices (tests/golden/make_fullsize_golden.py).
Errors are normwise relative unless stated, also printed relative to the
flow's perturbation y - mean(y).
"""
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


def gpu(pb, precision="fp64"):
    from paper_1607_06834_amd import Rok
    return Rok(pb, precision)


def _pert_rel(a, b, nvar):
    """||a - b|| / ||b - mean(b)||, the mean taken per variable."""
    b2 = b.reshape(nvar, -1)
    dev = b2 - b2.mean(dim=1, keepdim=True)
    return float(torch.linalg.norm((a - b).reshape(nvar, -1))) / float(torch.linalg.norm(dev))


CASES = {
    "tgv2d_32": lambda: (ri.tgv_problem(32, 2), 8, 5),
    "tgv3d_12": lambda: (ri.tgv_problem(12, 3), 8, 3),
    "vortex_muscl_32": lambda: (ri.vortex_problem(32, "muscl"), 8, 5),
}

# Relative distance from a switch below which FP32 rounding of the decision's
# inputs can take the other branch: the FP32 form rounds perturbations about a
# reference state (unit roundoff 6e-8), and the decisions' inputs carry a few
# such roundings of quantities up to the flow's spread.
FP32_DECISION = 1e-6


def _initial(pb, generic, seed=0):
    y0 = ri.tgv_state(pb) if pb["physics"] == "ns" else ri.vortex_state(pb)
    return ri.perturb_generic(pb, y0, seed=ri.PERTURB_SEED + 1 + seed) if generic else y0


def _decisions(P, y):
    with fv.branches(record=True) as br:
        fv.residual(P, y)
    return br


def _fragile(br, delta=FP32_DECISION):
    """{site: mask} of the decisions closer than delta to their switch."""
    return {s: m < delta for s, (_, m) in br.margins.items() if bool((m < delta).any())}


def _count(masks):
    return sum(int(m.sum()) for m in masks.values())


def _differ(ba, bb):
    """{site: mask} where two evaluations took different branches that matter:
    a minmod's |a| <= |b| decision (recorded just before its a b <= 0 decision)
    is moot where that minmod is flat in both."""
    out = {}
    for s, da in ba.decisions.items():
        d = da != bb.decisions[s]
        if ba.margins[s][0] == "minmod |a| <= |b|":
            d = d & ~(ba.decisions[s + 1] & bb.decisions[s + 1])
        if bool(d.any()):
            out[s] = d
    return out


def _step_with_flips(P, tab, M, h, y, flip):
    f, _ = rok.fv_system(P, "exact")

    def matvec_at(yy, fy):
        def mv(v):
            with fv.branches(flip=flip):
                return fv.jvp_exact(P, yy, v)
        return mv
    return rok.rok_step(f, matvec_at, tab, M, h, y)


def _local_error(P, tab, M, h, y_in, y_out, frag):
    """FP32 step result y_out from y_in against the oracle's exact-product step
    from the same y_in; where decisions sit within FP32 rounding of a switch
    (frag), the smallest error over taking up to two of them the other way
    (the other one-sided Jacobians, every one of which an FP32 evaluation may
    see)."""
    base = _step_with_flips(P, tab, M, h, y_in, {})
    e = relerr(y_out, base)
    if e <= 1e-5 or not frag:
        return e, None
    elems = [(s, i) for s, m in frag.items() for i in torch.nonzero(m.reshape(-1)).reshape(-1).tolist()]
    best = (e, None)
    import itertools
    for r in (1, 2):
        for combo in itertools.combinations(elems[:12], r):
            flip = {}
            for s, i in combo:
                mk = flip.setdefault(s, torch.zeros(frag[s].numel(), dtype=torch.bool))
                mk[i] = True
            flip = {s: mk.reshape(frag[s].shape) for s, mk in flip.items()}
            ef = relerr(y_out, _step_with_flips(P, tab, M, h, y_in, flip))
            if ef < best[0]:
                best = (ef, combo)
        if best[0] <= 1e-5:
            break
    return best


GENERIC = [(name, seed) for name in CASES for seed in range(6 if "3d" not in name else 4)]


@pytest.mark.parametrize("name,seed", GENERIC)
def test_fp32_trajectory_generic_states(dev, name, seed):
    """FP32 + tangent trajectory from a generic state (every primitive variable
    seeded-perturbed) against the FP64 exact-product oracle, bound 1e-5.

    f is piecewise smooth (minmod, |u_n|, the wave-speed maximum) and the
    exact-product step is discontinuous where J jumps.  Two checks per step:
    * local: the FP32 step from the GPU's own state y_n against the oracle's
      step from the same y_n, bound 1e-5, at every step (measured 1e-8 .. 1e-7);
      where a decision of f at y_n lies within FP32 rounding of its switch
      (relative margin < FP32_DECISION) the case is reported, and the bound
      holds against the oracle step taking that decision either way;
    * trajectory: the FP32 state against the oracle's own trajectory, bound
      1e-5, as long as the oracle takes the same branch decisions at both
      trajectories' states.  Once they differ (the two trajectories, 1e-8
      apart, straddle a switch) the case is reported on its own line with the
      oracle's own jump between the two states, and the local check carries
      the bound from there."""
    pb, M, K = CASES[name]()
    P = oracle_problem(pb)
    y0 = _initial(pb, True, seed)
    h = ri.cfl_step(pb, y0, 2.5)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "exact")
    ref = rok.trajectory(f, mv, tab, M, h, t64(y0), K, keep=True)
    g32 = gpu(pb, "fp32")
    y = torch.tensor(y0, device=dev)
    straddle = None
    for n in range(1, K + 1):
        y_in = y.cpu()
        y = g32.step(y, h, tab, M, "exact")
        assert g32.last_status()[0] == 0
        y_out = y.cpu()
        br_gpu = _decisions(P, y_in)
        frag = _fragile(br_gpu)
        e_loc, flips = _local_error(P, tab, M, h, y_in, y_out, frag)
        e_traj = relerr(y_out, ref[n])
        diff = _differ(br_gpu, _decisions(P, ref[n - 1]))
        if diff:
            # the oracle's own step from the GPU's state against its step from its own state
            jump = relerr(rok.rok_step(f, mv, tab, M, h, y_in), ref[n])
            kinds = {br_gpu.margins[s][0] for s in diff}
            if straddle is None:
                straddle = [n, _count(diff), kinds, jump]
            else:
                straddle[2] |= kinds
                straddle[3] = max(straddle[3], jump)
        tag = "" if not frag else f"  [{_count(frag)} decision(s) within FP32 rounding of a switch" + \
            (f"; best with {len(flips)} taken the other way]" if flips else "]")
        say(f"{name} seed {seed} step {n}: local {e_loc:.2e}, trajectory {e_traj:.2e}{tag}")
        assert e_loc <= 1e-5
        if straddle is None:
            assert e_traj <= 1e-5
    if straddle is not None:
        n, k, kinds, jump = straddle
        say(f"SWITCH {name} seed {seed}: from step {n} on, the oracle takes different branch decisions at the GPU's "
            f"and at its own state ({k} at step {n}; {', '.join(sorted(kinds))}); its own step differs by up to "
            f"{jump:.2e} between the two states; final trajectory difference {e_traj:.2e}")


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_analytic_states_on_switches(dev, name):
    """The analytic initial states are mirror-symmetric: minmod and the
    wave-speed maximum sit exactly on their switches at many faces (margin 0,
    counted below), where the FP32-rounded evaluation takes whichever branch
    rounding picks and so differentiates other one-sided Jacobians than the
    oracle's tie rule.  Too many ties to enumerate; the reading bounds the FP32
    form by the plain FP64 method with finite-difference products, whose
    increments eps v cross the same ties: FP32 error <= max(1e-5, FD error)."""
    pb, M, K = CASES[name]()
    P = oracle_problem(pb)
    y0 = _initial(pb, False)
    ties = _count(_fragile(_decisions(P, t64(y0)), 1e-300))
    say("fp32 analytic", name, pb["n"], M, K, f"exact ties at y0: {ties}")
    h = ri.cfl_step(pb, y0, 2.5)
    tab = ri.rok4_tableau()
    f, mv = rok.fv_system(P, "exact")
    ref = rok.trajectory(f, mv, tab, M, h, t64(y0), K, keep=True)
    g32, g64 = gpu(pb, "fp32"), gpu(pb, "fp64")
    y32, y64, yfd = (torch.tensor(y0, device=dev) for _ in range(3))
    nvar = len(pb["n"]) + 2
    assert ties > 0
    for n in range(1, K + 1):
        y32 = g32.step(y32, h, tab, M, "exact")
        y64 = g64.step(y64, h, tab, M, "exact")
        yfd = g64.step(yfd, h, tab, M, "fd")
        e32, e64, efd = relerr(y32.cpu(), ref[n]), relerr(y64.cpu(), ref[n]), relerr(yfd.cpu(), ref[n])
        ep = _pert_rel(y32.cpu(), ref[n], nvar)
        say(f"  SWITCH step {n}: fp32 {e32:.3e} (vs perturbation {ep:.3e}), fp64-FD {efd:.3e}, fp64 exact {e64:.3e}")
        assert e64 <= 1e-12
        assert g32.last_status()[0] == 0
        assert e32 <= max(1e-5, efd)


@pytest.mark.parametrize("name", ["tgv2d_32", "vortex_muscl_32"])
def test_fp32_krylov_pair_error(dev, name):
    """(V, H) of the FP32-product Arnoldi against the oracle's exact-product Arnoldi (generic state)."""
    pb, M, _ = CASES[name]()
    P = oracle_problem(pb)
    y = t64(_initial(pb, True))
    F = fv.residual(P, y)
    V, H, m = krylov.arnoldi(lambda v: fv.jvp_exact(P, y, v), F, M)
    g = gpu(pb, "fp32")
    Fg = g.residual(y.to(dev)).double()
    Vg, Hg, mg = g.arnoldi(y.to(dev), Fg, M, "exact")
    eH, eV = relerr(Hg.cpu(), H), relerr(Vg.cpu().T, V)
    say("fp32 krylov", name, "H", eH, "V", eV, "F", relerr(Fg.cpu(), F))
    assert mg == m
    assert eH <= 1e-4 and eV <= 1e-4


def _ke(pb, y):
    n = pb["n"]
    U = y.reshape((len(n) + 2,) + tuple(reversed(n)))
    dV = 1.0
    for d in range(len(n)):
        dV *= (pb["hi"][d] - pb["lo"][d]) / n[d]
    return float((0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]).sum()) * dV


def test_tgv2048_stability_by_cfl(dev):
    """Stability of the 2048^2 viscous Taylor-Green workload over its 20
    steps, CFL doubled from 5 (h = CFL / rho_est from the initial state).
    ROK is only conditionally stable (Table 1): the stated CFL 50 blows up
    within 4 steps in both precisions, CFL 20 within 20; CFL 5 and 10
    integrate the 20 steps, the kinetic energy following exp(-4 nu t) and the
    FP32 form within 1e-5 of the FP64 exact-product trajectory at every step.
    (The FP64 exact-product GPU path is the oracle's arithmetic to 1e-12 on
    the parity grids; the oracle itself is too slow for 2048^2 trajectories.)"""
    import math
    pb, y0, w = ri.workload("tgv2048_ns")
    tab = ri.rok4_tableau()
    yd = torch.tensor(y0, device=dev)
    ke0, nu = _ke(pb, yd), pb["mu"]
    g32, g64 = gpu(pb, "fp32"), gpu(pb, "fp64")
    stable = {}
    for cfl in (5.0, 10.0, 20.0, 50.0):
        h = ri.cfl_step(pb, y0, cfl)
        a, b = yd.clone(), yd.clone()
        worst, k_fail = 0.0, None
        for k in range(1, w["steps"] + 1):
            a = g32.step(a, h, tab, w["M"], "exact")
            b = g64.step(b, h, tab, w["M"], "exact")
            fa, fb = g32.last_status()[0], g64.last_status()[0]
            if fa or fb:
                k_fail = k
                break
            worst = max(worst, relerr(a, b))
        ratio = _ke(pb, b) / (ke0 * math.exp(-4 * nu * k * h)) if k_fail is None else float("nan")
        say(f"  CFL {cfl}: h {h:.3e}, " + (f"stable 20 steps, fp32 vs fp64 worst {worst:.2e}, "
                                            f"KE / (KE0 exp(-4 nu t)) {ratio:.6f}" if k_fail is None
                                            else f"non-finite / non-physical flag at step {k_fail}"))
        stable[cfl] = k_fail is None
        if k_fail is None:
            assert worst <= 1e-5 and abs(ratio - 1.0) <= 1e-3
    assert stable == {5.0: True, 10.0: True, 20.0: False, 50.0: False}
