"""Pins of the oracle's branch-decision context (oracle/fv.py `branches`).

f is piecewise smooth: minmod, |u_n| and the Rusanov maximum choose between
smooth branches.  The context records each decision's distance from its
switch and can take a decision the other way.  Pinned here: recording and an
empty flip change nothing (bit for bit); a constructed tie has margin 0; and
taking a near-switch decision the other way at y gives the product J v of the
state just across that switch (the other one-sided Jacobian), to the size of
the move across it.
"""
import pytest
import torch

import rok_inputs as ri
from oracle import fv
from tests._util import oracle_problem, relerr, t64

pytestmark = pytest.mark.filterwarnings("ignore")


def _setup(n=12, physics="euler"):
    pb = ri.tgv_problem(n, 2) if physics == "ns" else ri.vortex_problem(n, "muscl")
    y0 = ri.tgv_state(pb) if physics == "ns" else ri.vortex_state(pb)
    y = t64(ri.perturb_generic(pb, y0))
    return pb, oracle_problem(pb), y


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_recording_and_empty_flip_change_nothing(physics):
    pb, P, y = _setup(physics=physics)
    v = torch.tensor(ri.random_direction(y.numel(), 3))
    F = fv.residual(P, y)
    Jv = fv.jvp_exact(P, y, v)
    with fv.branches(record=True) as br:
        F2 = fv.residual(P, y)
    assert torch.equal(F, F2)
    assert len(br.margins) == 2 * (2 * 4 * 2 + 3)   # per direction: 4 primitives x 2 minmods x 2, Rusanov 3
    empty = {s: torch.zeros_like(m, dtype=torch.bool) for s, (_, m) in br.margins.items()}
    with fv.branches(flip=empty):
        Jv2 = fv.jvp_exact(P, y, v)
    assert torch.equal(Jv, Jv2)
    for kind, m in br.margins.values():
        assert bool((m >= 0).all())


def test_constructed_tie_has_zero_margin():
    """Uniform flow: every slope is 0 (minmod sign margin 0) and the two wave
    speeds of every face are equal (max margin 0)."""
    pb = ri.vortex_problem(8, "muscl")
    P = oracle_problem(pb)
    y = t64(ri.uniform_state(pb, 1.0, [0.3, 0.2], 1.0))
    with fv.branches(record=True) as br:
        fv.residual(P, y)
    kinds = {}
    for kind, m in br.margins.values():
        kinds.setdefault(kind, []).append(float(m.max()))
    assert max(kinds["minmod a b <= 0"]) == 0.0
    assert max(kinds["max(s_L, s_R)"]) == 0.0
    assert min(kinds["|u_n,L|"]) > 0.0


def _move_across(P, y, cell, var, amount):
    """y with the primitive `var` of one cell shifted by `amount` (others kept)."""
    U = y.reshape(P.nvar, -1).clone()
    r, vel, p = fv.primitives(P, [U[m] for m in range(P.nvar)])
    q = [r.clone()] + [u.clone() for u in vel] + [p.clone()]
    q[var][cell] = q[var][cell] + amount
    Un = fv.conserved(P, q[0], q[1:1 + P.ndim], q[P.ndim + 1])
    return torch.stack(Un).reshape(-1)


@pytest.mark.parametrize("var", [0, 3])
def test_flip_gives_the_other_one_sided_product(var):
    """Put one minmod slope a hair (1e-9 of the field's spread) on one side of
    its sign switch; flipping that decision at y must give J v of the state
    moved just across the switch (to ~1e-7 relative: the move itself), while
    the unflipped product differs from it by O(1) of that face's share."""
    pb, P, y = _setup(n=10)
    n = pb["n"][0]
    cell = 4 * n + 5                      # interior cell (i = 5, j = 4)
    U = y.reshape(P.nvar, -1)
    r, vel, p = fv.primitives(P, [U[m] for m in range(P.nvar)])
    q = ([r] + vel + [p])[var]
    spread = float(q.max() - q.min())
    # the left slope of the x-face reconstruction at `cell`: a = q[cell] - q[cell - 1]
    target = float(q[cell - 1]) + 1e-9 * spread
    y_near = _move_across(P, y, cell, var, target - float(q[cell]))
    y_far = _move_across(P, y, cell, var, target - float(q[cell]) - 2e-9 * spread)   # a = -1e-9 spread
    v = torch.tensor(ri.random_direction(y.numel(), 5))
    with fv.branches(record=True) as br:
        fv.residual(P, y_near)
    # every decision within 1e-8 of its switch: the slope q[cell] - q[cell - 1] enters
    # several minmods (as a or b of the faces on either side), all of which switch together
    flip = {s: m < 1e-8 for s, (k, m) in br.margins.items() if bool((m < 1e-8).any())}
    assert flip and all(k.startswith("minmod a b") for k in (br.margins[s][0] for s in flip))
    assert 2 <= sum(int(m.sum()) for m in flip.values()) <= 4
    with fv.branches(flip=flip):
        Jflip = fv.jvp_exact(P, y_near, v)
    J_near = fv.jvp_exact(P, y_near, v)
    J_far = fv.jvp_exact(P, y_far, v)
    e_flip = relerr(Jflip, J_far)
    e_plain = relerr(J_near, J_far)
    assert e_flip < 1e-6, (e_flip, e_plain)
    assert e_plain > 1e3 * max(e_flip, 1e-16)


def test_cells_near_switches():
    """The mask holds exactly the two cells of each face with a near-switch
    decision: a uniform flow (every slope 0 and every face's two wave speeds
    equal) is near a switch everywhere; a slope put 1e-9 of the spread from its
    sign switch marks the cells of the faces whose reconstruction uses it."""
    pb = ri.vortex_problem(8, "muscl")
    P = oracle_problem(pb)
    uni = t64(ri.uniform_state(pb, 1.0, [0.3, 0.2], 1.0))
    assert bool(fv.cells_near_switches(P, uni, 1e-6).all())
    pb, P, y = _setup(n=10)
    far = fv.cells_near_switches(P, y, 1e-12)
    n = pb["n"][0]
    cell = 4 * n + 5
    U = y.reshape(P.nvar, -1)
    r, vel, p = fv.primitives(P, [U[m] for m in range(P.nvar)])
    spread = float(r.max() - r.min())
    y_near = _move_across(P, y, cell, 0, float(r[cell - 1]) + 1e-9 * spread - float(r[cell]))
    m = fv.cells_near_switches(P, y_near, 1e-8) & ~far
    # the slope r[cell] - r[cell-1] enters the x-faces (cell-2)+1/2 .. cell+1/2: cells cell-2 .. cell+1 of row 4
    got = sorted(int(j) * n + int(i) for j, i in torch.nonzero(m).tolist())
    assert set(got) <= {cell - 2, cell - 1, cell, cell + 1} and {cell - 1, cell} <= set(got)
