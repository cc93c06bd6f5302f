"""Finite-volume right-hand side f(y) and its Jacobian-vector products.

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

What is computed (paper Sec. 3.2, eq. 11 and the paragraph after it):
the semi-discrete compressible Euler / Navier-Stokes equations on a periodic,
cell-centred Cartesian grid, written as the autonomous system y' = f(y) of
Sec. 2, eq. 1.  The paper's solver uses MUSCL reconstruction with selectable
limiters and an approximate Riemann flux; here the flux is Rusanov's and the
limiter is minmod, and the grid is Cartesian and periodic.  Readings of what
the paper leaves open:

* state order per cell: [rho, rho*u, rho*v, (rho*w), E]  (the printed order
  [rho, rho v, rho u, E_t] of Sec. 4.1 is a transposition; the L2 error is
  invariant under it);
* ideal gas, p = (gamma-1)(E - rho|u|^2/2), T = p/rho (R = 1), c = sqrt(gamma p/rho);
* MUSCL acts on primitive variables (rho, u, v, (w), p) with
  q_L = q_i + mm(q_i - q_{i-1}, q_{i+1} - q_i)/2,
  q_R = q_{i+1} - mm(q_{i+1} - q_i, q_{i+2} - q_{i+1})/2,
  mm(a, b) = 0 if a*b <= 0, a if |a| <= |b|, else b;
* Rusanov flux with wave speed a = max(|u_n,L| + c_L, |u_n,R| + c_R), or
  Roe's flux (the paper's solver offers Roe and Van Leer fluxes, Sec. 3.2)
  with Harten's entropy fix on the acoustic waves (`_roe`);
* viscous terms: Stokes hypothesis and q = -k grad T (eq. 11) with constant mu,
  or Sutherland's law evaluated at the face temperature (T_a + T_b)/2 (the
  paper's cylinder cases set Sutherland's coefficient, Sec. 4.2),
  k = mu*gamma/((gamma-1) Pr); the energy equation is read in its standard form
  dE/dt + div((E+p)u) = div(tau.u) - div(q) (the printed line repeats k and mu);
  face gradients: two-point difference along the face normal, the average of
  the two neighbouring cells' central differences along the face;
* assembly f_c = sum_d (Fhat_{c-1/2} - Fhat_{c+1/2}) / dx_d over d = x, y, z in
  that order, with 1/dx_d rounded once;
* curvilinear grids (2-D Euler; the paper's solver works on curvilinear
  structured grids, Sec. 3.2): face vectors from the node coordinates, the
  flux in the face frame, `metrics` and `_residual_curvilinear`.

Every formula below is written in one fixed operation order (no fused
multiply-add; left-to-right evaluation), which is the natural reading of the
formula.  Branches of |.|, max and minmod are written with explicit `where` so
that derivatives follow the branch the evaluation took (ties: |0|' = +1, max
tie takes the left state, minmod tie |a| = |b| takes a).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

EULER = "euler"
NS = "ns"
FIRST_ORDER = "first"
MUSCL = "muscl"
RUSANOV = "rusanov"
ROE = "roe"


@dataclass
class Problem:
    """Periodic box, physics and discretisation of f (Sec. 3.2)."""

    n: tuple            # cells per direction, (nx, ny) or (nx, ny, nz)
    lo: tuple           # lower corner per direction
    hi: tuple           # upper corner per direction
    physics: str = EULER
    recon: str = FIRST_ORDER
    gamma: float = 1.4
    mu: float = 0.0
    prandtl: float = 0.72
    flux: str = RUSANOV
    sutherland: float = 0.0   # S / T_ref of Sutherland's law; 0: constant viscosity mu
    t_ref: float = 1.0        # temperature at which the viscosity is mu
    nodes: tuple = None       # 2-D curvilinear grid: node coordinates (x, y), arrays [j][i]
    farfield: tuple = None    # O-grid (periodic in i, wall at j = 0, far field past the last row):
                              # the free-stream conserved state (rho, rho u, rho v, E)
    t_wall: float = 1.0       # O-grid with Navier-Stokes physics: the isothermal wall's temperature
    dtype: torch.dtype = field(default=torch.float64)

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def nvar(self) -> int:
        return self.ndim + 2

    @property
    def ncell(self) -> int:
        return int(math.prod(self.n))

    @property
    def size(self) -> int:
        return self.nvar * self.ncell

    @property
    def shape(self) -> tuple:
        """Tensor shape of the state: variable-major, x fastest."""
        return (self.nvar,) + tuple(reversed(self.n))

    def dx(self, d: int) -> float:
        return (self.hi[d] - self.lo[d]) / self.n[d]

    def invdx(self, d: int) -> float:
        return 1.0 / self.dx(d)


def _at(a: torch.Tensor, s: int, d: int) -> torch.Tensor:
    """Periodic neighbour: value at cell index + s along direction d (x = 0)."""
    return torch.roll(a, shifts=-s, dims=-1 - d)


def _sqrt(x):
    """Correctly rounded square root.

    torch's vectorised CPU float64 sqrt is not correctly rounded (about 1 in
    120 random inputs is one ulp off), so plain evaluations use numpy's IEEE
    square root.  Inside a derivative evaluation (a tensor that requires grad
    or a forward-mode dual) torch.sqrt is used: there only the derivative is
    consumed and one ulp in the value is immaterial.
    """
    try:
        return torch.from_numpy(np.sqrt(x.numpy()))
    except RuntimeError:
        return torch.sqrt(x)


def _absw(x):
    return torch.where(x >= 0, x, -x)


# f is piecewise smooth: minmod, the |.| of the face-normal velocity and the
# maximum of the two Rusanov wave speeds each choose between smooth branches,
# and J jumps where a state crosses such a switch (an exact-product ROK step is
# then discontinuous in y_n).  Inside `with branches(...)`, every one of these
# decisions is routed through the context, in the fixed order in which one
# evaluation of f makes them (a decision "site" = one call, elementwise over
# the grid): a plain evaluation can record each decision's distance from its
# switch, relative to the size of the quantities compared, and any evaluation
# (a forward-mode product included) can take listed decisions the other way,
# i.e. differentiate the other one-sided branch.  Outside a context nothing
# changes.  Roe's flux and the O-grid boundary slopes are not routed.
_BRANCHES = None


class branches:
    """Context: record = True stores {site: (kind, relative margin tensor)} in
    .margins and {site: the decision taken (bool tensor)} in .decisions (plain
    evaluations only); flip = {site: bool tensor} inverts those decisions where
    the mask is True."""

    def __init__(self, record: bool = False, flip: dict | None = None):
        self.record = record
        self.flip = dict(flip or {})
        self.margins = {}
        self.decisions = {}
        self.axes = {}      # site -> direction d of the faces it decides (element c: the face c + 1/2)
        self.axis = None
        self._site = 0
        self._prev = None

    def __enter__(self):
        global _BRANCHES
        self._prev = _BRANCHES
        self._site = 0
        _BRANCHES = self
        return self

    def __exit__(self, *exc):
        global _BRANCHES
        _BRANCHES = self._prev
        return False


def _decide(cond, kind, margin):
    """cond: boolean tensor of one decision site; margin(): its distances from
    the switch (called only when recording)."""
    ctx = _BRANCHES
    if ctx is None:
        return cond
    site = ctx._site
    ctx._site += 1
    f = ctx.flip.get(site)
    out = cond if f is None else torch.logical_xor(cond, f)
    if ctx.record:
        ctx.margins[site] = (kind, margin())
        ctx.decisions[site] = out.clone()
        ctx.axes[site] = ctx.axis
    return out


def _spread(q):
    """Size of a field's variation (its range), the scale of its slopes' decisions."""
    r = float(q.max() - q.min())
    return r if r > 0.0 else 1.0


def _minmod(a, b, q=None):
    """mm(a, b); q (optional): the field whose slopes a, b are (sets the scale of
    the recorded margins, else max |a|, |b|)."""
    zero = torch.zeros_like(a)
    aa, ab = _absw(a), _absw(b)

    def scale():
        return _spread(q) if q is not None else max(float(torch.maximum(aa, ab).max()), 1e-300)

    pick_a = _decide(aa <= ab, "minmod |a| <= |b|",
                     lambda: torch.where(a * b > 0, (aa - ab).abs() / scale(), torch.full_like(a, math.inf)))
    pick = torch.where(pick_a, a, b)
    flat = _decide(a * b <= 0, "minmod a b <= 0", lambda: torch.minimum(aa, ab) / scale())
    return torch.where(flat, zero, pick)


def primitives(P: Problem, U):
    """Conserved -> primitive variables (rho, velocity list, p) per cell."""
    D = P.ndim
    gm1 = P.gamma - 1.0
    r = U[0]
    vel = [U[1 + d] / r for d in range(D)]
    E = U[D + 1]
    ke = vel[0] * vel[0]
    for d in range(1, D):
        ke = ke + vel[d] * vel[d]
    p = gm1 * (E - 0.5 * r * ke)
    return r, vel, p


def conserved(P: Problem, r, vel, p):
    """Primitive -> conserved variables (list of nvar tensors)."""
    D = P.ndim
    gm1 = P.gamma - 1.0
    ke = vel[0] * vel[0]
    for d in range(1, D):
        ke = ke + vel[d] * vel[d]
    E = p / gm1 + 0.5 * r * ke
    return [r] + [r * vel[d] for d in range(D)] + [E]


def _euler_flux(P: Problem, U, vel, p, d):
    """Physical inviscid flux along direction d, from conserved and primitive states."""
    D = P.ndim
    un = vel[d]
    F = [U[1 + d]]
    for e in range(D):
        if e == d:
            F.append(U[1 + e] * un + p)
        else:
            F.append(U[1 + e] * un)
    F.append((U[D + 1] + p) * un)
    return F


def _rusanov(P: Problem, UL, rL, vL, pL, UR, rR, vR, pR, d):
    g = P.gamma
    cL = _sqrt(g * pL / rL)
    cR = _sqrt(g * pR / rR)
    uL, uR = vL[d], vR[d]

    def speed():   # scale of the |u_n| decisions: the largest wave speed at the faces
        return max(float(torch.maximum(uL.abs() + cL, uR.abs() + cR).max()), 1e-300)

    sL = torch.where(_decide(uL >= 0, "|u_n,L|", lambda: uL.abs() / speed()), uL, -uL) + cL
    sR = torch.where(_decide(uR >= 0, "|u_n,R|", lambda: uR.abs() / speed()), uR, -uR) + cR
    a = torch.where(_decide(sL >= sR, "max(s_L, s_R)", lambda: (sL - sR).abs() / torch.maximum(sL, sR)), sL, sR)
    FL = _euler_flux(P, UL, vL, pL, d)
    FR = _euler_flux(P, UR, vR, pR, d)
    return [0.5 * (FL[m] + FR[m]) - 0.5 * a * (UR[m] - UL[m]) for m in range(P.nvar)]


ROE_ENTROPY_FIX = 0.125


def _roe(P: Problem, UL, rL, vL, pL, UR, rR, vR, pR, d):
    """Roe's approximate Riemann flux (Roe 1981) along direction d:
    Fhat = (F_L + F_R)/2 - (sum_k |lambda_k| alpha_k r_k)/2 with the
    density-weighted averages, written in primitive differences.

    Waves (n = e_d): lambda = u_n - c, u_n (entropy and D-1 shear waves),
    u_n + c; strengths alpha_1,3 = (dp -+ rho c du_n)/(2 c^2),
    alpha_2 = drho - dp/c^2, shear alpha_e = rho du_e (e != d); right
    eigenvectors (1, u - c n, H - u_n c), (1, u, |u|^2/2), (0, e_e, u_e),
    (1, u + c n, H + u_n c).  Harten's entropy fix on the two acoustic waves:
    |lambda| < delta -> (lambda^2 + delta^2) / (2 delta), delta = c / 8.
    """
    D = P.ndim
    gm1 = P.gamma - 1.0
    FL = _euler_flux(P, UL, vL, pL, d)
    FR = _euler_flux(P, UR, vR, pR, d)
    sL = _sqrt(rL)
    sR = _sqrt(rR)
    den = sL + sR
    wL = sL / den
    wR = sR / den
    u = [wL * vL[e] + wR * vR[e] for e in range(D)]
    HL = (UL[D + 1] + pL) / rL
    HR = (UR[D + 1] + pR) / rR
    H = wL * HL + wR * HR
    rho = sL * sR
    ke = u[0] * u[0]
    for e in range(1, D):
        ke = ke + u[e] * u[e]
    hke = 0.5 * ke
    c2 = gm1 * (H - hke)
    c = _sqrt(c2)
    un = u[d]
    dr = rR - rL
    dp = pR - pL
    dun = vR[d] - vL[d]
    rc = rho * c
    cc = c2 + c2
    a1 = (dp - rc * dun) / cc
    a3 = (dp + rc * dun) / cc
    a2 = dr - dp / c2
    delta = ROE_ENTROPY_FIX * c

    def fixed(lam):
        l = _absw(lam)
        return torch.where(l < delta, (l * l + delta * delta) / (delta + delta), l)

    l1 = fixed(un - c)
    l2 = _absw(un)
    l3 = fixed(un + c)
    w1 = l1 * a1
    w2 = l2 * a2
    w3 = l3 * a3
    wt = [None] * D
    for e in range(D):
        if e != d:
            wt[e] = l2 * (rho * (vR[e] - vL[e]))
    Dv = [w1 + w2 + w3]
    for e in range(D):
        if e == d:
            Dv.append(w1 * (u[e] - c) + w2 * u[e] + w3 * (u[e] + c))
        else:
            Dv.append(w1 * u[e] + w2 * u[e] + w3 * u[e] + wt[e])
    unc = un * c
    en = w1 * (H - unc) + w2 * hke + w3 * (H + unc)
    for e in range(D):
        if e != d:
            en = en + wt[e] * u[e]
    Dv.append(en)
    return [0.5 * (FL[m] + FR[m]) - 0.5 * Dv[m] for m in range(P.nvar)]


def face_flux(P: Problem, UL, rL, vL, pL, UR, rR, vR, pR, d):
    """The inviscid numerical flux selected by P.flux."""
    if P.flux == RUSANOV:
        return _rusanov(P, UL, rL, vL, pL, UR, rR, vR, pR, d)
    if P.flux == ROE:
        return _roe(P, UL, rL, vL, pL, UR, rR, vR, pR, d)
    raise ValueError(f"unknown flux {P.flux!r}")


def _face_states(P: Problem, U, r, vel, p, d):
    """Left/right states at the face c+1/2 along d, for every cell c."""
    D = P.ndim
    if P.recon == FIRST_ORDER:
        UL = list(U)
        UR = [_at(u, 1, d) for u in U]
        return (UL, r, vel, p), (UR, _at(r, 1, d), [_at(u, 1, d) for u in vel], _at(p, 1, d))
    if P.recon != MUSCL:
        raise ValueError(f"unknown reconstruction {P.recon!r}")
    q = [r] + list(vel) + [p]
    qL, qR = [], []
    for a in q:
        am1, ap1, ap2 = _at(a, -1, d), _at(a, 1, d), _at(a, 2, d)
        qL.append(a + 0.5 * _minmod(a - am1, ap1 - a, a))
        qR.append(ap1 - 0.5 * _minmod(ap1 - a, ap2 - ap1, a))
    rL, vL, pL = qL[0], qL[1:1 + D], qL[D + 1]
    rR, vR, pR = qR[0], qR[1:1 + D], qR[D + 1]
    return (conserved(P, rL, vL, pL), rL, vL, pL), (conserved(P, rR, vR, pR), rR, vR, pR)


def sutherland_mu(P: Problem, T):
    """Sutherland's law mu(T) = mu (T/T_ref)^(3/2) (T_ref + S) / (T + S), written
    with theta = T / T_ref and s = S / T_ref as mu theta sqrt(theta) (1 + s) / (theta + s)."""
    s = P.sutherland
    th = T / P.t_ref
    return P.mu * th * _sqrt(th) * (1.0 + s) / (th + s)


def _viscous_flux(P: Problem, r, vel, p, d):
    """Viscous flux (tau row and energy term) at the face c+1/2 along d."""
    D = P.ndim
    T = p / r
    if P.sutherland > 0.0:
        mu = sutherland_mu(P, 0.5 * (T + _at(T, 1, d)))   # at the face temperature
    else:
        mu = P.mu
    c23mu = (2.0 / 3.0) * mu
    kappa = mu * P.gamma / ((P.gamma - 1.0) * P.prandtl)
    inv = [P.invdx(b) for b in range(D)]

    def grad(a, b):
        """d u_a / d x_b at the face c+1/2 along d."""
        u = vel[a]
        if b == d:
            return (_at(u, 1, d) - u) * inv[d]
        h = 0.5 * inv[b]
        gc = (_at(u, 1, b) - _at(u, -1, b)) * h
        return 0.5 * (gc + _at(gc, 1, d))

    G = [[grad(a, b) for b in range(D)] for a in range(D)]
    div = G[0][0]
    for a in range(1, D):
        div = div + G[a][a]
    tau = []
    for a in range(D):
        if a == d:
            tau.append(mu * (G[a][d] + G[d][a]) - c23mu * div)
        else:
            tau.append(mu * (G[a][d] + G[d][a]))
    uf = [0.5 * (vel[a] + _at(vel[a], 1, d)) for a in range(D)]
    work = uf[0] * tau[0]
    for a in range(1, D):
        work = work + uf[a] * tau[a]
    dTdn = (_at(T, 1, d) - T) * inv[d]
    energy = work + kappa * dTdn
    return [torch.zeros_like(r)] + tau + [energy]


def metrics(P: Problem):
    """Face vectors and inverse cell areas of a 2-D curvilinear periodic grid.

    Cell (i, j) has the nodes p0 = (i, j), p1 = (i+1, j), p2 = (i+1, j+1) and
    p3 = (i, j+1) (periodic offsets Lx, Ly applied past the last node).  Its
    east face (towards i+1) is the edge p1 -> p2 and its north face (towards
    j+1) the edge p3 -> p2; the face vectors are those edges turned by 90
    degrees (length = face length, pointing to increasing i or j), and the
    area is half the cross product of the diagonals.  Returns torch tensors
    (Sx_e, Sy_e, Sx_n, Sy_n, 1/A, dx_e, dy_e, dx_n, dy_n), each [j][i], the last
    four the centroid differences across the east and north faces."""
    xn, yn = (np.asarray(a, dtype=np.float64) for a in P.nodes)
    Lx, Ly = P.hi[0] - P.lo[0], P.hi[1] - P.lo[1]

    def node(di, dj):
        x = np.roll(np.roll(xn, -di, axis=1), -dj, axis=0).copy()
        y = np.roll(np.roll(yn, -di, axis=1), -dj, axis=0).copy()
        if di:
            x[:, -di:] = x[:, -di:] + Lx
        if dj:
            y[-dj:, :] = y[-dj:, :] + Ly
        return x, y

    x0, y0 = xn, yn
    x1, y1 = node(1, 0)
    x2, y2 = node(1, 1)
    x3, y3 = node(0, 1)
    sxe = y2 - y1
    sye = x1 - x2
    sxn = y3 - y2
    syn = x2 - x3
    area = 0.5 * ((x2 - x0) * (y3 - y1) - (x3 - x1) * (y2 - y0))
    # centroid differences across the east and north faces (cell centroid: mean of its nodes)
    x4, y4 = node(2, 0)
    x5, y5 = node(2, 1)
    x6, y6 = node(0, 2)
    x7, y7 = node(1, 2)
    dxe = 0.25 * ((x4 + x5) - (x0 + x3))
    dye = 0.25 * ((y4 + y5) - (y0 + y3))
    dxn = 0.25 * ((x6 + x7) - (x0 + x1))
    dyn = 0.25 * ((y6 + y7) - (y0 + y1))
    return tuple(torch.from_numpy(a) for a in (sxe, sye, sxn, syn, 1.0 / area, dxe, dye, dxn, dyn))


def ogrid_metrics(P: Problem):
    """Face vectors and inverse areas of an O-grid: nodes (x, y) indexed [j][i] with
    j = 0..ny (row 0 on the wall, row ny on the far-field boundary) and i periodic
    without offset (node nx is node 0).  Same conventions as `metrics` (the north
    centroid difference of the last row is zero: that face is the far field);
    also the wall face vectors (the south faces of row 0, pointing into the
    domain) and the vectors from each wall face's midpoint to the first
    cell's centroid."""
    xn, yn = (np.asarray(a, dtype=np.float64) for a in P.nodes)
    r1 = lambda a: np.roll(a, -1, axis=1)
    x0, y0 = xn[:-1], yn[:-1]
    x1, y1 = r1(xn)[:-1], r1(yn)[:-1]
    x2, y2 = r1(xn)[1:], r1(yn)[1:]
    x3, y3 = xn[1:], yn[1:]
    sxe = y2 - y1
    sye = x1 - x2
    sxn = y3 - y2
    syn = x2 - x3
    area = 0.5 * ((x2 - x0) * (y3 - y1) - (x3 - x1) * (y2 - y0))
    wx = yn[0] - r1(yn)[0]
    wy = r1(xn)[0] - xn[0]
    r2 = lambda a: np.roll(a, -2, axis=1)
    dxe = 0.25 * ((r2(xn)[:-1] + r2(xn)[1:]) - (x0 + x3))
    dye = 0.25 * ((r2(yn)[:-1] + r2(yn)[1:]) - (y0 + y3))
    z = np.zeros((1, xn.shape[1]))
    dxn = np.concatenate([0.25 * ((xn[2:] + r1(xn)[2:]) - (xn[:-2] + r1(xn)[:-2])), z])   # no face past the far field
    dyn = np.concatenate([0.25 * ((yn[2:] + r1(yn)[2:]) - (yn[:-2] + r1(yn)[:-2])), z])
    awx = 0.25 * ((x2[0] + x3[0]) - (x0[0] + x1[0]))      # first centroid minus wall-face midpoint
    awy = 0.25 * ((y2[0] + y3[0]) - (y0[0] + y1[0]))
    return tuple(torch.from_numpy(a) for a in (sxe, sye, sxn, syn, 1.0 / area, dxe, dye, dxn, dyn, wx, wy, awx, awy))


def _rotated_flux(P: Problem, UL, rL, vL, pL, UR, rR, vR, pR, sx, sy):
    """Numerical flux through a face with vector (sx, sy): states rotated into the
    face frame, the one-dimensional flux, rotated back, times the face length."""
    ln = _sqrt(sx * sx + sy * sy)
    nx = sx / ln
    ny = sy / ln
    vLr = [vL[0] * nx + vL[1] * ny, vL[1] * nx - vL[0] * ny]
    vRr = [vR[0] * nx + vR[1] * ny, vR[1] * nx - vR[0] * ny]
    ULr = [UL[0], UL[1] * nx + UL[2] * ny, UL[2] * nx - UL[1] * ny, UL[3]]
    URr = [UR[0], UR[1] * nx + UR[2] * ny, UR[2] * nx - UR[1] * ny, UR[3]]
    Fr = face_flux(P, ULr, rL, vLr, pL, URr, rR, vRr, pR, 0)
    return [Fr[0] * ln, (Fr[1] * nx - Fr[2] * ny) * ln, (Fr[1] * ny + Fr[2] * nx) * ln, Fr[3] * ln]


def _residual_ogrid(P: Problem, y: torch.Tensor) -> torch.Tensor:
    """f on an O-grid around a body (2-D): periodic in i; along j the faces
    j + 1/2 for j = -1 (the wall), 0..ny-2 (interior; MUSCL slopes that would
    reach past the wall or the far field are zero) and ny - 1 (the far field:
    the numerical flux between the last cell's primitive state, taken back to
    conserved variables, and the free stream).  Euler: a slip wall carrying the
    first cell's pressure, Fhat = (0, p S, 0).  Navier-Stokes: the same pressure
    flux plus the viscous flux of an isothermal no-slip wall (velocity 0 and
    temperature t_wall on the wall; gradients from the wall value and the first
    cell, through the vector from the wall face's midpoint to that cell's
    centroid); index-space derivatives along j at rows 0 and ny-1 are one-sided;
    no viscous flux through the far field."""
    if P.ndim != 2:
        raise ValueError("O-grids: 2-D only")
    ns = P.physics == NS
    nx, ny = P.n
    U = y.reshape(P.shape)
    U = [U[m] for m in range(P.nvar)]
    r, vel, p = primitives(P, U)
    T = p / r
    sxe, sye, sxn, syn, inva, dxe, dye, dxn, dyn, wx, wy, awx, awy = ogrid_metrics(P)
    phis = [vel[0], vel[1], T]
    # i direction: periodic, as on the curvilinear box
    (UL, rL, vL, pL), (UR, rR, vR, pR) = _face_states(P, U, r, vel, p, 0)
    Fh = _rotated_flux(P, UL, rL, vL, pL, UR, rR, vR, pR, sxe, sye)
    if ns:
        dn = [_at(a, 1, 0) - a for a in phis]
        gc = [torch.cat([(a[1] - a[0])[None], (a[2:] - a[:-2]) * 0.5, (a[-1] - a[-2])[None]]) for a in phis]
        dt = [0.5 * (g + _at(g, 1, 0)) for g in gc]
        uf = [0.5 * (vel[0] + _at(vel[0], 1, 0)), 0.5 * (vel[1] + _at(vel[1], 1, 0))]
        fx, fy, en = _viscous_flux_curv(P, (sxe, sye), (dxe, dye), 0.5 * (T + _at(T, 1, 0)), dn[:2], dt[:2], dn[2],
                                        dt[2], uf, -1)
        Fh = [Fh[0], Fh[1] - fx, Fh[2] - fy, Fh[3] - en]
    out = torch.stack([(_at(Fh[m], -1, 0) - Fh[m]) * inva for m in range(P.nvar)])
    # j direction: faces 1/2 .. ny - 3/2 between rows j and j + 1
    q = [r] + list(vel) + [p]
    if P.recon == FIRST_ORDER:
        qL = [a[:-1] for a in q]
        qR = [a[1:] for a in q]
    else:
        qL, qR = [], []
        zero = torch.zeros_like(r[:1])
        for a in q:
            a0, ap1 = a[:-1], a[1:]
            sl = torch.cat([zero, _minmod(a[1:-1] - a[:-2], a[2:] - a[1:-1])])       # row 0: no slope
            sr = torch.cat([_minmod(a[1:-1] - a[:-2], a[2:] - a[1:-1]), zero])       # row ny-1: no slope
            qL.append(a0 + 0.5 * sl)
            qR.append(ap1 - 0.5 * sr)
    rL, vL, pL = qL[0], qL[1:3], qL[3]
    rR, vR, pR = qR[0], qR[1:3], qR[3]
    if P.recon == FIRST_ORDER:
        ULc = [u[:-1] for u in U]
        URc = [u[1:] for u in U]
    else:
        ULc = conserved(P, rL, vL, pL)
        URc = conserved(P, rR, vR, pR)
    Fi = _rotated_flux(P, ULc, rL, vL, pL, URc, rR, vR, pR, sxn[:-1], syn[:-1])
    if ns:
        dn = [a[1:] - a[:-1] for a in phis]
        gc = [(_at(a, 1, 0) - _at(a, -1, 0)) * 0.5 for a in phis]
        dt = [0.5 * (g[:-1] + g[1:]) for g in gc]
        uf = [0.5 * (vel[0][:-1] + vel[0][1:]), 0.5 * (vel[1][:-1] + vel[1][1:])]
        fx, fy, en = _viscous_flux_curv(P, (sxn[:-1], syn[:-1]), (dxn[:-1], dyn[:-1]), 0.5 * (T[:-1] + T[1:]), dn[:2],
                                        dt[:2], dn[2], dt[2], uf, 1)
        Fi = [Fi[0], Fi[1] - fx, Fi[2] - fy, Fi[3] - en]
    # wall and far field
    zw = torch.zeros_like(wx)
    Fw = [zw, p[0] * wx, p[0] * wy, zw]
    if ns:
        tw = P.t_wall
        fx, fy, en = _viscous_flux_curv(P, (wx, wy), (awx, awy), 0.5 * (T[0] + tw),
                                        [vel[0][0] - 0.0, vel[1][0] - 0.0], [zw, zw], T[0] - tw, zw, [zw, zw], 1)
        Fw = [Fw[0], Fw[1] - fx, Fw[2] - fy, Fw[3] - en]
    Uf = [torch.full_like(r[-1], float(v)) for v in P.farfield]
    rf, vf, pf = primitives(P, Uf)
    vb = [v[-1] for v in vel]
    Ub = conserved(P, r[-1], vb, p[-1])          # from the last cell's primitive state
    Ff = _rotated_flux(P, Ub, r[-1], vb, p[-1], Uf, rf, vf, pf, sxn[-1], syn[-1])
    Fj = [torch.cat([Fw[m][None], Fi[m], Ff[m][None]]) for m in range(P.nvar)]    # faces j - 1/2, j = 0..ny
    out = out + torch.stack([(Fj[m][:-1] - Fj[m][1:]) * inva for m in range(P.nvar)])
    return out.reshape(-1)


def _viscous_flux_curv(P: Problem, S, dc, mu_T, un, ut, Tn, Tt, uf, sign):
    """Viscous flux through a curvilinear face with face vector S = (Sx, Sy) and
    centroid difference dc across it, from index-space derivatives across the
    face (un = (u_n, v_n), Tn) and along it (ut, Tt): with J = dc . S,
    grad phi = (phi_n S -+ phi_t (dcy, -dcx)) / J (sign = -1 across i, +1 across
    j: the chain rule through the face's two grid directions).  mu_T: the face
    temperature for Sutherland's law.  uf: face velocity.  Returns
    (F_v . S) for momentum x, y and energy."""
    Sx, Sy = S
    dcx, dcy = dc
    J = dcx * Sx + dcy * Sy
    if sign < 0:
        grad = lambda n, t: ((n * Sx - t * dcy) / J, (n * Sy + t * dcx) / J)
    else:
        grad = lambda n, t: ((n * Sx + t * dcy) / J, (n * Sy - t * dcx) / J)
    ux, uy = grad(un[0], ut[0])
    vx, vy = grad(un[1], ut[1])
    Tx, Ty = grad(Tn, Tt)
    mu = sutherland_mu(P, mu_T) if P.sutherland > 0.0 else P.mu
    c23 = (2.0 / 3.0) * mu
    kap = mu * P.gamma / ((P.gamma - 1.0) * P.prandtl)
    div = ux + vy
    txx = mu * (ux + ux) - c23 * div
    tyy = mu * (vy + vy) - c23 * div
    txy = mu * (uy + vx)
    fx = txx * Sx + txy * Sy
    fy = txy * Sx + tyy * Sy
    en = (uf[0] * txx + uf[1] * txy + kap * Tx) * Sx + (uf[0] * txy + uf[1] * tyy + kap * Ty) * Sy
    return fx, fy, en


def _residual_curvilinear(P: Problem, y: torch.Tensor) -> torch.Tensor:
    """f on a 2-D curvilinear periodic grid (Euler physics): reconstruction in
    index space as on the Cartesian grid, then at each face the states are
    rotated into the face frame (n = S/|S|: normal and tangential momentum and
    velocity), the one-dimensional numerical flux is taken there, rotated back
    and scaled by the face length; f_c = sum_d (Fhat_{c-1/2} - Fhat_{c+1/2}) / A_c."""
    if P.ndim != 2:
        raise ValueError("curvilinear grids: 2-D only")
    U = y.reshape(P.shape)
    U = [U[m] for m in range(P.nvar)]
    r, vel, p = primitives(P, U)
    sxe, sye, sxn, syn, inva, dxe, dye, dxn, dyn = metrics(P)
    T = p / r
    out = None
    for d in range(2):
        (UL, rL, vL, pL), (UR, rR, vR, pR) = _face_states(P, U, r, vel, p, d)
        sx, sy = (sxe, sye) if d == 0 else (sxn, syn)
        ln = _sqrt(sx * sx + sy * sy)
        nx = sx / ln
        ny = sy / ln
        vLr = [vL[0] * nx + vL[1] * ny, vL[1] * nx - vL[0] * ny]
        vRr = [vR[0] * nx + vR[1] * ny, vR[1] * nx - vR[0] * ny]
        ULr = [UL[0], UL[1] * nx + UL[2] * ny, UL[2] * nx - UL[1] * ny, UL[3]]
        URr = [UR[0], UR[1] * nx + UR[2] * ny, UR[2] * nx - UR[1] * ny, UR[3]]
        Fr = face_flux(P, ULr, rL, vLr, pL, URr, rR, vRr, pR, 0)
        Fh = [Fr[0] * ln, (Fr[1] * nx - Fr[2] * ny) * ln, (Fr[1] * ny + Fr[2] * nx) * ln, Fr[3] * ln]
        if P.physics == NS:
            t = 1 - d                      # the grid direction along the face
            phis = [vel[0], vel[1], T]
            dn = [_at(a, 1, d) - a for a in phis]
            gc = [(_at(a, 1, t) - _at(a, -1, t)) * 0.5 for a in phis]
            dt = [0.5 * (g + _at(g, 1, d)) for g in gc]
            uf = [0.5 * (vel[0] + _at(vel[0], 1, d)), 0.5 * (vel[1] + _at(vel[1], 1, d))]
            dc = (dxe, dye) if d == 0 else (dxn, dyn)
            fx, fy, en = _viscous_flux_curv(P, (sx, sy), dc, 0.5 * (T + _at(T, 1, d)), dn[:2], dt[:2], dn[2], dt[2],
                                            uf, -1 if d == 0 else 1)
            Fh = [Fh[0], Fh[1] - fx, Fh[2] - fy, Fh[3] - en]
        term = torch.stack([(_at(Fh[m], -1, d) - Fh[m]) * inva for m in range(P.nvar)])
        out = term if out is None else out + term
    return out.reshape(-1)


def residual(P: Problem, y: torch.Tensor, part: str = "all", terms: list | None = None) -> torch.Tensor:
    """f(y) for a flat state vector y of length P.size (float64).

    part = "inviscid" or "viscous" assembles f from that flux alone (the
    split output of the residual: the two parts add up to f).  terms: if a
    list is given (Cartesian grids), each direction's flux difference
    (F_{c-1/2} - F_{c+1/2}) / dx_d is appended to it, flat; f is their sum in
    direction order."""
    if part not in ("all", "inviscid", "viscous"):
        raise ValueError(f"unknown part {part!r}")
    if P.nodes is not None:
        if part != "all":
            raise ValueError("curvilinear grids: the whole residual only")
        if P.farfield is not None:
            return _residual_ogrid(P, y)
        return _residual_curvilinear(P, y)
    U = y.reshape(P.shape)
    U = [U[m] for m in range(P.nvar)]
    r, vel, p = primitives(P, U)
    out = None
    for d in range(P.ndim):
        if _BRANCHES is not None:
            _BRANCHES.axis = d
        (UL, rL, vL, pL), (UR, rR, vR, pR) = _face_states(P, U, r, vel, p, d)
        if part == "viscous":
            Fh = [torch.zeros_like(r) for _ in range(P.nvar)]
        else:
            Fh = face_flux(P, UL, rL, vL, pL, UR, rR, vR, pR, d)
        if P.physics not in (EULER, NS):
            raise ValueError(f"unknown physics {P.physics!r}")
        if P.physics == NS and part != "inviscid":
            Fv = _viscous_flux(P, r, vel, p, d)
            Fh = [Fh[m] - Fv[m] for m in range(P.nvar)]
        inv = P.invdx(d)
        term = torch.stack([(_at(Fh[m], -1, d) - Fh[m]) * inv for m in range(P.nvar)])
        if terms is not None:
            terms.append(term.reshape(-1))
        out = term if out is None else out + term
    return out.reshape(-1)


def cells_near_switches(P: Problem, y: torch.Tensor, delta: float) -> torch.Tensor:
    """Cells (a boolean tensor of the grid's shape) whose value of f contains a
    face flux with a branch decision closer than delta to its switch: both
    cells c and c + 1 of such a face c + 1/2 (Cartesian grids)."""
    with branches(record=True) as br:
        residual(P, y)
    mask = torch.zeros(P.shape[1:], dtype=torch.bool)
    for site, (_, m) in br.margins.items():
        near = m < delta
        if bool(near.any()):
            mask |= near | _at(near, -1, br.axes[site])
    return mask


def residual_terms(P: Problem, y: torch.Tensor) -> torch.Tensor:
    """The D per-direction flux differences whose sum (in direction order) is f(y), as a (D, N) tensor."""
    terms = []
    residual(P, y, terms=terms)
    return torch.stack(terms)


# ---------------------------------------------------------------------------
# Jacobian-vector products (Sec. 2.3)
# ---------------------------------------------------------------------------

EPS_MACH = 2.0 ** -52


def fd_epsilon(y: torch.Tensor, v: torch.Tensor) -> float:
    """Default finite-difference increment: sqrt((1 + ||y||) eps_mach) / ||v||.

    The paper defers the choice of epsilon to the literature on Jacobian-free
    Newton-Krylov methods (Sec. 2.3).  Of the two usual rules, this one and
    sqrt(eps_mach) (1 + ||y||) / ||v|| (a per-entry perturbation of about
    sqrt(eps_mach) times the size of y), this one gives the smaller error
    against the exact product on the seeded workloads at their sizes: f is
    only piecewise smooth, and the larger perturbation crosses more switches
    of minmod and of the wave-speed maximum.  Operation order: the sum, its
    product with eps_mach (exact), a correctly rounded square root, then the
    division.
    """
    from .krylov import dot
    ny = math.sqrt(dot(y, y))
    nv = math.sqrt(dot(v, v))
    return math.sqrt((1.0 + ny) * EPS_MACH) / nv


def jvp_fd(P: Problem, y, fy, v, eps: float):
    """First-order finite-difference J(y) v = (f(y + eps v) - f(y)) / eps (Sec. 2.3, eq. 10)."""
    return (residual(P, y + eps * v) - fy) / eps


def jvp_exact(P: Problem, y, v):
    """Exact J(y) v: forward-mode derivative of residual() (Sec. 2.3, exact products)."""
    _, t = torch.func.jvp(lambda z: residual(P, z), (y,), (v,))
    return t


def vjp(P: Problem, y, wbar):
    """Adjoint product J(y)^T wbar, by reverse-mode differentiation of residual()."""
    z = y.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(residual(P, z), z, wbar)
    return g


def vjp_second(P: Problem, y, v, wbar):
    """Second-order adjoint d/dt [J(y + t v)^T wbar] at t = 0 (forward-over-reverse)."""
    _, t = torch.func.jvp(lambda z: vjp_fn(P, z, wbar), (y,), (v,))
    return t


def vjp_fn(P: Problem, y, wbar):
    _, pull = torch.func.vjp(lambda z: residual(P, z), y)
    return pull(wbar)[0]


def dense_jacobian_fd(P: Problem, y, delta: float = 1e-6):
    """Brute-force Jacobian by column-wise central differences (tiny grids only)."""
    N = y.numel()
    J = torch.empty(N, N, dtype=torch.float64)
    for c in range(N):
        e = torch.zeros(N, dtype=torch.float64)
        e[c] = delta
        J[:, c] = (residual(P, y + e) - residual(P, y - e)) / (2.0 * delta)
    return J
