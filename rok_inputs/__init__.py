"""Seeded synthetic inputs shared by the GPU tests, the benchmark and the oracle tests.

This module holds initial conditions, problem descriptions, time-step sizes
and stored ROK coefficient tables.  It contains none of the method's
arithmetic (no residual, product, Arnoldi or ROK step).  Everything it returns
is plain numpy / Python data that both the GPU library and the CPU oracle
take as input.

Workloads (periodic synthetic flows standing in for the paper's cylinder and
aerofoil meshes, which are not available):

* ``vortex_2d``   isentropic vortex, strength 5, free stream Mach 0.5 along the
                  diagonal, on [-5, 5]^2 (gamma = 1.4);
* ``tgv_2d``      2-D Taylor-Green vortex on [0, 2 pi]^2, Mach 0.1, Re 100;
* ``tgv_3d``      3-D Taylor-Green vortex on [0, 2 pi]^3, Mach 0.1, Re 1600.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

GAMMA = 1.4
PERTURB_SEED = 20160726


def problem(n, lo, hi, physics="euler", recon="first", gamma=GAMMA, mu=0.0, prandtl=0.72, flux="rusanov",
            sutherland=0.0, t_ref=1.0):
    """Plain description of f: grid, physics and discretisation (sutherland = S / T_ref,
    0 for a constant viscosity)."""
    return {"n": tuple(int(x) for x in n), "lo": tuple(float(x) for x in lo),
            "hi": tuple(float(x) for x in hi), "physics": physics, "recon": recon,
            "gamma": float(gamma), "mu": float(mu), "prandtl": float(prandtl), "flux": flux,
            "sutherland": float(sutherland), "t_ref": float(t_ref)}


def size(pb) -> int:
    return (len(pb["n"]) + 2) * int(np.prod(pb["n"]))


def _centres(pb, d):
    n, lo, hi = pb["n"][d], pb["lo"][d], pb["hi"][d]
    dx = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * dx


def _mesh(pb):
    cs = [_centres(pb, d) for d in range(len(pb["n"]))]
    # arrays indexed [z][y][x] (x fastest)
    return np.meshgrid(*reversed(cs), indexing="ij")[::-1]


def _pack(pb, rho, vel, p):
    g = pb["gamma"]
    ke = sum(u * u for u in vel)
    E = p / (g - 1.0) + 0.5 * rho * ke
    return np.stack([rho] + [rho * u for u in vel] + [E]).reshape(-1).astype(np.float64)


# ---------------------------------------------------------------------------
# Curvilinear (mapped) periodic grids, 2-D
# ---------------------------------------------------------------------------

def warped_nodes(pb, amplitude=0.06):
    """Node coordinates (x, y), arrays indexed [j][i] (node i along x, j along y),
    of a smoothly warped periodic grid on the problem's box:
    x = X + a Lx sin(2 pi (Y - lo_y) / Ly),  y = Y + a Ly sin(2 pi (X - lo_x) / Lx),
    (X, Y) the Cartesian node positions.  Periodic: node (i + nx, j) is node
    (i, j) shifted by (Lx, 0), node (i, j + ny) by (0, Ly).  The mapping is
    one-to-one for 2 pi a < 1."""
    nx, ny = pb["n"][:2]
    lo, hi = pb["lo"], pb["hi"]
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    X, Y = np.meshgrid(lo[0] + np.arange(nx) * (Lx / nx), lo[1] + np.arange(ny) * (Ly / ny))
    x = X + amplitude * Lx * np.sin(2.0 * math.pi * (Y - lo[1]) / Ly)
    y = Y + amplitude * Ly * np.sin(2.0 * math.pi * (X - lo[0]) / Lx)
    return x.astype(np.float64), y.astype(np.float64)


def cartesian_nodes(pb):
    """The nodes of the problem's uniform Cartesian grid in the same layout."""
    return warped_nodes(pb, 0.0)


def cylinder_ogrid(nx, ny, radius=0.5, far=10.0, recon="first", flux="rusanov", cluster=None):
    """O-grid around a circular cylinder: nodes x(i, j), y(i, j) (arrays [j][i],
    j = 0..ny) at angle -2 pi i / nx (clockwise, so that (i, j) is right-handed)
    and radius r_j = radius q^j growing geometrically to `far`, or, with
    cluster = beta, r_j = radius + (far - radius)(e^{beta j / ny} - 1)/(e^beta - 1)
    (very thin cells at the wall, as on viscous meshes).  Returns (problem with
    n = (nx, ny), (x, y))."""
    if cluster is None:
        q = (far / radius) ** (1.0 / ny)
        rj = radius * q ** np.arange(ny + 1)
    else:
        rj = radius + (far - radius) * np.expm1(cluster * np.arange(ny + 1) / ny) / np.expm1(cluster)
    th = -2.0 * math.pi * np.arange(nx) / nx
    x = rj[:, None] * np.cos(th)[None, :]
    y = rj[:, None] * np.sin(th)[None, :]
    pb = problem((nx, ny), (0.0, 0.0), (1.0, 1.0), "euler", recon, flux=flux)
    return pb, (x.astype(np.float64), y.astype(np.float64))


def ogrid_centres(xn, yn):
    """Cell centres of an O-grid (mean of the four nodes; i periodic, no offset)."""
    r1 = lambda a: np.roll(a, -1, axis=1)
    return (0.25 * (xn[:-1] + r1(xn)[:-1] + r1(xn)[1:] + xn[1:]),
            0.25 * (yn[:-1] + r1(yn)[:-1] + r1(yn)[1:] + yn[1:]))


def freestream(gamma=GAMMA, mach=0.3, rho=1.0, p=1.0, angle=0.0):
    """Conserved free-stream state (rho, rho u, rho v, E) at the given Mach number."""
    c = math.sqrt(gamma * p / rho)
    u, v = mach * c * math.cos(angle), mach * c * math.sin(angle)
    return (rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v))


def node_centres(pb, xn, yn):
    """Cell centres (mean of the four nodes, periodic offsets applied)."""
    Lx, Ly = pb["hi"][0] - pb["lo"][0], pb["hi"][1] - pb["lo"][1]
    x1 = np.roll(xn, -1, axis=1); x1[:, -1] += Lx
    y2 = np.roll(yn, -1, axis=0); y2[-1, :] += Ly
    x3 = np.roll(x1, -1, axis=0)
    y3 = np.roll(yn, -1, axis=1); y3 = np.roll(y3, -1, axis=0); y3[-1, :] += Ly
    x2 = np.roll(xn, -1, axis=0)
    y1 = np.roll(yn, -1, axis=1)
    return 0.25 * (xn + x1 + x2 + x3), 0.25 * (yn + y1 + y2 + y3)


# ---------------------------------------------------------------------------
# Isentropic vortex
# ---------------------------------------------------------------------------

def vortex_problem(n, recon="first"):
    return problem((n, n), (-5.0, -5.0), (5.0, 5.0), "euler", recon)


def vortex_freestream(gamma=GAMMA, mach=0.5):
    """Free-stream velocity of Mach `mach` along the diagonal (rho = p = 1)."""
    speed = mach * math.sqrt(gamma)
    return speed / math.sqrt(2.0), speed / math.sqrt(2.0)


def vortex_state(pb, t=0.0, strength=5.0, mach=0.5, centres=None):
    """Vortex centred at the origin at t = 0, translated by the free stream
    (minimum-image periodic displacement).  At t > 0 this is the exact
    solution of the Euler equations up to the periodic Gaussian tail.
    centres: optional (x, y) cell centres of a curvilinear grid."""
    g = pb["gamma"]
    x, y = _mesh(pb) if centres is None else centres
    uinf, vinf = vortex_freestream(g, mach)
    Lx = pb["hi"][0] - pb["lo"][0]
    Ly = pb["hi"][1] - pb["lo"][1]
    dx = x - uinf * t
    dy = y - vinf * t
    dx = dx - Lx * np.round(dx / Lx)
    dy = dy - Ly * np.round(dy / Ly)
    r2 = dx * dx + dy * dy
    e = np.exp(0.5 * (1.0 - r2))
    du = -strength / (2.0 * math.pi) * dy * e
    dv = strength / (2.0 * math.pi) * dx * e
    T = 1.0 - (g - 1.0) * strength**2 / (8.0 * g * math.pi**2) * e * e
    rho = T ** (1.0 / (g - 1.0))
    p = rho * T
    return _pack(pb, rho, [uinf + du, vinf + dv], p)


def perturb_density(pb, y, amplitude=0.01, seed=PERTURB_SEED):
    """rho <- rho (1 + amplitude xi), xi ~ U(-1, 1) per cell; u and p kept."""
    g = pb["gamma"]
    D = len(pb["n"])
    U = y.reshape((D + 2,) + tuple(reversed(pb["n"])))
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(D)]
    ke = sum(u * u for u in vel)
    p = (g - 1.0) * (U[D + 1] - 0.5 * rho * ke)
    xi = np.random.default_rng(seed).uniform(-1.0, 1.0, size=rho.shape)
    return _pack(pb, rho * (1.0 + amplitude * xi), vel, p)


def perturb_generic(pb, y, amplitude=1e-3, seed=PERTURB_SEED + 1):
    """Seeded perturbation of every primitive variable (relative to its spread):
    rho, each velocity component and p get amplitude * (spread) * xi, xi ~ U(-1, 1)
    per cell.  Breaks the exact symmetries of the analytic initial states, at
    whose mirror-image cells minmod and the wave-speed maximum sit on ties."""
    g = pb["gamma"]
    D = len(pb["n"])
    U = y.reshape((D + 2,) + tuple(reversed(pb["n"])))
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(D)]
    ke = sum(u * u for u in vel)
    p = (g - 1.0) * (U[D + 1] - 0.5 * rho * ke)
    rng = np.random.default_rng(seed)

    def bump(q):
        spread = float(np.max(q) - np.min(q)) or float(np.max(np.abs(q))) or 1.0
        return q + amplitude * spread * rng.uniform(-1.0, 1.0, size=q.shape)

    return _pack(pb, bump(rho), [bump(u) for u in vel], bump(p))


# ---------------------------------------------------------------------------
# Taylor-Green vortices
# ---------------------------------------------------------------------------

def tgv_problem(n, ndim=2, reynolds=None, recon="muscl"):
    if reynolds is None:
        reynolds = 100.0 if ndim == 2 else 1600.0
    L = 2.0 * math.pi
    return problem((n,) * ndim, (0.0,) * ndim, (L,) * ndim, "ns", recon, mu=1.0 / reynolds)


def tgv_state(pb, mach=0.1):
    g = pb["gamma"]
    p0 = 1.0 / (g * mach * mach)
    if len(pb["n"]) == 2:
        x, y = _mesh(pb)
        u = np.sin(x) * np.cos(y)
        v = -np.cos(x) * np.sin(y)
        p = p0 + 0.25 * (np.cos(2 * x) + np.cos(2 * y))
        return _pack(pb, np.ones_like(x), [u, v], p)
    x, y, z = _mesh(pb)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    return _pack(pb, np.ones_like(x), [u, v, w], p)


# ---------------------------------------------------------------------------
# Generic seeded states and directions
# ---------------------------------------------------------------------------

def smooth_random_state(pb, seed, amplitude=0.05):
    """A positive, smooth-ish random flow: uniform state plus seeded Fourier modes."""
    rng = np.random.default_rng(seed)
    g = pb["gamma"]
    D = len(pb["n"])
    X = _mesh(pb)
    L = [pb["hi"][d] - pb["lo"][d] for d in range(D)]

    def field():
        acc = np.zeros_like(X[0])
        for _ in range(3):
            k = [rng.integers(1, 3) for _ in range(D)]
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(2 * math.pi * k[d] * X[d] / L[d] for d in range(D)) + ph
            acc = acc + rng.uniform(0.5, 1.0) * np.sin(arg)
        return acc

    rho = 1.0 + amplitude * field()
    vel = [0.3 * (d + 1) / D + amplitude * field() for d in range(D)]
    p = 1.0 / g + amplitude * field()
    noise = rng.uniform(-1, 1, size=(3,) + rho.shape) * amplitude * 0.1
    return _pack(pb, rho * (1 + noise[0]), vel, p * (1 + noise[1]))


def random_direction(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    return scale * v / np.linalg.norm(v)


def uniform_state(pb, rho=1.0, vel=None, p=1.0):
    D = len(pb["n"])
    shape = tuple(reversed(pb["n"]))
    vel = vel if vel is not None else [0.3] * D
    return _pack(pb, np.full(shape, rho), [np.full(shape, u) for u in vel], np.full(shape, p))


# ---------------------------------------------------------------------------
# Step size
# ---------------------------------------------------------------------------

def spectral_estimate(pb, y) -> float:
    """rho_est = max sum_d (|u_d| + c)/dx_d + max(nu_eff) 4 sum_d dx_d^-2,
    nu_eff = max(4/3, gamma/Pr) mu/rho (0 for Euler)."""
    g = pb["gamma"]
    D = len(pb["n"])
    U = y.reshape((D + 2,) + tuple(reversed(pb["n"])))
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(D)]
    ke = sum(u * u for u in vel)
    p = (g - 1.0) * (U[D + 1] - 0.5 * rho * ke)
    c = np.sqrt(g * p / rho)
    dxs = [(pb["hi"][d] - pb["lo"][d]) / pb["n"][d] for d in range(D)]
    acoustic = sum((np.abs(vel[d]) + c) / dxs[d] for d in range(D)).max()
    visc = 0.0
    if pb["physics"] == "ns" and pb["mu"] > 0:
        nu = max(4.0 / 3.0, g / pb["prandtl"]) * pb["mu"] / rho
        visc = float(nu.max()) * 4.0 * sum(1.0 / dx**2 for dx in dxs)
    return float(acoustic + visc)


def cfl_step(pb, y, cfl) -> float:
    """Fixed step size h = CFL / rho_est, from the initial state."""
    return cfl / spectral_estimate(pb, y)


# ---------------------------------------------------------------------------
# ROK coefficient tables (derived from the order conditions; see the JSON notes)
# ---------------------------------------------------------------------------

def _table(name):
    with open(os.path.join(_HERE, name)) as fh:
        t = json.load(fh)
    return {k: t[k] for k in ("s", "alpha", "gam", "gamma", "b")}


def rok4_tableau():
    return _table("rok4_tableau.json")


def ros4_only_tableau():
    return _table("ros4_only_tableau.json")


def rk4_tableau():
    """Classical RK4 as a ROK table (only meaningful with M = 0)."""
    return {"s": 4, "gamma": 0.5,
            "alpha": [[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]],
            "gam": [[0.0] * 4 for _ in range(4)], "b": [1 / 6, 1 / 3, 1 / 3, 1 / 6]}


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

WORKLOADS = {
    "vortex32_fo": dict(kind="vortex", n=32, recon="first", M=8, steps=10, cfl=5.0, jvp="fd", precision="fp64"),
    "vortex1024_muscl": dict(kind="vortex", n=1024, recon="muscl", M=16, steps=100, cfl=10.0, jvp="fd", precision="fp64"),
    "tgv2048_ns": dict(kind="tgv2", n=2048, recon="muscl", M=20, steps=20, cfl=50.0, jvp="exact", precision="fp32"),
    "vortex512_adjoint": dict(kind="vortex", n=512, recon="first", M=16, steps=50, cfl=2.0, jvp="exact", precision="fp64",
                              perturb=True),
    "tgv256_3d": dict(kind="tgv3", n=256, recon="muscl", M=16, steps=20, cfl=10.0, jvp="exact", precision="fp32"),
    "tgv256_3d_fp64": dict(kind="tgv3", n=256, recon="muscl", M=16, steps=20, cfl=10.0, jvp="fd", precision="fp64"),
}


def workload(name, n=None):
    """(problem, initial state, settings) of a named workload, optionally at another size n."""
    w = dict(WORKLOADS[name])
    n = n or w["n"]
    if w["kind"] == "vortex":
        pb = vortex_problem(n, w["recon"])
        y0 = vortex_state(pb)
    elif w["kind"] == "tgv2":
        pb = tgv_problem(n, 2)
        y0 = tgv_state(pb)
    else:
        pb = tgv_problem(n, 3)
        y0 = tgv_state(pb)
    if w.get("perturb"):
        y0 = perturb_density(pb, y0)
    return pb, y0, w
