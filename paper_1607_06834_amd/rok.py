"""Python binding of librok (argument marshalling only).

Every computation runs in the HIP kernels of librok.so; this module converts
torch device tensors to pointers, owns the workspace tensors and forwards
the current torch stream.  If the library is missing the calls raise: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librok.so")

ROK_OK, ROK_EINVAL, ROK_EUNSUPPORTED, ROK_EHIP = 0, -1, -2, -3
EULER, NS = 0, 1
FIRST_ORDER, MUSCL_MINMOD = 0, 1
RUSANOV, ROE = 0, 1
FP64, FP32_RESIDUAL = 0, 1
JVP_FD, JVP_TANGENT = 0, 1
FLAG_NONFINITE, FLAG_BREAKDOWN, FLAG_ZERO_RHS, FLAG_BARRIER, FLAG_NONPHYSICAL = 1, 2, 4, 8, 16
MAX_STAGES, MAX_M = 8, 64

SYMBOLS = ["rok_create", "rok_destroy", "rok_set_mgs_path", "rok_arnoldi_path", "rok_state_size", "rok_workspace_bytes", "rok_residual", "rok_residual_split",
           "rok_jvp", "rok_jvp_noalloc", "rok_arnoldi", "rok_step", "rok_residual_vjp", "rok_residual_vjp2", "rok_step_vjp",
           "rok_step_vjp_workspace_bytes", "rok_step_vjp_stored", "rok_step_vjp_adjoint_bytes", "rok_mgs_column",
           "rok_eigs", "rok_eigs_workspace_bytes", "rok_set_grid", "rok_grid_metric_bytes", "rok_set_ogrid",
           "rok_ogrid_metric_bytes", "rok_error_norm", "rok_integrate_adaptive", "rok_adaptive_workspace_bytes", "rok_workspace_init", "rok_read_status", "rok_read_meff", "rok_strerror"]
MGS_PATHS = {"auto": 0, "pass": 1, "resident": 2, "one_reduce": 3}


class RokProblem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("physics", ctypes.c_int), ("recon", ctypes.c_int),
                ("flux", ctypes.c_int), ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("prandtl", ctypes.c_double), ("precision", ctypes.c_int), ("sutherland", ctypes.c_double),
                ("t_ref", ctypes.c_double)]


class RokTableau(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("alpha", ctypes.c_double * (MAX_STAGES * MAX_STAGES)),
                ("gam", ctypes.c_double * (MAX_STAGES * MAX_STAGES)), ("gamma", ctypes.c_double),
                ("b", ctypes.c_double * MAX_STAGES)]


class RokAdaptiveStats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h_next", ctypes.c_double), ("accepted", ctypes.c_int),
                ("rejected", ctypes.c_int), ("recorded", ctypes.c_int)]


class RokError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librok.so (built by paper_1607_06834_amd.build) and declare its C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RokError(f"{path} is missing: build it with `python -m paper_1607_06834_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.rok_create.argtypes = [ctypes.POINTER(RokProblem), ctypes.POINTER(vp)]
    lib.rok_create.restype = i
    lib.rok_destroy.argtypes = [vp]
    lib.rok_destroy.restype = None
    lib.rok_set_mgs_path.argtypes = [vp, i]
    lib.rok_set_mgs_path.restype = i
    lib.rok_arnoldi_path.argtypes = [vp, i]
    lib.rok_arnoldi_path.restype = i
    lib.rok_state_size.argtypes = [vp]
    lib.rok_state_size.restype = sz
    lib.rok_workspace_bytes.argtypes = [vp, i, i]
    lib.rok_workspace_bytes.restype = sz
    lib.rok_residual.argtypes = [vp, vp, vp, vp]
    lib.rok_residual.restype = i
    lib.rok_residual_split.argtypes = [vp, vp, vp, vp, vp]
    lib.rok_residual_split.restype = i
    lib.rok_jvp.argtypes = [vp, vp, vp, vp, vp, i, d, vp, sz, vp]
    lib.rok_jvp.restype = i
    lib.rok_jvp_noalloc.argtypes = [vp, vp, vp, vp, vp, i, d, vp]
    lib.rok_jvp_noalloc.restype = i
    lib.rok_arnoldi.argtypes = [vp, vp, vp, i, i, d, vp, vp, vp, vp, sz, vp]
    lib.rok_arnoldi.restype = i
    lib.rok_step.argtypes = [vp, ctypes.POINTER(RokTableau), i, i, d, vp, vp, vp, sz, vp]
    lib.rok_step.restype = i
    lib.rok_residual_vjp.argtypes = [vp, vp, vp, vp, i, vp]
    lib.rok_residual_vjp.restype = i
    lib.rok_residual_vjp2.argtypes = [vp, vp, vp, vp, vp, vp, i, vp]
    lib.rok_residual_vjp2.restype = i
    lib.rok_step_vjp.argtypes = [vp, ctypes.POINTER(RokTableau), i, d, vp, vp, vp, vp, vp, sz, vp]
    lib.rok_step_vjp.restype = i
    lib.rok_step_vjp_workspace_bytes.argtypes = [vp, i, i]
    lib.rok_step_vjp_workspace_bytes.restype = sz
    lib.rok_step_vjp_stored.argtypes = [vp, ctypes.POINTER(RokTableau), i, d, vp, vp, vp, vp, sz, vp, sz, vp]
    lib.rok_step_vjp_stored.restype = i
    lib.rok_step_vjp_adjoint_bytes.argtypes = [vp, i, i]
    lib.rok_step_vjp_adjoint_bytes.restype = sz
    pd, pi = ctypes.POINTER(d), ctypes.POINTER(i)
    lib.rok_set_grid.argtypes = [vp, vp, vp, vp, vp]
    lib.rok_set_grid.restype = i
    lib.rok_grid_metric_bytes.argtypes = [vp]
    lib.rok_grid_metric_bytes.restype = sz
    lib.rok_set_ogrid.argtypes = [vp, vp, vp, pd, d, vp, vp]
    lib.rok_set_ogrid.restype = i
    lib.rok_ogrid_metric_bytes.argtypes = [vp]
    lib.rok_ogrid_metric_bytes.restype = sz
    lib.rok_eigs.argtypes = [vp, vp, vp, i, i, i, d, pd, pd, pd, pi, vp, sz, vp]
    lib.rok_eigs.restype = i
    lib.rok_eigs_workspace_bytes.argtypes = [vp, i, i]
    lib.rok_eigs_workspace_bytes.restype = sz
    lib.rok_error_norm.argtypes = [vp, vp, vp, vp, d, d, d, vp, vp, sz, vp]
    lib.rok_error_norm.restype = i
    lib.rok_integrate_adaptive.argtypes = [vp, ctypes.POINTER(RokTableau), i, i, i, d, d, d, d, i, vp,
                                           ctypes.POINTER(RokAdaptiveStats), ctypes.POINTER(d), i, vp, sz, vp]
    lib.rok_integrate_adaptive.restype = i
    lib.rok_adaptive_workspace_bytes.argtypes = [vp, i, i]
    lib.rok_adaptive_workspace_bytes.restype = sz
    lib.rok_mgs_column.argtypes = [vp, vp, i, i, vp, vp, vp, vp, sz, vp]
    lib.rok_mgs_column.restype = i
    lib.rok_workspace_init.argtypes = [vp, vp, sz, i, i, vp]
    lib.rok_workspace_init.restype = i
    lib.rok_read_status.argtypes = [vp, vp, ctypes.POINTER(i), vp]
    lib.rok_read_status.restype = i
    lib.rok_read_meff.argtypes = [vp, vp, ctypes.POINTER(i), vp]
    lib.rok_read_meff.restype = i
    lib.rok_strerror.argtypes = [i]
    lib.rok_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != ROK_OK:
        msg = _lib.rok_strerror(status).decode()
        raise RokError(f"{what} failed: {msg} ({status})")


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_tableau(tab: dict) -> RokTableau:
    s = int(tab["s"])
    if not 1 <= s <= MAX_STAGES:
        raise ValueError("1 <= s <= 8 stages")
    t = RokTableau()
    t.s = s
    t.gamma = float(tab["gamma"])
    for i in range(s):
        t.b[i] = float(tab["b"][i])
        for j in range(i):
            t.alpha[i * MAX_STAGES + j] = float(tab["alpha"][i][j])
            t.gam[i * MAX_STAGES + j] = float(tab["gam"][i][j])
    return t


class ForwardRecord:
    """An exact-product step kept for Rok.step_vjp_stored: the state y_n (held,
    not copied: it must not change) and the step's own forward workspace."""
    __slots__ = ("y", "h", "tableau", "M", "ws")

    def __init__(self, y, h, tableau, M, ws):
        self.y, self.h, self.tableau, self.M, self.ws = y, h, tableau, M, ws


class Rok:
    """One problem (grid, physics, discretisation, precision) on the current GPU."""

    def __init__(self, problem: dict, precision: str = "fp64", mgs: str = "auto"):
        lib = load_library()
        p = RokProblem()
        self._n = tuple(int(v) for v in problem["n"])
        D = len(problem["n"])
        p.ndim = D
        for d in range(3):
            p.n[d] = int(problem["n"][d]) if d < D else 1
            p.lo[d] = float(problem["lo"][d]) if d < D else 0.0
            p.hi[d] = float(problem["hi"][d]) if d < D else 1.0
        p.physics = NS if problem["physics"] == "ns" else EULER
        p.recon = MUSCL_MINMOD if problem["recon"] == "muscl" else FIRST_ORDER
        p.flux = {"rusanov": RUSANOV, "roe": ROE}[problem.get("flux", "rusanov")]
        p.gamma = float(problem["gamma"])
        p.mu = float(problem.get("mu", 0.0))
        p.prandtl = float(problem.get("prandtl", 0.72))
        p.sutherland = float(problem.get("sutherland", 0.0))
        p.t_ref = float(problem.get("t_ref", 1.0))
        p.precision = FP32_RESIDUAL if precision == "fp32" else FP64
        self.precision = precision
        self._ctx = ctypes.c_void_p()
        _check(lib.rok_create(ctypes.byref(p), ctypes.byref(self._ctx)), "rok_create")
        self.N = int(lib.rok_state_size(self._ctx))
        _check(lib.rok_set_mgs_path(self._ctx, MGS_PATHS[mgs]), "rok_set_mgs_path")
        self.mgs = mgs
        self._work = {}
        self.device = torch.device("cuda", torch.cuda.current_device())

    def __del__(self):
        if getattr(self, "_ctx", None) and _lib is not None:
            _lib.rok_destroy(self._ctx)
            self._ctx = None

    # -- workspace ---------------------------------------------------------
    def workspace(self, M: int, s: int, adjoint: bool | str = False) -> torch.Tensor:
        """Cached aligned workspace: rok_workspace_bytes (adjoint=False),
        rok_step_vjp_workspace_bytes (True), rok_step_vjp_adjoint_bytes ("only")
        or rok_adaptive_workspace_bytes ("adaptive")."""
        if adjoint == "only":
            nb = int(_lib.rok_step_vjp_adjoint_bytes(self._ctx, int(M), int(s)))
        elif adjoint == "adaptive":
            nb = int(_lib.rok_adaptive_workspace_bytes(self._ctx, int(M), int(s)))
        elif adjoint:
            nb = int(_lib.rok_step_vjp_workspace_bytes(self._ctx, int(M), int(s)))
        else:
            nb = int(_lib.rok_workspace_bytes(self._ctx, int(M), int(s)))
        if nb == 0:
            raise ValueError(f"invalid workspace request M={M}, s={s}")
        key = (int(M), int(s), adjoint if isinstance(adjoint, str) else bool(adjoint))
        w = self._work.get(key)
        if w is None or w.numel() < nb:
            w = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            self._work[key] = w
        off = (-w.data_ptr()) % 256
        return w[off:off + nb]

    def _vec(self, t: torch.Tensor, name: str):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.N):
            raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor of {self.N} elements")
        return t

    def _out_dtype(self):
        return torch.float32 if self.precision == "fp32" else torch.float64

    # -- entry points --------------------------------------------------------
    def residual(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._vec(y, "y")
        F = out if out is not None else torch.empty(self.N, dtype=self._out_dtype(), device=y.device)
        _check(_lib.rok_residual(self._ctx, _ptr(y), _ptr(F), _stream()), "rok_residual")
        return F

    def residual_split(self, y: torch.Tensor):
        """(inviscid part, viscous part) of f(y) (rok_residual_split)."""
        self._vec(y, "y")
        Fi = torch.empty(self.N, dtype=self._out_dtype(), device=y.device)
        Fv = torch.empty_like(Fi)
        _check(_lib.rok_residual_split(self._ctx, _ptr(y), _ptr(Fi), _ptr(Fv), _stream()), "rok_residual_split")
        return Fi, Fv

    def jvp(self, y, v, mode: str = "fd", fy=None, eps: float = 0.0, out=None) -> torch.Tensor:
        self._vec(y, "y")
        self._vec(v, "v")
        m = JVP_FD if mode == "fd" else JVP_TANGENT
        if m == JVP_FD:
            if fy is None:
                raise ValueError("the finite-difference product needs fy = f(y)")
            self._vec(fy, "fy")
        w = out if out is not None else torch.empty(self.N, dtype=self._out_dtype(), device=y.device)
        ws = self.workspace(0, 0)
        _check(_lib.rok_jvp(self._ctx, _ptr(y), _ptr(fy), _ptr(v), _ptr(w), m, float(eps), _ptr(ws), ws.numel(),
                            _stream()), "rok_jvp")
        return w

    def jvp_noalloc(self, y, v, mode: str = "fd", fy=None, eps: float = 0.0, out=None) -> torch.Tensor:
        """rok_jvp_noalloc: the product of `jvp` without a workspace (the library's
        own per-device scratch array holds the reductions of the default FD increment)."""
        self._vec(y, "y")
        self._vec(v, "v")
        m = JVP_FD if mode == "fd" else JVP_TANGENT
        if m == JVP_FD:
            if fy is None:
                raise ValueError("the finite-difference product needs fy = f(y)")
            self._vec(fy, "fy")
        w = out if out is not None else torch.empty(self.N, dtype=self._out_dtype(), device=y.device)
        _check(_lib.rok_jvp_noalloc(self._ctx, _ptr(y), _ptr(fy), _ptr(v), _ptr(w), m, float(eps), _stream()),
               "rok_jvp_noalloc")
        return w

    def arnoldi(self, y, fy, M: int, mode: str = "fd", eps: float = 0.0):
        """Returns (V as an (M, N) tensor whose rows are the basis vectors, H (M, M), M_eff)."""
        self._vec(y, "y")
        self._vec(fy, "fy")
        M = min(int(M), self.N)
        V = torch.zeros(M, self.N, dtype=torch.float64, device=y.device)
        H = torch.empty(M, M, dtype=torch.float64, device=y.device)
        meff = torch.empty(1, dtype=torch.int32, device=y.device)
        ws = self.workspace(M, 0)
        m = JVP_FD if mode == "fd" else JVP_TANGENT
        _check(_lib.rok_arnoldi(self._ctx, _ptr(y), _ptr(fy), M, m, float(eps), _ptr(V), _ptr(H), _ptr(meff),
                                _ptr(ws), ws.numel(), _stream()), "rok_arnoldi")
        self._last_arnoldi_ws = ws
        k = int(meff.item())
        return V[:k], H[:k, :k], k

    def step(self, y, h: float, tableau: dict, M: int, mode: str = "fd", out=None) -> torch.Tensor:
        self._vec(y, "y")
        y1 = out if out is not None else torch.empty_like(y)
        tab = make_tableau(tableau)
        ws = self.workspace(M, tab.s)
        m = JVP_FD if mode == "fd" else JVP_TANGENT
        _check(_lib.rok_step(self._ctx, ctypes.byref(tab), int(M), m, float(h), _ptr(y), _ptr(y1), _ptr(ws),
                             ws.numel(), _stream()), "rok_step")
        self._last_step_ws = ws
        return y1

    def set_grid(self, xn, yn):
        """Use a 2-D curvilinear periodic grid with these node coordinates (arrays [j][i];
        rok_set_grid); None, None: back to the Cartesian grid."""
        if xn is None and yn is None:
            _check(_lib.rok_set_grid(self._ctx, None, None, None, _stream()), "rok_set_grid")
            self._metrics = None
            return
        nb = int(_lib.rok_grid_metric_bytes(self._ctx))
        if nb == 0:
            raise ValueError("curvilinear grids need a 2-D problem with at least 2 x 2 cells")
        xd = torch.as_tensor(xn, dtype=torch.float64).to(self.device).contiguous()
        yd = torch.as_tensor(yn, dtype=torch.float64).to(self.device).contiguous()
        if xd.numel() * 9 * 8 != nb or yd.numel() != xd.numel():
            raise ValueError("node arrays must have n[0] * n[1] entries")
        met = torch.empty(nb // 8, dtype=torch.float64, device=self.device)
        _check(_lib.rok_set_grid(self._ctx, _ptr(xd), _ptr(yd), _ptr(met), _stream()), "rok_set_grid")
        self._metrics = met            # kept alive while the context uses it

    def set_ogrid(self, xn, yn, freestream, t_wall: float = 1.0):
        """Use an O-grid (nodes [j][i], j = 0..n[1]; wall at row 0 (isothermal at t_wall for
        Navier-Stokes), far field past the last row, free stream (rho, rho u, rho v, E));
        rok_set_ogrid."""
        nb = int(_lib.rok_ogrid_metric_bytes(self._ctx))
        if nb == 0:
            raise ValueError("O-grids need a 2-D problem with at least 2 x 2 cells")
        xd = torch.as_tensor(xn, dtype=torch.float64).to(self.device).contiguous()
        yd = torch.as_tensor(yn, dtype=torch.float64).to(self.device).contiguous()
        n0, n1 = self._n[0], self._n[1]
        if xd.numel() != n0 * (n1 + 1) or yd.numel() != xd.numel():
            raise ValueError("node arrays must have n[0] * (n[1] + 1) entries")
        met = torch.empty(nb // 8, dtype=torch.float64, device=self.device)
        fs = (ctypes.c_double * 4)(*[float(v) for v in freestream])
        _check(_lib.rok_set_ogrid(self._ctx, _ptr(xd), _ptr(yd), fs, float(t_wall), _ptr(met), _stream()),
               "rok_set_ogrid")
        self._metrics = met

    def eigs(self, y, v0, k: int = 6, m: int = 40, max_restarts: int = 50, tol: float = 1e-10):
        """k largest-magnitude eigenvalues of J(y) (rok_eigs; k + 2 <= m <= 2048, m + 1 <= N).
        Returns (values as a complex numpy array, residual estimates, restarts used, number
        converged)."""
        import numpy as np
        self._vec(y, "y")
        self._vec(v0, "v0")
        nb = int(_lib.rok_eigs_workspace_bytes(self._ctx, int(k), int(m)))
        if nb == 0:
            raise ValueError(f"invalid eigenvalue request k={k}, m={m} for N={self.N}")
        w = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-w.data_ptr()) % 256
        ws = w[off:off + nb]
        re, im, rs = (ctypes.c_double * k)(), (ctypes.c_double * k)(), (ctypes.c_double * k)()
        info = (ctypes.c_int * 2)()
        _check(_lib.rok_eigs(self._ctx, _ptr(y), _ptr(v0), int(k), int(m), int(max_restarts), float(tol), re, im,
                             rs, info, _ptr(ws), ws.numel(), _stream()), "rok_eigs")
        vals = np.array([complex(re[t], im[t]) for t in range(k)])
        return vals, np.array(list(rs)), info[0], info[1]

    def error_norm(self, y_n, y_a, y_b, rtol: float, atol: float, scale: float, out=None) -> torch.Tensor:
        """sqrt(sum_i q_i^2 / N), q_i = (y_a - y_b)_i / (scale (atol + rtol max(|y_n|, |y_a|)_i)),
        as a one-element device tensor."""
        for t, nm in ((y_n, "y_n"), (y_a, "y_a"), (y_b, "y_b")):
            self._vec(t, nm)
        e = out if out is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        ws = self.workspace(0, 0)
        _check(_lib.rok_error_norm(self._ctx, _ptr(y_n), _ptr(y_a), _ptr(y_b), float(rtol), float(atol),
                                   float(scale), _ptr(e), _ptr(ws), ws.numel(), _stream()), "rok_error_norm")
        return e

    def integrate_adaptive(self, y0, T: float, H0: float, tableau: dict, M: int, mode: str = "fd", order: int = 4,
                           rtol: float = 1e-6, atol: float = 1e-6, max_steps: int = 100000,
                           history_cap: int = 4096):
        """Integrate from y0 to T under step-doubling control (rok_integrate_adaptive).

        Returns (y_T, record) with record = {"accepted": [(t, H, err)], "rejected": [(t, H, err)],
        "t": time reached, "h_next": next proposed step}; raises if T was not reached.
        """
        self._vec(y0, "y0")
        y = y0.clone()
        tab = make_tableau(tableau)
        ws = self.workspace(M, tab.s, adjoint="adaptive")
        st = RokAdaptiveStats()
        hist = (ctypes.c_double * (4 * max(1, history_cap)))()
        m = JVP_FD if mode == "fd" else JVP_TANGENT
        _check(_lib.rok_integrate_adaptive(self._ctx, ctypes.byref(tab), int(M), m, int(order), float(T), float(H0),
                                           float(rtol), float(atol), int(max_steps), _ptr(y), ctypes.byref(st),
                                           hist, int(history_cap), _ptr(ws), ws.numel(), _stream()),
               "rok_integrate_adaptive")
        rec = {"accepted": [], "rejected": [], "t": st.t, "h_next": st.h_next,
               "n_accepted": st.accepted, "n_rejected": st.rejected}
        for k in range(st.recorded):
            e = (hist[4 * k], hist[4 * k + 1], hist[4 * k + 2])
            rec["accepted" if hist[4 * k + 3] == 1.0 else "rejected"].append(e)
        if st.t < T:
            why = "max_steps attempts" if st.accepted + st.rejected >= max_steps else "step size underflow"
            raise RokError(f"rok_integrate_adaptive stopped at t = {st.t} < T = {T} ({why}: "
                           f"{st.accepted} accepted, {st.rejected} rejected)")
        return y, rec

    def vjp(self, y, wbar, v=None, accumulate_into=None, accumulate_into2=None):
        """J(y)^T wbar; with v also d/dt [J(y + t v)^T wbar] (returned as a pair).

        accumulate_into(2): add to these tensors instead of returning new ones.
        """
        self._vec(y, "y")
        self._vec(wbar, "wbar")
        acc = accumulate_into is not None
        yb = accumulate_into if acc else torch.empty_like(y)
        self._vec(yb, "ybar")
        if v is None:
            _check(_lib.rok_residual_vjp(self._ctx, _ptr(y), _ptr(wbar), _ptr(yb), int(acc), _stream()),
                   "rok_residual_vjp")
            return yb
        self._vec(v, "v")
        if acc != (accumulate_into2 is not None):
            raise ValueError("accumulate both outputs or neither")
        yb2 = accumulate_into2 if acc else torch.empty_like(y)
        self._vec(yb2, "ybar2")
        _check(_lib.rok_residual_vjp2(self._ctx, _ptr(y), _ptr(v), _ptr(wbar), _ptr(yb), _ptr(yb2), int(acc),
                                      _stream()), "rok_residual_vjp2")
        return yb, yb2

    def step_vjp(self, y, ybar_next, h: float, tableau: dict, M: int, y_next_out=None, out=None):
        """(d y_{n+1}/d y_n)^T ybar_next for the exact-product step from y; optionally writes y_{n+1}."""
        self._vec(y, "y")
        self._vec(ybar_next, "ybar_next")
        yb = out if out is not None else torch.empty_like(y)
        self._vec(yb, "out")
        if y_next_out is not None:
            self._vec(y_next_out, "y_next_out")
        tab = make_tableau(tableau)
        ws = self.workspace(M, tab.s, adjoint=True)
        _check(_lib.rok_step_vjp(self._ctx, ctypes.byref(tab), int(M), float(h), _ptr(y), _ptr(ybar_next), _ptr(yb),
                                 _ptr(y_next_out), _ptr(ws), ws.numel(), _stream()), "rok_step_vjp")
        self._last_step_ws = ws   # the status header leads the adjoint workspace too
        return yb

    def step_keep(self, y, h: float, tableau: dict, M: int, out=None):
        """Exact-product step in a workspace of its own, kept for step_vjp_stored:
        returns (y_{n+1}, ForwardRecord).  Memory: one forward workspace (about
        M + 2 s state vectors) per kept step."""
        self._vec(y, "y")
        y1 = out if out is not None else torch.empty_like(y)
        tab = make_tableau(tableau)
        nb = int(_lib.rok_workspace_bytes(self._ctx, int(M), tab.s))
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=y.device)
        off = (-buf.data_ptr()) % 256
        ws = buf[off:off + nb]
        _check(_lib.rok_step(self._ctx, ctypes.byref(tab), int(M), JVP_TANGENT, float(h), _ptr(y), _ptr(y1),
                             _ptr(ws), ws.numel(), _stream()), "rok_step")
        self._last_step_ws = ws
        return y1, ForwardRecord(y, float(h), tableau, int(M), ws)

    def step_vjp_stored(self, rec: ForwardRecord, ybar_next, out=None):
        """(d y_{n+1}/d y_n)^T ybar_next from a kept step, without recomputing it
        (bitwise equal to step_vjp)."""
        self._vec(ybar_next, "ybar_next")
        yb = out if out is not None else torch.empty_like(ybar_next)
        self._vec(yb, "out")
        tab = make_tableau(rec.tableau)
        aws = self.workspace(rec.M, tab.s, adjoint="only")
        _check(_lib.rok_step_vjp_stored(self._ctx, ctypes.byref(tab), rec.M, rec.h, _ptr(rec.y), _ptr(ybar_next),
                                        _ptr(yb), _ptr(rec.ws), rec.ws.numel(), _ptr(aws), aws.numel(), _stream()),
               "rok_step_vjp_stored")
        self._last_step_ws = rec.ws
        return yb

    def arnoldi_path(self, M: int) -> str:
        """How the Arnoldi columns are orthogonalised on this context for Krylov
        dimension M (rok_arnoldi_path): "pass", "resident" or "one_reduce"."""
        r = int(_lib.rok_arnoldi_path(self._ctx, int(M)))
        names = {v: k for k, v in MGS_PATHS.items()}
        if r not in names or r == 0:
            raise RokError(f"rok_arnoldi_path: {r}")
        return names[r]

    def mgs_workspace(self, M: int) -> torch.Tensor:
        """A workspace for column-level calls, prepared for Krylov dimension M."""
        ws = self.workspace(M, 0)
        _check(_lib.rok_workspace_init(self._ctx, _ptr(ws), ws.numel(), int(M), 0, _stream()), "rok_workspace_init")
        self._last_step_ws = ws
        return ws

    def mgs_column(self, V: torch.Tensor, j: int, w: torch.Tensor, H: torch.Tensor, ws: torch.Tensor,
                   vnext: torch.Tensor | None = None):
        """One modified Gram-Schmidt column: V is (M, N) with rows as basis vectors, H is (M + 1, M)."""
        M = V.shape[0]
        if not (V.is_cuda and V.dtype == torch.float64 and V.is_contiguous() and V.shape[1] == self.N):
            raise ValueError("V: expected a contiguous (M, N) float64 CUDA tensor")
        if not (H.is_cuda and H.dtype == torch.float64 and H.is_contiguous() and tuple(H.shape) == (M + 1, M)):
            raise ValueError("H: expected a contiguous (M + 1, M) float64 CUDA tensor")
        self._vec(w, "w")
        if vnext is not None:
            self._vec(vnext, "vnext")
        _check(_lib.rok_mgs_column(self._ctx, _ptr(V), int(M), int(j), _ptr(w), _ptr(H), _ptr(vnext), _ptr(ws),
                                   ws.numel(), _stream()), "rok_mgs_column")

    def last_arnoldi_flags(self) -> int:
        """Status flags (FLAG_*) of the last rok_arnoldi call (synchronises the stream)."""
        f = ctypes.c_int()
        _check(_lib.rok_read_status(self._ctx, _ptr(self._last_arnoldi_ws), ctypes.byref(f), _stream()),
               "rok_read_status")
        return f.value

    def last_status(self) -> tuple[int, int]:
        """(flags, M_eff) of the last step (synchronises the stream)."""
        ws = self._last_step_ws
        f, m = ctypes.c_int(), ctypes.c_int()
        _check(_lib.rok_read_status(self._ctx, _ptr(ws), ctypes.byref(f), _stream()), "rok_read_status")
        _check(_lib.rok_read_meff(self._ctx, _ptr(ws), ctypes.byref(m), _stream()), "rok_read_meff")
        return f.value, m.value
