"""Benchmark: ROK steps per second on one MI355X.

Workload (default): the 3-D compressible Navier-Stokes Taylor-Green vortex on
a periodic 256^3 grid (Re 1600, Mach 0.1, N = 83.9 M unknowns), MUSCL (minmod)
+ Rusanov inviscid flux and central viscous fluxes, four-stage ROK4 with
Krylov dimension M = 16, the plain FP64 method with finite-difference
Jacobian-vector products, fixed step at CFL 10.  Inputs are synthetic (seeded)
and resident in HBM before the timed region starts.

Prints one JSON line with the step rate, a roofline entry for the dominant
kernel of the step (the Arnoldi column by the one-reduce Gram-Schmidt, whose
work vector does not fit on chip at this size; timed live with HIP events on
the launch stream) and for the FD product and residual kernels, the
Arnoldi share of the step against its algorithmic bytes, the precision form's
rate on the same workload (FP32 residual and tangent products, FP64 Krylov)
with its error, the 1024^2 MUSCL vortex as a secondary workload, the
equal-error comparison of FP32 + tangent against FP64 + FD (work-precision
sweeps on a 512^2 2-D and a 96^3 3-D Taylor-Green proxy), and the CPU
oracle's rate on a bounded sample of the workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-equal-error]
                    [--no-secondary] [--adjoint] [--krylov-sweep]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles (16 lanes), 2.4 GHz
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tgv256_3d_fp64")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the precision form's rate and the 1024^2 vortex next to the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the CPU oracle sample")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only the roofline kernel loop and a calibration copy (for counter runs)")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with counter figures per launch of the roofline kernels (default: "
                         "profiles/traffic_<workload>.json)")
    ap.add_argument("--traffic-from", default=None, metavar="DIR",
                    help="write profiles/traffic_<workload>.json from the three counter runs under DIR "
                         "(pmc_<workload>_FETCH_SIZE, _WRITE_SIZE, _SQ_INSTS_VALU_SQ_WAVES; see build_traffic) "
                         "and exit; needs no GPU")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the discrete adjoint of the step (rok_step_vjp; on by default for the "
                         "differentiation workload)")
    ap.add_argument("--no-equal-error", action="store_true",
                    help="skip the FP32-tangent vs FP64-FD equal-error sweep")
    ap.add_argument("--krylov-sweep", action="store_true",
                    help="also run the Krylov-dimension sweep (M = 4..20: error and time at fixed final time)")
    ap.add_argument("--adaptive", action="store_true",
                    help="also run the adaptive work-precision sweep (step doubling; ERK4 vs ROK4 M = 4, 8)")
    ap.add_argument("--adaptive-cases", default="all",
                    help="comma-separated name prefixes of the adaptive sweep's cases (default: all)")
    ap.add_argument("--adjoint-ogrid", action="store_true",
                    help="also time the gradient through 20 steps on the viscous cylinder O-grid")
    ap.add_argument("--eigs", action="store_true",
                    help="also run the stiffness diagnostic (largest eigenvalues of J on the cylinder O-grids)")
    ap.add_argument("--chain", action="store_true",
                    help="time a trajectory (each step starts from the previous result) instead of K passes "
                         "over the seeded input state")
    return ap.parse_args()


RESIDUAL_SOURCES = ("rok_residual.hip", "rok_flux.hpp", "rok_device.hpp")
MGS_SOURCES = ("rok_mgs.hip", "rok_kernels.hpp", "rok_device.hpp")
KRED_SOURCES = ("rok_krylov.hip", "rok_kernels.hpp", "rok_device.hpp")
LS_SOURCES = ("rok_lowsync.hip", "rok_krylov.hip", "rok_kernels.hpp", "rok_device.hpp")


def _source_hash(names):
    """sha256 (16 hex digits) of the kernel sources with comments and white space
    removed: any change to the code invalidates stored counters, a comment does not."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1607_06834_amd", "csrc")
    data = ""
    for name in names:
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        data += " ".join(text.split()) + "\n"
    return hashlib.sha256(data.encode()).hexdigest()[:16]


def _traffic_path(args):
    if args.traffic:
        return args.traffic
    return os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")


def gpu_leg(args, pb, y0, w, tab, h, workload=None, rooflines=True):
    import torch

    from paper_1607_06834_amd import Rok

    dev = torch.device("cuda", 0)
    g = Rok(pb, w["precision"])
    mode = "fd" if w["jvp"] == "fd" else "exact"
    M = w["M"]
    ya = torch.tensor(y0, dtype=torch.float64, device=dev)
    yb = torch.empty_like(ya)

    def one_step(ya, yb):
        g.step(ya, h, tab, M, mode, out=yb)
        return (yb, ya) if args.chain else (ya, yb)

    steps = 0 if args.roofline_only else args.steps
    for _ in range(0 if args.roofline_only else args.warmup):
        ya, yb = one_step(ya, yb)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ya, yb = one_step(ya, yb)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    flags, meff = g.last_status() if steps else (0, 0)
    finite = bool(torch.isfinite(yb if not args.chain else ya).all()) if steps else True
    out = {"ms_per_step": ev_ms / max(steps, 1), "wall_s": wall, "flags": flags, "M_eff": meff, "finite": finite}
    if not rooflines:
        return out
    # calibration kernel for the HBM counters: a plain copy of one state vector (8 N bytes read, 8 N written)
    calib = torch.empty_like(ya)
    calib.copy_(ya)
    torch.cuda.synchronize()
    del calib, yb
    mgs, arn = _mgs_roofline(args, g, ya, M, mode, stream, out["ms_per_step"])
    out.update(roofline=mgs, arnoldi_step=arn, roofline_jvp=_jvp_roofline(args, g, ya, w, stream),
               roofline_residual=_residual_roofline(args, g, ya, w, stream), adjoint=None)
    if (args.adjoint or args.workload == "vortex512_adjoint") and not args.roofline_only:
        out["adjoint"] = _adjoint_leg(args, g, ya, h, tab, M, stream)
    return out


def _adjoint_leg(args, g, y, h, tab, M, stream):
    """Discrete adjoint of one exact-product step (rok_step_vjp: recomputation of
    the step from y_n plus the reverse sweep), K calls from the seeded state,
    HIP events; next to the forward exact-product step for comparison."""
    import torch
    if g.precision != "fp64":
        return None
    yb = torch.ones_like(y) / math.sqrt(y.numel())
    out = torch.empty_like(y)
    for _ in range(2):
        g.step_vjp(y, yb, h, tab, M, out=out)
        g.step(y, h, tab, M, mode="tangent")
    torch.cuda.synchronize()
    K = max(1, args.steps // 2)

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(K):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    fwd = timed(lambda: g.step(y, h, tab, M, mode="tangent"))
    bwd = timed(lambda: g.step_vjp(y, yb, h, tab, M, out=out))
    _, rec = g.step_keep(y, h, tab, M)         # the forward kept: reverse sweep only
    g.step_vjp_stored(rec, yb, out=out)
    stored = timed(lambda: g.step_vjp_stored(rec, yb, out=out))
    return {"forward_exact_ms_per_step": round(fwd, 4), "step_vjp_ms_per_step": round(bwd, 4),
            "ratio": round(bwd / fwd, 3), "step_vjp_stored_ms_per_step": round(stored, 4),
            "ratio_stored": round(stored / fwd, 3), "steps": K}


def _timed(stream, launches):
    """Average milliseconds per launch: each callable in `launches` enqueues one
    kernel, bracketed by its own pair of HIP events on `stream`, so host-side
    gaps between launches are not counted."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in launches]
    for (a, b), fn in zip(ev, launches):
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / len(ev)


def _ls_column_bytes(N, m):
    """Bytes the kernels of a one-reduce column move, averaged over the m
    columns of a basis (as rok_mgs_column runs them): k_ls_dots reads
    v_0..v_j and w (j + 2 vectors), k_ls_update reads them again and writes
    the next column (j + 3), k_normalize reads and writes it (2); the last
    column runs k_ls_dots alone.  Inside rok_step the normalisation pass is
    deferred (2j + 5 per column)."""
    return sum(((j + 2) + ((j + 3) + 2 if j + 1 < m else 0)) * 8 * N for j in range(m)) / m


def _traffic(path, sources, key, field="hbm_bytes_per_launch"):
    """A counter figure per launch (HBM bytes by default) stored for `key`, or None."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(key)
    # counters are only valid for the kernel source they were taken on
    if not ent or ent.get("source_sha256_16") != _source_hash(sources):
        return None
    return ent.get(field)


def _mgs_roofline(args, g, y, M, mode, stream, ms_step):
    """The Arnoldi columns (a4), as the step runs them.

    The basis of the step's Arnoldi process at y and the products w_j = J v_j
    are prepared first; the timed loop then runs the M columns j = 0..M-1 as
    the step does, one HIP event pair per column.
    * Resident path (N <= 4.19 M: one cooperative kernel per column, w held
      on chip): a launch is a column; algorithmic bytes of column j: w and
      v_0..v_j read, v_{j+1} written.
    * One-reduce path (the default for larger N: w does not fit on chip):
      a launch is a column of four kernels (dots against w and the Gram row,
      the small solve, the update with the norm's partial sums, the
      normalisation); algorithmic bytes as for the resident column, the
      kernels themselves read the basis twice (`kernel_bytes_per_launch`).
    * Per-pass path (modified Gram-Schmidt forced, larger N): column j runs j update passes
      (w <- w - h v_{i-1}, <v_i, w>), a first dot, a norm pass and the
      normalisation; the time of one update pass is the slope of the column
      time in j (least squares over j = 1..M-1), the per-launch average that
      rocprofv3 reports for k_red<true, false>.  Algorithmic bytes of a pass:
      24 per element (w read and written, v_i read), the figure for a
      modified Gram-Schmidt pass whose work vector is not on chip; the kernel
      also reads v_{i-1} (32 bytes, `kernel_bytes_per_launch`).
    arnoldi_step: all M columns of a step against the step's Arnoldi
    algorithmic bytes, M(M+1)/2 + M vectors (each basis vector read once per
    pass it enters, each written once) -- the resident algorithm's traffic."""
    import torch
    N = g.N
    F = g.residual(y).to(torch.float64)
    V, H, m = g.arnoldi(y, F, M, mode)
    V = V.contiguous()
    del H
    Ws = torch.empty(m, N, dtype=torch.float64, device=y.device)
    for j in range(m):
        Ws[j].copy_(g.jvp(y, V[j], mode="fd" if mode == "fd" else "tangent", fy=F, eps=1e-7).to(torch.float64))
    Hs = torch.zeros(m + 1, m, dtype=torch.float64, device=y.device)
    ws = g.mgs_workspace(m)
    wk = torch.empty(N, dtype=torch.float64, device=y.device)
    vn = torch.empty(N, dtype=torch.float64, device=y.device)
    path = g.arnoldi_path(m)

    def column_timed(j, reps):
        # the copy that restores w (a column may overwrite it) is outside the events
        ev = []
        for _ in range(reps):
            wk.copy_(Ws[j])
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.mgs_column(V, j, wk, Hs, ws, vnext=vn if j + 1 < m else None)
            b.record(stream)
            ev.append((a, b))
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in ev) / reps

    for j in range(m):
        column_timed(j, 1)
    reps = max(1, args.kernel_reps // 4)
    col_ms = [column_timed(j, reps) for j in range(m)]
    a4_bytes = (m * (m + 1) // 2 + m) * 8 * N
    arn_ms = sum(col_ms)
    arn = {"ms_per_step": round(arn_ms, 4), "share_of_step": round(arn_ms / ms_step, 4) if ms_step else None,
           "alg_bytes_per_step": a4_bytes, "achieved": round(a4_bytes / (arn_ms * 1e-3) / 1e9, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(a4_bytes / (arn_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "what": f"the {m} Arnoldi columns of a step (HIP events per column) against M(M+1)/2 + M basis-vector "
                   f"reads and writes"}
    tpath = _traffic_path(args)
    traffic = None
    col_alg = sum((j + 2) * 8 * N + (8 * N if j + 1 < m else 0) for j in range(m)) / m
    if path == "resident":
        ms = sum(col_ms) / m
        alg = col_alg
        traffic = _traffic(tpath, MGS_SOURCES, "mgs_column")
        kernel = f"modified Gram-Schmidt Arnoldi column (k_mgs_resident), average over the {m} columns of a step"
        extra = {}
    elif path == "one_reduce":
        ms = sum(col_ms) / m
        alg = col_alg
        traffic = _traffic(tpath, LS_SOURCES, "ls_column")
        kb = _ls_column_bytes(N, m)
        kernel = (f"one-reduce Gram-Schmidt Arnoldi column (k_ls_dots, k_ls_solve, k_ls_update, k_normalize), "
                  f"average over the {m} columns of a step")
        extra = {"kernel_bytes_per_launch": int(kb),
                 "timing": "one HIP event pair per column of rok_mgs_column (its four launches, the normalisation "
                           "included; rok_step defers that pass)"}
    else:
        js = list(range(1, m))
        mj = sum(js) / len(js)
        mt = sum(col_ms[j] for j in js) / len(js)
        ms = sum((j - mj) * (col_ms[j] - mt) for j in js) / sum((j - mj) ** 2 for j in js)
        alg = 24 * N
        traffic = _traffic(tpath, KRED_SOURCES, "mgs_pass")
        kernel = "modified Gram-Schmidt pass with the work vector streamed (k_red<true, false>)"
        extra = {"kernel_bytes_per_launch": 32 * N, "timing": "slope of the column time in j (HIP events per column)"}
    achieved = alg / (ms * 1e-3) / 1e9
    rl = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
          "avg_launch_ms": round(ms, 5), "alg_bytes_per_launch": int(alg)}
    rl.update(extra)
    return rl, arn


def _residual_roofline(args, g, y, w, stream):
    """The residual kernel F = f(y): reads y, writes F (16 B per element in
    FP64; 12 B when F is written in FP32)."""
    import torch
    N = g.N
    out = torch.empty(N, dtype=torch.float64 if w["precision"] == "fp64" else torch.float32, device=y.device)
    for _ in range(3):
        g.residual(y, out=out)
    torch.cuda.synchronize()
    ms = _timed(stream, [lambda: g.residual(y, out=out)] * args.kernel_reps)
    alg = (8 + out.element_size()) * N
    achieved = alg / (ms * 1e-3) / 1e9
    traffic = _traffic(_traffic_path(args), RESIDUAL_SOURCES, "residual")
    valu = _traffic(_traffic_path(args), RESIDUAL_SOURCES, "residual", "valu_insts_per_launch")
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    common = {"kernel": "finite-volume residual F = f(y)", "avg_launch_ms": round(ms, 5), "alg_bytes_per_launch": alg}
    if valu is None:
        return dict(hbm, **common)
    ginst = valu / (ms * 1e-3) / 1e9
    return dict({"bound": "alu", "achieved": round(ginst, 1), "peak": VALU_PEAK_GINST,
                 "unit": "G VALU wave-instructions/s", "frac": round(ginst / VALU_PEAK_GINST, 4),
                 "valu_insts_per_launch": valu, "hbm": hbm}, **common)


def _jvp_roofline(args, g, y, w, stream):
    """The product kernel of the workload.  FP64: the FD Jacobian-vector
    product, reads y, v, f(y), writes w (32 B per element).  FP32 form: the
    exact (tangent) product in FP32, reads y and v, writes w in FP32 (20 B per
    element; inside rok_step the same kernel writes FP64 for the Krylov side)."""
    import torch
    N = g.N
    dev = y.device
    v = torch.randn(N, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
    v /= torch.linalg.vector_norm(v)
    if w["precision"] == "fp64":
        F = g.residual(y)
        out = torch.empty(N, dtype=torch.float64, device=dev)
        launch = lambda: g.jvp(y, v, "fd", fy=F, eps=1e-7, out=out)
        alg, key = 4 * 8 * N, "fd_jvp"
        kernel = "FD Jacobian-vector product (residual at y + eps v, minus f(y), over eps)"
    else:
        out = torch.empty(N, dtype=torch.float32, device=dev)
        launch = lambda: g.jvp(y, v, "tangent", out=out)
        alg, key = (8 + 8 + 4) * N, "tangent"
        kernel = "exact (tangent) Jacobian-vector product, FP32 dual numbers in reference-state form"
    for _ in range(3):
        launch()
    torch.cuda.synchronize()
    ms = _timed(stream, [launch] * args.kernel_reps)
    achieved = alg / (ms * 1e-3) / 1e9
    traffic = _traffic(_traffic_path(args), RESIDUAL_SOURCES, key)
    valu = _traffic(_traffic_path(args), RESIDUAL_SOURCES, key, "valu_insts_per_launch")
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    common = {"kernel": kernel, "avg_launch_ms": round(ms, 5), "alg_bytes_per_launch": alg}
    if valu is None:
        return dict(hbm, **common)
    # the binding roof: wave-level VALU instructions issued per second (SQ_INSTS_VALU per launch, counter run)
    ginst = valu / (ms * 1e-3) / 1e9
    return dict({"bound": "alu", "achieved": round(ginst, 1), "peak": VALU_PEAK_GINST,
                 "unit": "G VALU wave-instructions/s", "frac": round(ginst / VALU_PEAK_GINST, 4),
                 "valu_insts_per_launch": valu, "hbm": hbm}, **common)




def equal_error_leg(args, ndim=2):
    """FP32 residual/tangent + FP64 Krylov against plain FP64 with finite-difference
    products, at equal final-time error (work-precision sweep).

    ndim = 2: proxy of the 2048^2 viscous Taylor-Green workload at 512^2 (Re
    100, Mach 0.1, MUSCL, M = 20), T = 10 h(CFL 4), CFL 1, 2, 4, 8.
    ndim = 3: proxy of the 256^3 workload at 96^3 (Re 1600, Mach 0.1, MUSCL,
    M = 16), T = 2 h(CFL 20), CFL 2.5, 5, 10, 20.
    Both forms integrate to the same final time; the error is
    ||y_N - y_ref|| / ||y_ref|| with y_ref the FP64 exact-product ROK solution
    at CFL 1/8.  Trajectories are timed with HIP events.
    speedup_at_equal_error: for each FP32 point, the FD time at the same error
    (log-log interpolation between the bracketing FD points) over the FP32
    time.  fp32_floor: the smallest FP32 error reached (where its curve
    flattens)."""
    import torch

    import rok_inputs as ri
    from paper_1607_06834_amd import Rok

    dev = torch.device("cuda", 0)
    if ndim == 2:
        pb = ri.tgv_problem(512, 2)
        M, cfls, T_cfl, T_mult = 20, (1.0, 2.0, 4.0, 8.0), 4.0, 10
        label = "Taylor-Green 2-D, 512x512, Re 100, Mach 0.1, MUSCL, M = 20, T = 10 h(CFL 4)"
    else:
        pb = ri.tgv_problem(96, 3)
        M, cfls, T_cfl, T_mult = 16, (2.5, 5.0, 10.0, 20.0), 20.0, 2
        label = "Taylor-Green 3-D, 96^3, Re 1600, Mach 0.1, MUSCL, M = 16, T = 2 h(CFL 20)"
    y0 = ri.tgv_state(pb)
    tab = ri.rok4_tableau()
    T = T_mult * ri.cfl_step(pb, y0, T_cfl)
    g64, g32 = Rok(pb, "fp64"), Rok(pb, "fp32")
    stream = torch.cuda.current_stream()

    def run(g, cfl, mode):
        K = int(round(T / ri.cfl_step(pb, y0, cfl)))
        h = T / K
        y = torch.tensor(y0, device=dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(K):
            y = g.step(y, h, tab, M, mode)
        e1.record(stream)
        torch.cuda.synchronize()
        return y, e0.elapsed_time(e1), K

    ref, _, _ = run(g64, 0.125, "exact")
    nref = float(torch.linalg.vector_norm(ref))
    pts = {"fp64_fd": [], "fp32_tangent": []}
    for cfl in cfls:
        for name, g, mode in (("fp64_fd", g64, "fd"), ("fp32_tangent", g32, "exact")):
            y, ms, K = run(g, cfl, mode)
            err = float(torch.linalg.vector_norm(y - ref)) / nref
            err = float(f"{err:.4e}") if math.isfinite(err) else None   # None: the trajectory blew up
            pts[name].append({"cfl": cfl, "steps": K, "ms": round(ms, 3), "error": err})
    fd = sorted((q for q in pts["fp64_fd"] if q["error"] is not None), key=lambda q: q["error"])
    ratios = []
    for q in pts["fp32_tangent"]:
        e = q["error"]
        if e is None:
            continue
        for a, b in zip(fd, fd[1:]):
            if a["error"] <= e <= b["error"] and a["error"] > 0 and b["error"] > a["error"]:
                f = (math.log(e) - math.log(a["error"])) / (math.log(b["error"]) - math.log(a["error"]))
                t_fd = math.exp(math.log(a["ms"]) + f * (math.log(b["ms"]) - math.log(a["ms"])))
                ratios.append({"error": e, "fp32_ms": q["ms"], "fp64_fd_ms": round(t_fd, 3),
                               "speedup": round(t_fd / q["ms"], 3)})
                break
    floor = min((q["error"] for q in pts["fp32_tangent"] if q["error"] is not None), default=None)
    return {"workload": label, "reference": "FP64 exact-product ROK at CFL 1/8", "points": pts,
            "speedup_at_equal_error": ratios, "fp32_floor": floor}


def krylov_sweep_leg(args):
    """Krylov dimension M in {4, 8, 12, 16, 20} (FP64, FD products): error at a
    fixed final time T = 10 h(CFL 4) and its cost, at CFL 1, 2, 4, 8, on the
    512^2 Taylor-Green proxy and the 1024^2 MUSCL vortex.  Error: ||y_N - y_ref||
    / ||y_ref|| with y_ref the exact-product ROK solution at CFL 1/8 and M = 20;
    trajectories timed with HIP events; null where the trajectory is not finite."""
    import torch

    import rok_inputs as ri
    from paper_1607_06834_amd import Rok

    dev = torch.device("cuda", 0)
    tab = ri.rok4_tableau()
    stream = torch.cuda.current_stream()
    out = {}
    for name, (pb, y0) in (("taylor_green_512", (ri.tgv_problem(512, 2), None)),
                           ("vortex_muscl_1024", (ri.vortex_problem(1024, "muscl"), None))):
        y0 = ri.tgv_state(pb) if pb["physics"] == "ns" else ri.vortex_state(pb)
        T = 10 * ri.cfl_step(pb, y0, 4.0)
        g = Rok(pb, "fp64")

        def run(cfl, M, mode):
            K = int(round(T / ri.cfl_step(pb, y0, cfl)))
            h = T / K
            y = torch.tensor(y0, device=dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(K):
                y = g.step(y, h, tab, M, mode)
            e1.record(stream)
            torch.cuda.synchronize()
            return y, e0.elapsed_time(e1), K

        ref, _, _ = run(0.125, 20, "exact")
        nref = float(torch.linalg.vector_norm(ref))
        rows = []
        for M in (4, 8, 12, 16, 20):
            for cfl in (1.0, 2.0, 4.0, 8.0):
                y, ms, K = run(cfl, M, "fd")
                fin = bool(torch.isfinite(y).all())
                err = float(torch.linalg.vector_norm(y - ref)) / nref if fin else None
                rows.append({"M": M, "cfl": cfl, "steps": K, "ms": round(ms, 3),
                             "ms_per_step": round(ms / K, 4), "error": float(f"{err:.4e}") if err is not None else None})
        out[name] = rows
        del g
    return out


def adaptive_leg(args):
    """Adaptive step-size control (step doubling, rok_integrate_adaptive):
    explicit RK4 (M = 0) against ROK4 with FD products (FP64) at rtol = atol in
    {1e-3, 1e-4, 1e-5, 1e-6}, from H0 = h(CFL 1), on
      * the 512^2 Taylor-Green proxy at Mach 0.1 to T = 100 h(CFL 4), and at
        Mach 0.01 to T = 0.25 (flow time; about 4000 h(CFL 1)): acoustic waves
        set the explicit limit, the vortical flow the accuracy, and the gap
        between the two grows as the Mach number falls;
      * the 1024^2 MUSCL vortex to T = 40 h(CFL 4);
      * an impulsively started Mach 0.3 flow around a cylinder on a 128 x 64
        O-grid with very thin wall cells (first cell 2.5e-5, and 6.1e-7 in a
        second case; slip wall, far field, Roe flux) to T = 0.05 from H0 = 1e-5,
        and a viscous one (Navier-Stokes, mu = 0.01 with Sutherland's law,
        isothermal wall at the free-stream temperature, first cell 1.5e-4) to
        T = 0.01.
    Error: ||y_T - y_ref|| / ||y_ref|| with y_ref the exact-product ROK solution
    (M = 20) at CFL 1/8, explicit RK4 at CFL 1/4 for the Mach 0.01 case, and
    adaptive explicit RK4 at rtol = atol = 1e-11 for the cylinder (the paper's
    choice of reference).
    Reported per run: accepted and rejected macro steps, ROK steps taken (3 per
    attempt), wall time of the call (it synchronises once per macro step), the
    mean accepted step in CFL units and the error; a run that does not reach T
    is reported with a note."""
    import time

    import numpy as np
    import torch

    import rok_inputs as ri
    from paper_1607_06834_amd import Rok

    dev = torch.device("cuda", 0)
    tab = ri.rok4_tableau()
    out = {}
    tg = ri.tgv_problem(512, 2)
    vx = ri.vortex_problem(1024, "muscl")
    cases = [
        ("taylor_green_512", tg, ri.tgv_state(tg), ("cfl4", 100), "rok_exact", (0, 4, 8)),
        ("taylor_green_512_mach0.01", tg, ri.tgv_state(tg, mach=0.01), ("time", 0.25), "erk", (0, 4, 8, 16)),
        ("vortex_muscl_1024", vx, ri.vortex_state(vx), ("cfl4", 40), "rok_exact", (0, 4, 8)),
    ]
    # cylinder O-grid with thin wall cells (first cell 2.5e-5 of 19.5 radial extent): the stiffness
    # sits in the few modes of the wall cells, the configuration of the paper's cylinder cases
    cpb, cnodes = ri.cylinder_ogrid(128, 64, radius=0.5, far=20.0, recon="first", flux="roe", cluster=12.0)
    cfs = ri.freestream(mach=0.3)
    cy0 = np.tile(np.asarray(cfs, dtype=np.float64)[:, None], (1, 128 * 64)).reshape(-1)
    cases.append(("cylinder_ogrid_128x64", cpb, cy0, ("time", 0.05), "erk_tight", (0, 4, 8)))
    # the same with wall cells 40 times thinner (first cell 6.1e-7)
    spb, snodes = ri.cylinder_ogrid(128, 64, radius=0.5, far=20.0, recon="first", flux="roe", cluster=16.0)
    cases.append(("cylinder_ogrid_128x64_thin", spb, cy0, ("time", 0.05), "erk_tight", (0, 4, 8)))
    # viscous cylinder (Re about 35 on the diameter, isothermal wall at the free-stream temperature, Sutherland
    # viscosity): the wall-normal diffusion in the thin wall cells is the stiffest part of the spectrum
    vpb, vnodes = ri.cylinder_ogrid(128, 64, radius=0.5, far=20.0, recon="first", flux="roe", cluster=10.0)
    vpb = dict(vpb, physics="ns", mu=0.01, sutherland=0.4, t_ref=1.0)
    cases.append(("cylinder_ns_128x64", vpb, cy0, ("time", 0.01), "erk_tight", (0, 4, 8)))
    grids = {"cylinder_ogrid_128x64": cnodes, "cylinder_ogrid_128x64_thin": snodes, "cylinder_ns_128x64": vnodes}
    if args.adaptive_cases != "all":
        keep = args.adaptive_cases.split(",")
        cases = [c for c in cases if any(c[0].startswith(k) for k in keep)]
    for name, pb, y0, (kind, span), ref_kind, Ms in cases:
        g = Rok(pb, "fp64")
        if name.startswith("cylinder"):
            g.set_ogrid(*grids[name], cfs, t_wall=(1.4 - 1.0) * (cfs[3] - 0.5 * cfs[1] ** 2 / cfs[0]) / cfs[0])
            h1 = 1e-5                   # first attempted step; "mean_cfl" is then in units of h1
        else:
            h1 = ri.cfl_step(pb, y0, 1.0)
        T = span * ri.cfl_step(pb, y0, 4.0) if kind == "cfl4" else float(span)
        y = torch.tensor(y0, device=dev)
        if ref_kind == "erk_tight":
            K = 0
            y, _ = g.integrate_adaptive(y, T, h1, tab, 0, "fd", order=4, rtol=1e-11, atol=1e-11, max_steps=200000,
                                        history_cap=0)
        elif ref_kind == "rok_exact":
            K = int(round(T / ri.cfl_step(pb, y0, 0.125)))
            for _ in range(K):
                y = g.step(y, T / K, tab, 20, "exact")
        else:
            K = int(round(T / ri.cfl_step(pb, y0, 0.25)))
            for _ in range(K):
                y = g.step(y, T / K, tab, 0, "fd")
        ref = y
        nref = float(torch.linalg.vector_norm(ref))
        print(f"[adaptive] {name} reference: {ref_kind}, {K} steps", file=sys.stderr, flush=True)
        yd = torch.tensor(y0, device=dev)
        g.integrate_adaptive(yd, h1, h1, tab, 4, "fd")          # warm-up (workspace, code objects)
        rows = []
        for M in Ms:
            for tol in (1e-3, 1e-4, 1e-5, 1e-6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                try:
                    yT, rec = g.integrate_adaptive(yd, T, h1, tab, M, "fd", order=4, rtol=tol, atol=tol,
                                                   max_steps=60000, history_cap=0)
                except Exception as exc:        # noqa: BLE001 - a run that does not reach T is reported
                    rows.append({"M": M, "tol": tol, "error": None,
                                 "ms": round((time.perf_counter() - t0) * 1e3, 2), "note": str(exc)[:160]})
                    print(f"[adaptive] {name} {rows[-1]}", file=sys.stderr, flush=True)
                    continue
                ms = (time.perf_counter() - t0) * 1e3
                fin = bool(torch.isfinite(yT).all())
                err = float(torch.linalg.vector_norm(yT - ref)) / nref if fin else None
                na, nr = rec["n_accepted"], rec["n_rejected"]
                rows.append({"M": M, "tol": tol, "accepted": na, "rejected": nr, "rok_steps": 3 * (na + nr),
                             "ms": round(ms, 2), "mean_cfl": round(T / na / h1, 3),
                             "error": float(f"{err:.4e}") if err is not None else None})
                print(f"[adaptive] {name} {rows[-1]}", file=sys.stderr, flush=True)
        out[name] = {"T": T, "h_cfl1": h1, "reference": ref_kind, "rows": rows}
        del g
    return out


def adjoint_ogrid_leg(args):
    """Gradient through a trajectory on the viscous cylinder O-grid of the adaptive
    sweep (128 x 64, isothermal wall, Sutherland viscosity, Roe flux): K = 20
    exact-product ROK4 steps (M = 8, h = 2e-6: the impulsive start of the
    no-slip wall allows no larger fixed step) from the free stream, then the
    discrete adjoint (rok_step_vjp from each stored y_n) of L = the x-momentum of
    the wall row.  Reports forward and adjoint milliseconds per step (HIP events
    over the whole sweep) and the directional derivative of L along a random
    direction against central differences of the GPU forward trajectory (best of
    a sweep of steps)."""
    import numpy as np
    import torch

    import rok_inputs as ri
    from paper_1607_06834_amd import Rok

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    fs = ri.freestream(mach=0.3)
    tw = (1.4 - 1.0) * (fs[3] - 0.5 * fs[1] ** 2 / fs[0]) / fs[0]
    nx, ny = 128, 64
    pb, nodes = ri.cylinder_ogrid(nx, ny, radius=0.5, far=20.0, recon="first", flux="roe", cluster=10.0)
    pb = dict(pb, physics="ns", mu=0.01, sutherland=0.4, t_ref=1.0)
    g = Rok(pb, "fp64")
    g.set_ogrid(*nodes, fs, t_wall=tw)
    y0 = torch.tensor(np.tile(np.asarray(fs, dtype=np.float64)[:, None], (1, nx * ny)).reshape(-1), device=dev)
    tab = ri.rok4_tableau()
    K, M, h = 20, 8, 2e-6
    c = torch.zeros_like(y0)
    c[nx * ny:nx * ny + nx] = 1.0            # x-momentum of the wall row j = 0

    def forward(y):
        ys = [y]
        for _ in range(K):
            ys.append(g.step(ys[-1], h, tab, M, mode="tangent"))
        return ys

    def backward(ys):
        yb = c.clone()
        for k in range(K - 1, -1, -1):
            yb = g.step_vjp(ys[k], yb, h, tab, M)
        return yb

    backward(forward(y0))                    # warm-up
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(stream)
    ys = forward(y0)
    e[1].record(stream)
    grad = backward(ys)
    e[2].record(stream)
    torch.cuda.synchronize()
    fwd, bwd = e[0].elapsed_time(e[1]) / K, e[1].elapsed_time(e[2]) / K
    d = torch.tensor(ri.random_direction(g.N, seed=21), device=dev) * y0.abs()
    exact = float(torch.dot(grad, d))
    errs = {}
    for eps in (1e-4, 1e-5, 1e-6):
        lp = float(torch.dot(c, forward(y0 + eps * d)[-1]))
        lm = float(torch.dot(c, forward(y0 - eps * d)[-1]))
        fd = (lp - lm) / (2 * eps)
        errs[eps] = abs(fd - exact) / abs(exact)
    best = min(errs, key=errs.get)
    out = {"grid": f"{nx}x{ny}", "steps": K, "M": M, "h": h, "forward_exact_ms_per_step": round(fwd, 3),
           "step_vjp_ms_per_step": round(bwd, 3), "ratio": round(bwd / fwd, 3),
           "directional_derivative": exact, "central_difference_relerr": float(f"{errs[best]:.3g}"),
           "best_eps": best, "finite": bool(torch.isfinite(grad).all())}
    print(f"[adjoint-ogrid] {out}", file=sys.stderr, flush=True)
    return out


def eigs_leg(args):
    """Stiffness diagnostic (rok_eigs): the 12 largest-magnitude eigenvalues of J at
    the free stream on the cylinder O-grids of the adaptive sweep (inviscid with
    wall cells of 2.5e-5 and 6.2e-7, viscous with 1.5e-4), with the restarts used,
    the number converged (relative residual 1e-8) and the time of the call."""
    import time

    import numpy as np
    import torch

    import rok_inputs as ri
    from paper_1607_06834_amd import Rok

    dev = torch.device("cuda", 0)
    fs = ri.freestream(mach=0.3)
    y0 = np.tile(np.asarray(fs, dtype=np.float64)[:, None], (1, 128 * 64)).reshape(-1)
    tw = (1.4 - 1.0) * (fs[3] - 0.5 * fs[1] ** 2 / fs[0]) / fs[0]
    out = {}
    for name, cluster, ns in (("inviscid_wall_2.5e-5", 12.0, False), ("inviscid_wall_6.2e-7", 16.0, False),
                              ("viscous_wall_1.5e-4", 10.0, True)):
        pb, nodes = ri.cylinder_ogrid(128, 64, radius=0.5, far=20.0, recon="first", flux="roe", cluster=cluster)
        if ns:
            pb = dict(pb, physics="ns", mu=0.01, sutherland=0.4, t_ref=1.0)
        g = Rok(pb, "fp64")
        g.set_ogrid(*nodes, fs, t_wall=tw)
        y = torch.tensor(y0, device=dev)
        v0 = torch.tensor(ri.random_direction(g.N, seed=11), device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vals, res, restarts, conv = g.eigs(y, v0, k=12, m=40, max_restarts=300, tol=1e-8)
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"eigenvalues": [[round(float(v.real), 3), round(float(v.imag), 3)] for v in vals],
                     "restarts": restarts, "converged": conv, "ms": round(ms, 1)}
        print(f"[eigs] {name} {out[name]}", file=sys.stderr, flush=True)
    return out


def _oracle_step_rate(pb, w, tab, cfl, threads, budget_s):
    """Steps/s of the oracle (as it stands) on one configuration with `threads` threads:
    steps from the seeded state until budget_s has passed (at least one)."""
    import numpy as np
    import torch

    import rok_inputs as ri
    from oracle import fv, rok

    torch.set_num_threads(threads)
    y0 = ri.tgv_state(pb) if pb["physics"] == "ns" else ri.vortex_state(pb)
    h = ri.cfl_step(pb, y0, cfl)
    P = fv.Problem(n=pb["n"], lo=pb["lo"], hi=pb["hi"], physics=pb["physics"], recon=pb["recon"],
                   gamma=pb["gamma"], mu=pb["mu"], prandtl=pb["prandtl"])
    f, mv = rok.fv_system(P, "fd" if w["jvp"] == "fd" else "exact")
    y = torch.from_numpy(np.asarray(y0, dtype=np.float64))
    steps, t0 = 0, time.perf_counter()
    while True:
        rok.rok_step(f, mv, tab, w["M"], h, y)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            return steps, el


def _lscpu():
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "NUMA node(s)")
    out = {}
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keep:
            out[k.strip()] = v.strip()
    try:
        out["usable_cpus"] = len(os.sched_getaffinity(0))
    except OSError:
        pass
    return out


def cpu_leg(args, pb, y0, w, tab, h):
    """The oracle on the host's cores.  Large grids take the oracle minutes per
    step (256^3: about ten), so the sample is one configuration of the same
    physics, discretisation, Krylov dimension and CFL number on a smaller grid,
    and the rate is scaled by the ratio of unknowns (every part of the step is
    linear in N).  All threads the process may use, then one thread on a grid
    with half the cells per direction."""
    import torch

    import rok_inputs as ri

    N = ri.size(pb)
    threads = torch.get_num_threads()
    D = len(pb["n"])
    nvar = D + 2
    # sample grid: cells per direction so that the sample has at most ~4.5 M unknowns (an oracle step
    # then takes 10-30 s on 8-16 threads), a multiple of 8; the one-thread sample halves it
    ns = min(int(pb["n"][0]), int((4.5e6 / nvar) ** (1.0 / D)) // 8 * 8)
    sample = dict(pb, n=tuple([ns] * D))
    one = dict(pb, n=tuple([ns // 2] * D))
    steps, el = _oracle_step_rate(sample, w, tab, w["cfl"], threads, args.cpu_seconds)
    ns = ri.size(sample)
    s1, e1 = _oracle_step_rate(one, w, tab, w["cfl"], 1, args.cpu_seconds)
    n1 = ri.size(one)
    torch.set_num_threads(threads)
    grid = "x".join(str(x) for x in sample["n"])
    grid1 = "x".join(str(x) for x in one["n"])
    return {"value": round(steps / el * ns / N, 6), "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} oracle ROK step(s) of the same configuration on a {grid} grid ({ns} unknowns, "
                      f"{el:.1f} s, {threads} threads), rate scaled by {ns}/{N} unknowns",
            "one_thread": {"value": round(s1 / e1 * n1 / N, 7), "unit": "steps/s",
                           "sample": f"{s1} step(s) on {grid1} ({n1} unknowns, {e1:.1f} s), scaled by {n1}/{N}"},
            "lscpu": _lscpu()}


def fp32_leg(args, stream=None):
    """The precision form on the headline workload: FP32 residual and tangent
    products, FP64 Krylov, solve and accumulation; its rate (same K steps
    from the seeded state) and one step's error against the FP64 GPU step
    with exact products from the same state (whose full-size parity with the
    oracle is tested at sampled indices), beside the plain FP64 + FD step's."""
    import torch

    import rok_inputs as ri
    from paper_1607_06834_amd import Rok

    pb, y0, w = ri.workload("tgv256_3d")
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y0, w["cfl"])
    res = gpu_leg(args, pb, y0, w, tab, h, rooflines=False)
    dev = torch.device("cuda", 0)
    yd = torch.tensor(y0, device=dev)
    g32 = Rok(pb, "fp32")
    s32 = g32.step(yd, h, tab, w["M"], "exact").clone()
    del g32
    g64 = Rok(pb, "fp64")
    ref = g64.step(yd, h, tab, w["M"], "exact").clone()
    fd = g64.step(yd, h, tab, w["M"], "fd")
    nref = float(torch.linalg.vector_norm(ref))
    e32 = float(torch.linalg.vector_norm(s32 - ref)) / nref
    efd = float(torch.linalg.vector_norm(fd - ref)) / nref
    del g64, s32, ref, fd
    return {"value": round(1000.0 / res["ms_per_step"], 3), "unit": "steps/s",
            "ms_per_step": round(res["ms_per_step"], 4), "dtype": "f32-residual/f64-krylov", "jvp": "tangent",
            "flags": res["flags"], "M_eff": res["M_eff"],
            "step_error_vs_fp64_exact": float(f"{e32:.3e}"), "fp64_fd_step_error_vs_fp64_exact": float(f"{efd:.3e}")}


def secondary_leg(args):
    """The 1024^2 MUSCL vortex (M = 16, FD products, CFL 10), its rate and resident-MGS roofline."""
    import rok_inputs as ri

    pb, y0, w = ri.workload("vortex1024_muscl")
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y0, w["cfl"])
    sub = argparse.Namespace(**vars(args))
    sub.workload = "vortex1024_muscl"
    sub.traffic = None
    res = gpu_leg(sub, pb, y0, w, tab, h)
    return {"value": round(1000.0 / res["ms_per_step"], 3), "unit": "steps/s", "ms_per_step": round(res["ms_per_step"], 4),
            "config": {"grid": "1024x1024", "physics": "euler", "recon": "muscl", "krylov_M": 16, "jvp": "fd",
                       "cfl": 10.0, "N": ri.size(pb)},
            "flags": res["flags"], "roofline": _dominant(res, w, tab), "arnoldi_step": res["arnoldi_step"],
            "roofline_jvp": res["roofline_jvp"], "roofline_residual": res["roofline_residual"]}


def _dominant(res, w, tab):
    """The roofline entry of the kernel that takes the most time per step: the
    Arnoldi unit (per-pass kernel x passes, or the columns), the product kernel
    (M launches) or the residual (s launches), by their live launch times."""
    if not res.get("roofline"):
        return None
    M, s = w["M"], tab["s"]
    cands = []
    arn = res["roofline"]
    if "slope" in arn.get("timing", ""):
        cands.append((arn["avg_launch_ms"] * M * (M - 1) / 2, arn))
    else:
        cands.append((arn["avg_launch_ms"] * M, arn))
    for key, count in (("roofline_jvp", M), ("roofline_residual", s)):
        ent = res.get(key)
        if ent:
            cands.append((ent["avg_launch_ms"] * count, ent))
    ms, ent = max(cands, key=lambda c: c[0])
    return dict(ent, ms_per_step=round(ms, 3), share_of_step=round(ms / res["ms_per_step"], 4))


PMC_SETS = ("FETCH_SIZE", "WRITE_SIZE", "SQ_INSTS_VALU SQ_WAVES")


def build_traffic(workload, cdir, out_path):
    """Counter figures per launch of the roofline kernels from three rocprofv3
    runs of `bench.py --workload W --roofline-only --no-cpu-baseline
    --kernel-reps 4`, one per entry of PMC_SETS, written to
    cdir/pmc_<W>_<set>/run_counter_collection.csv.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read
    for the run's calibration copy of one state vector (8 N bytes read and
    written; the copy kernel reads twice what it moves), averaged over the
    dispatches of each kernel.  An Arnoldi column of the one-reduce path is its
    four kernels (k_ls_dots, k_ls_solve, k_ls_update, k_normalize): their
    bytes summed over the run and divided by the number of columns (one
    k_ls_solve per column).  Each entry carries the hash of the kernel sources
    (run this on the tree the counters were taken on); bench.py reports no
    traffic for a kernel changed since."""
    import collections
    import csv

    import rok_inputs as ri
    pb, _, w = ri.workload(workload)
    N = ri.size(pb)

    def load(tag):
        agg = collections.defaultdict(list)
        path = os.path.join(cdir, f"pmc_{workload}_{tag.replace(' ', '_')}", "run_counter_collection.csv")
        with open(path) as fh:
            for r in csv.DictReader(fh):
                agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
        return agg

    F, W, V = (load(t) for t in PMC_SETS)

    def vals(agg, prefix, counter):
        out = []
        for (k, c), v in agg.items():
            if k.startswith(prefix) and c == counter:
                out += v
        return out

    cf = vals(F, "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    cw = vals(W, "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    cf, cw = sum(cf) / len(cf), sum(cw) / len(cw)
    vec_kib = 8 * N / 1024
    fs, ws = vec_kib / cf, vec_kib / cw
    cmd = ("timeout -s KILL 240 rocprofv3 --pmc {} --output-format csv -d gpurun_out/pmc_{}_{} -o run -- "
           "python bench.py --workload {} --roofline-only --no-cpu-baseline --kernel-reps 4")
    rec = {"workload": workload, "N": N,
           "method": "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, one counter per run, KiB per dispatch averaged "
                     "over the dispatches, each scaled by what it reads for a copy of one state vector (8 N bytes "
                     "read, 8 N written) in the same run; SQ_INSTS_VALU and SQ_WAVES in a third run; written by "
                     f"python bench.py --workload {workload} --traffic-from gpurun_out",
           "commands": [cmd.format(t, workload, t.replace(" ", "_"), workload) for t in PMC_SETS],
           "calibration": {"kernel": f"__amd_rocclr_copyBuffer, {8 * N / 2 ** 20:.0f} MiB",
                           "fetch_kib": round(cf, 2), "write_kib": round(cw, 2),
                           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)},
           "source_hash": "sha256 of the listed kernel sources with comments and white space removed "
                          "(bench._source_hash)"}
    m = w["M"]
    col_alg = sum((j + 2) * 8 * N + (8 * N if j + 1 < m else 0) for j in range(m)) / m
    D = len(pb["n"])
    ns = "true" if pb["physics"] == "ns" else "false"
    single = {"mgs_pass": ("void rok::k_red<true, false>", KRED_SOURCES, 24 * N),
              "mgs_column": (f"void rok::k_mgs_resident<{m}>", MGS_SOURCES, col_alg)}
    res = f"void rok::k_residual<{D}, 1, {ns}, 0, 0, "
    if w["precision"] == "fp64" and D == 3 and pb["n"][0] % 16 == 0 and pb["n"][1] % 16 == 0:
        # 3-D FP64 MUSCL on columns of 16 x 16 cells: the column-marching kernel
        fl = 1 if pb.get("flux", "rusanov") == "roe" else 0
        single["fd_jvp"] = (f"void rok::k_res3z<{ns}, {fl}, 1>", RESIDUAL_SOURCES, 32 * N)
        single["residual"] = (f"void rok::k_res3z<{ns}, {fl}, 0>", RESIDUAL_SOURCES, 16 * N)
    elif w["precision"] == "fp64":
        single["fd_jvp"] = (res + "double, 1, double", RESIDUAL_SOURCES, 32 * N)
        single["residual"] = (res + "double, 0, double", RESIDUAL_SOURCES, 16 * N)
    else:   # the API's FP32 products and residual write FP32
        single["tangent"] = (res + "rok::Dual<float>, 2, float", RESIDUAL_SOURCES, 20 * N)
        single["residual"] = (res + "float, 0, float", RESIDUAL_SOURCES, 12 * N)
    for key, (kn, src, alg) in single.items():
        f = vals(F, kn, "FETCH_SIZE")
        if not f:
            continue
        wr, vi, wv = vals(W, kn, "WRITE_SIZE"), vals(V, kn, "SQ_INSTS_VALU"), vals(V, kn, "SQ_WAVES")
        fa, wa = sum(f) / len(f), sum(wr) / len(wr)
        hbm = fa * 1024 * fs + wa * 1024 * ws
        rec[key] = {"kernel": kn, "dispatches": len(f), "fetch_kib_avg": round(fa, 1), "write_kib_avg": round(wa, 1),
                    "hbm_bytes_per_launch": int(hbm), "alg_bytes_per_launch": int(alg),
                    "over_algorithmic": round(hbm / alg - 1, 4), "source_sha256_16": _source_hash(src),
                    "valu_insts_per_launch": int(sum(vi) / len(vi)), "waves_per_launch": int(sum(wv) / len(wv))}
    ncol = len(vals(F, "rok::k_ls_solve", "FETCH_SIZE"))
    if ncol:
        parts = ("void rok::k_ls_dots<", "rok::k_ls_solve", "void rok::k_ls_update<", "rok::k_normalize")
        tf = sum(sum(vals(F, k, "FETCH_SIZE")) for k in parts)
        tw = sum(sum(vals(W, k, "WRITE_SIZE")) for k in parts)
        tv = sum(sum(vals(V, k, "SQ_INSTS_VALU")) for k in parts)
        hbm = (tf * 1024 * fs + tw * 1024 * ws) / ncol
        kb = _ls_column_bytes(N, m)
        rec["ls_column"] = {"kernel": "one-reduce Gram-Schmidt column: " + ", ".join(p.split("::")[-1].rstrip("<")
                                                                                      for p in parts),
                            "columns": ncol, "fetch_kib_avg": round(tf / ncol, 1), "write_kib_avg": round(tw / ncol, 1),
                            "hbm_bytes_per_launch": int(hbm), "alg_bytes_per_launch": int(col_alg),
                            "kernel_bytes_per_launch": int(kb), "over_algorithmic": round(hbm / col_alg - 1, 4),
                            "over_kernel_bytes": round(hbm / kb - 1, 4), "source_sha256_16": _source_hash(LS_SOURCES),
                            "valu_insts_per_launch": int(tv / ncol)}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def main():
    args = parse()
    if args.traffic_from:
        out = _traffic_path(args)
        build_traffic(args.workload, args.traffic_from, out)
        print(f"wrote {out}")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the path has no multi-GPU form",
              file=sys.stderr)
        sys.exit(2)
    import rok_inputs as ri

    pb, y0, w = ri.workload(args.workload)
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y0, w["cfl"])
    res = gpu_leg(args, pb, y0, w, tab, h)
    print(f"[bench] {args.workload}: {res['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    dominant = _dominant(res, w, tab)
    extra = not (args.no_secondary or args.roofline_only) and args.workload == "tgv256_3d_fp64"
    f32 = fp32_leg(args) if extra else None
    sec = secondary_leg(args) if extra else None
    eq = None if (args.no_equal_error or args.roofline_only) else {"2d": equal_error_leg(args, 2),
                                                                    "3d": equal_error_leg(args, 3)}
    ksw = krylov_sweep_leg(args) if (args.krylov_sweep and not args.roofline_only) else None
    ada = adaptive_leg(args) if (args.adaptive and not args.roofline_only) else None
    eig = eigs_leg(args) if (args.eigs and not args.roofline_only) else None
    adj_og = adjoint_ogrid_leg(args) if (args.adjoint_ogrid and not args.roofline_only) else None
    cpu = None if (args.no_cpu_baseline or args.roofline_only) else cpu_leg(args, pb, y0, w, tab, h)
    n = "x".join(str(x) for x in pb["n"])
    wl = {"tgv256_3d_fp64": "tgv256_3d"}.get(args.workload, args.workload)
    line = {
        "metric": "ROK steps/sec",
        "value": round(1000.0 / res["ms_per_step"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["precision"] == "fp64" else "f32-residual/f64-krylov",
        "data": "synthetic",
        "config": {"workload": wl, "grid": n, "physics": pb["physics"], "recon": pb["recon"],
                   "flux": "rusanov", "krylov_M": w["M"], "stages": tab["s"], "jvp": w["jvp"],
                   "precision": w["precision"], "cfl": w["cfl"], "h": h, "N": ri.size(pb),
                   "timed_steps": ("trajectory" if args.chain else
                                   "K full ROK steps, each from the seeded initial state (the per-step work does "
                                   "not depend on the state)")},
        "status": {"flags": res["flags"], "M_eff": res["M_eff"], "finite": res["finite"]},
        "roofline": dominant,
        "roofline_arnoldi": res.get("roofline"),
        "arnoldi_step": res.get("arnoldi_step"),
        "roofline_jvp": res.get("roofline_jvp"),
        "roofline_residual": res.get("roofline_residual"),
        "fp32_tangent": f32,
        "secondary": {"vortex1024_muscl": sec} if sec else None,
        "adjoint": res.get("adjoint"),
        "equal_error": eq,
        "krylov_sweep": ksw,
        "adaptive": ada,
        "eigs": eig,
        "adjoint_ogrid": adj_og,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
