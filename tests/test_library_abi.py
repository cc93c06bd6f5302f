"""The C-ABI library loads and exports every entry point declared in include/rok.h (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "rok.h")).read()
    return sorted(set(re.findall(r"\b(rok_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["rok_residual", "rok_jvp", "rok_arnoldi", "rok_step", "rok_create", "rok_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1607_06834_amd import rok
    path = rok.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("librok.so not built")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(rok.SYMBOLS) <= set(_declared())


def test_host_validation_without_gpu():
    """rok_create validates the problem on the host (no device call)."""
    from paper_1607_06834_amd import rok
    if not os.path.exists(rok.LIB_PATH):
        pytest.skip("librok.so not built")
    lib = rok.load_library()
    p = rok.RokProblem()
    p.ndim = 4
    ctx = ctypes.c_void_p()
    assert lib.rok_create(ctypes.byref(p), ctypes.byref(ctx)) == rok.ROK_EINVAL
    p.ndim = 2
    p.n[0], p.n[1] = 8, 8
    p.lo[0], p.lo[1] = 0.0, 0.0
    p.hi[0], p.hi[1] = 1.0, 1.0
    p.gamma, p.prandtl = 1.4, 0.72
    assert lib.rok_create(ctypes.byref(p), ctypes.byref(ctx)) == rok.ROK_OK
    assert lib.rok_state_size(ctx) == 4 * 64
    assert lib.rok_workspace_bytes(ctx, 8, 4) > lib.rok_workspace_bytes(ctx, 8, 0) > 0
    assert lib.rok_workspace_bytes(ctx, 8, 9) == 0
    tab = rok.RokTableau()
    tab.s = 0
    assert lib.rok_step(ctx, ctypes.byref(tab), 4, 0, 0.1, ctypes.c_void_p(8), ctypes.c_void_p(16),
                        ctypes.c_void_p(256), 1 << 20, None) == rok.ROK_EINVAL
    st = rok.RokAdaptiveStats()
    assert lib.rok_integrate_adaptive(ctx, ctypes.byref(tab), 4, 0, 4, 1.0, 0.1, 1e-6, 1e-6, 100,
                                      ctypes.c_void_p(8), ctypes.byref(st), None, 0, ctypes.c_void_p(256), 1 << 20,
                                      None) == rok.ROK_EINVAL
    assert lib.rok_error_norm(ctx, ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.c_void_p(24), 0.0, 0.0, 15.0,
                              ctypes.c_void_p(32), ctypes.c_void_p(256), 1 << 20, None) == rok.ROK_EINVAL
    # curvilinear grids: validated on the host (a partial set of pointers; 3-D or Navier-Stokes refused)
    assert lib.rok_grid_metric_bytes(ctx) == 9 * 64 * 8
    assert lib.rok_set_grid(ctx, ctypes.c_void_p(8), None, ctypes.c_void_p(16), None) == rok.ROK_EINVAL
    assert lib.rok_set_grid(ctx, None, None, None, None) == rok.ROK_OK
    assert lib.rok_ogrid_metric_bytes(ctx) == (9 * 64 + 4 * 8) * 8
    bad_fs = (ctypes.c_double * 4)(1.0, 0.0, 0.0, -1.0)          # negative pressure
    assert lib.rok_set_ogrid(ctx, ctypes.c_void_p(8), ctypes.c_void_p(16), bad_fs, 1.0, ctypes.c_void_p(24),
                             None) == rok.ROK_EINVAL
    # eigenvalue estimate: sizes are validated on the host
    assert lib.rok_eigs_workspace_bytes(ctx, 6, 40) > 0
    assert lib.rok_eigs_workspace_bytes(ctx, 9, 10) == 0 and lib.rok_eigs_workspace_bytes(ctx, 0, 10) == 0
    assert lib.rok_eigs_workspace_bytes(ctx, 4, 64) > 0            # past ROK_MAX_M: the pass-by-pass kernels
    assert lib.rok_eigs_workspace_bytes(ctx, 4, 255) > 0 and lib.rok_eigs_workspace_bytes(ctx, 4, 256) == 0  # m + 1 <= N
    assert lib.rok_eigs_workspace_bytes(ctx, 4, 2049) == 0           # past ROK_EIGS_MAX_M (and N)
    # a basis past ROK_MAX_M is orthogonalised pass by pass: an explicit request for the resident kernel is
    # refused before any device work
    assert lib.rok_set_mgs_path(ctx, 2) == rok.ROK_OK                  # ROK_MGS_RESIDENT
    nb = lib.rok_eigs_workspace_bytes(ctx, 4, 100)
    re_, im_, rs_ = (ctypes.c_double * 4)(), (ctypes.c_double * 4)(), (ctypes.c_double * 4)()
    info = (ctypes.c_int * 2)()
    assert lib.rok_eigs(ctx, ctypes.c_void_p(256), ctypes.c_void_p(512), 4, 100, 1, 1e-8, re_, im_, rs_, info,
                        ctypes.c_void_p(1 << 20), nb, None) == rok.ROK_EUNSUPPORTED
    assert lib.rok_set_mgs_path(ctx, 0) == rok.ROK_OK
    re_, im_, rs_ = (ctypes.c_double * 4)(), (ctypes.c_double * 4)(), (ctypes.c_double * 4)()
    inf = (ctypes.c_int * 2)()
    assert lib.rok_eigs(ctx, ctypes.c_void_p(8), ctypes.c_void_p(16), 4, 5, 10, 1e-8, re_, im_, rs_, inf,
                        ctypes.c_void_p(256), 1 << 30, None) == rok.ROK_EINVAL
    lib.rok_destroy(ctx)
    # inviscid flux and Sutherland's law are validated on the host
    for flux, suth, tref, want in ((rok.ROE, 0.0, 1.0, rok.ROK_OK), (2, 0.0, 1.0, rok.ROK_EINVAL),
                                   (0, -0.5, 1.0, rok.ROK_EINVAL), (0, 0.5, 0.0, rok.ROK_EINVAL),
                                   (0, 0.5, 2.0, rok.ROK_OK)):
        p.flux, p.sutherland, p.t_ref = flux, suth, tref
        ctx = ctypes.c_void_p()
        assert lib.rok_create(ctypes.byref(p), ctypes.byref(ctx)) == want, (flux, suth, tref)
        if want == rok.ROK_OK:
            lib.rok_destroy(ctx)
    p.flux, p.sutherland, p.physics, p.mu = 0, 0.0, rok.NS, 0.05
    ctx = ctypes.c_void_p()
    assert lib.rok_create(ctypes.byref(p), ctypes.byref(ctx)) == rok.ROK_OK
    assert lib.rok_grid_metric_bytes(ctx) == 9 * 64 * 8          # Navier-Stokes on curvilinear grids
    ok_fs = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 2.5)
    assert lib.rok_set_ogrid(ctx, ctypes.c_void_p(8), ctypes.c_void_p(16), ok_fs, -1.0, ctypes.c_void_p(24),
                             None) == rok.ROK_EINVAL              # wall temperature must be positive
    lib.rok_destroy(ctx)
    p.ndim, p.n[2], p.hi[2] = 3, 4, 1.0
    ctx = ctypes.c_void_p()
    assert lib.rok_create(ctypes.byref(p), ctypes.byref(ctx)) == rok.ROK_OK
    assert lib.rok_grid_metric_bytes(ctx) == 0
    assert lib.rok_set_grid(ctx, ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.c_void_p(24), None) == \
        rok.ROK_EUNSUPPORTED
    lib.rok_destroy(ctx)
