// C-ABI of librok: argument validation, workspace carving and the launch
// sequences of the residual, Jacobian-vector product, Arnoldi and ROK step
// (declared and documented in include/rok.h).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"

struct rok_ctx {
    rok_problem pb;
    rok::Geom G;
    int mgs_path;
};

namespace {

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

rok_status hip_status(hipError_t e) {
    if (e == hipSuccess) return ROK_OK;
    if (e == hipErrorNotSupported) return ROK_EUNSUPPORTED;
    return ROK_EHIP;
}

#define ROK_TRY(expr)                            \
    do {                                         \
        hipError_t _e = (expr);                  \
        if (_e != hipSuccess) return hip_status(_e); \
    } while (0)

bool fp32(const rok_ctx* c) { return c->pb.precision == ROK_FP32_RESIDUAL; }

// The adjoint kernels cover Euler and Navier-Stokes physics on every grid, in FP64.
bool adjoint_supported(const rok_ctx* c) {
    return !fp32(c);
}

rok::ResArgs plain_args(const double* y, void* out) {
    rok::ResArgs A{};
    A.y = y;
    A.out = out;
    return A;
}

// w = J(y) v into a double vector (internal use).  FD reads eps from eps_dev.
hipError_t jvp_into(const rok_ctx* c, const double* y, const double* fy, const double* v, double* w, int mode,
                    const double* eps_dev, double eps, hipStream_t st, const int* gate = nullptr, int gate_col = 0,
                    int* status = nullptr, const int* stop = nullptr, const double* vscale = nullptr) {
    rok::ResArgs A{};
    A.vscale = vscale;
    A.status = status;
    A.stop = stop;
    A.gate = gate;
    A.gate_col = gate_col;
    A.y = y;
    A.v = v;
    A.f0 = fy;
    A.eps_dev = eps_dev;
    A.eps = eps;
    A.out = w;
    int kind = (mode == ROK_JVP_FD) ? 1 : 2;
    return rok::launch_residual(c->G, c->pb.recon, c->pb.physics == ROK_NS, fp32(c), kind, true, A, st);
}

// How the Arnoldi columns are orthogonalised: modified Gram-Schmidt pass by
// pass or with w resident on chip (the same bits), or the one-reduce form
// (w too large for the chip; M <= 24).  `mgs_only`: a forward
// that the step adjoint differentiates (the adjoint is that of modified
// Gram-Schmidt).  -1: the requested path is not available.
enum { ORTHO_PASS = 0, ORTHO_RESIDENT = 1, ORTHO_ONE_REDUCE = 2 };

int pick_ortho(const rok_ctx* c, int M, bool mgs_only) {
    const long N = c->G.N;
    const bool resident_ok = rok::mgs_resident_per(N) > 0 && rok::mgs_resident_available();
    if (mgs_only) return (c->mgs_path != ROK_MGS_PER_PASS && resident_ok) ? ORTHO_RESIDENT : ORTHO_PASS;
    switch (c->mgs_path) {
        case ROK_MGS_PER_PASS: return ORTHO_PASS;
        case ROK_MGS_RESIDENT: return resident_ok ? ORTHO_RESIDENT : -1;
        case ROK_MGS_ONE_REDUCE: return rok::lowsync_supported(M) ? ORTHO_ONE_REDUCE : -1;
        default:
            if (resident_ok) return ORTHO_RESIDENT;
            if (rok::lowsync_supported(M)) return ORTHO_ONE_REDUCE;
            return ORTHO_PASS;
    }
}

// Arnoldi (Sec. 2.2.2) into V (N x M columns), H inside W.  deferred: with
// the one-reduce form, the columns after the first are left unnormalised,
// column c holding v_c / W.sig[c] (the caller applies the scales; rok_step's
// own basis), which saves a pass over each new column.
hipError_t arnoldi_core(const rok_ctx* c, const rok::Work& W, const double* y, const double* fy, int M, int mode,
                        double eps, double* V, hipStream_t st, bool mgs_only = false, bool deferred = false) {
    const long N = c->G.N;
    const double* epsp = nullptr;
    const int ortho = pick_ortho(c, M, mgs_only);
    if (ortho < 0) return hipErrorNotSupported;
    deferred = deferred && ortho == ORTHO_ONE_REDUCE;
    hipError_t e;
    if (mode == ROK_JVP_FD && !(eps > 0.0)) {
        e = rok::launch_norm_eps(W, y, nullptr, N, st);  // unit Arnoldi vectors: ||v_j|| = 1
        if (e != hipSuccess) return e;
        epsp = W.scal + 1;
    }
    e = rok::launch_start_basis(W, fy, N, V, st);
    if (e != hipSuccess) return e;
    for (int j = 0; j < M; ++j) {
        double* vj = V + (long)j * N;
        // after a breakdown (stop word set) column j was never written: the product is skipped
        e = jvp_into(c, y, fy, vj, W.w, mode, epsp, eps, st, nullptr, 0, W.ints + 2, W.ints + 1,
                     deferred ? W.sig + j : nullptr);
        if (e != hipSuccess) return e;
        double* vnext = (j + 1 < M) ? V + (long)(j + 1) * N : nullptr;
        if (ortho == ORTHO_RESIDENT)
            e = rok::launch_mgs_resident(W, W.w, V, N, M, j, vnext, st);
        else if (ortho == ORTHO_ONE_REDUCE)
            e = rok::launch_ls_column(W, W.w, V, N, M, j, vnext, st, deferred);
        else
            e = rok::launch_mgs_column(W, W.w, V, N, M, j, vnext, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The launch sequence of one ROK step into the carved workspace W.
hipError_t step_core(const rok_ctx* c, const rok_tableau* tab, int M, int mode, double h, const double* y_n,
                     double* y_np1, const rok::Work& W, hipStream_t st, bool mgs_only = false) {
    const int s = tab->s;
    const long N = c->G.N;
    const bool ns = c->pb.physics == ROK_NS;
    hipError_t e = rok::launch_init(W, M, s, st);
    if (e != hipSuccess) return e;
    {   // F_1 = f(y_n)
        rok::ResArgs A = plain_args(y_n, W.F);
        A.status = W.ints + 2;
        e = rok::launch_residual(c->G, c->pb.recon, ns, fp32(c), 0, true, A, st);
        if (e != hipSuccess) return e;
    }
    // the one-reduce basis is kept unnormalised (scales W.sig) inside the step
    const bool deferred = M > 0 && pick_ortho(c, M, mgs_only) == ORTHO_ONE_REDUCE;
    const double* sig = deferred ? W.sig : nullptr;
    if (M > 0) {
        e = arnoldi_core(c, W, y_n, W.F, M, mode, 0.0, W.V, st, mgs_only, deferred);
        if (e != hipSuccess) return e;
        e = rok::launch_lu(W, M, h * tab->gamma, st);
        if (e != hipSuccess) return e;
    }
    // Y_i = y_n + sum_{j<i} alpha_ij k_j is written by the recovery of k_{i-1}
    // (into k_i's slot, free until k_i is formed), in the residual's order
    auto has_terms = [&](int i) {
        for (int j = 0; j < i; ++j)
            if (tab->alpha[i * ROK_MAX_STAGES + j] != 0.0) return true;
        return false;
    };
    for (int i = 0; i < s; ++i) {
        double* Fi = W.F + (long)i * N;
        if (i > 0) {
            rok::ResArgs A = plain_args(has_terms(i) ? W.K + (long)i * N : y_n, Fi);
            A.status = W.ints + 2;
            e = rok::launch_residual(c->G, c->pb.recon, ns, fp32(c), 0, true, A, st);
            if (e != hipSuccess) return e;
        }
        if (M > 0) {
            // with the one-reduce basis (not the library's bitwise path) the first stage's
            // projection is taken from F_1 = beta v_0 instead of a pass over the basis
            e = (i == 0 && deferred) ? rok::launch_project_first(W, M, st) : rok::launch_project(W, W.V, Fi, N, M, st);
            if (e != hipSuccess) return e;
            double grow[ROK_MAX_STAGES];
            for (int j = 0; j < ROK_MAX_STAGES; ++j) grow[j] = (j < i) ? tab->gam[i * ROK_MAX_STAGES + j] : 0.0;
            e = rok::launch_lambda(W, M, i, grow, h, st, sig);
            if (e != hipSuccess) return e;
        }
        if (i + 1 < s && has_terms(i + 1))
            e = rok::launch_recover(W, W.V, Fi, N, M, i, h, W.K + (long)i * N, y_n, W.K, 0, nullptr, st, sig,
                                    W.K + (long)(i + 1) * N, tab->alpha + (i + 1) * ROK_MAX_STAGES);
        else if (i + 1 < s)
            e = rok::launch_recover(W, W.V, Fi, N, M, i, h, W.K + (long)i * N, nullptr, nullptr, 0, nullptr, st, sig);
        else
            e = rok::launch_recover(W, W.V, Fi, N, M, i, h, y_np1, y_n, W.K, s, tab->b, st, sig);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Reverse sweep of one step whose forward quantities sit in W (exact
// products): ybar_n = (d y_{n+1} / d y_n)^T ybar_np1.
hipError_t step_adjoint(const rok_ctx* c, const rok_tableau* tab, int M, double h, const double* y_n,
                        const double* ybar_np1, double* ybar_n, const rok::Work& W, const rok::AdjWork& A,
                        hipStream_t st) {
    const int s = tab->s;
    const long N = c->G.N;
    const int Mm = M > 0 ? M : 1;
    const int recon = c->pb.recon;
    hipError_t e = rok::launch_adj_init(A, M, s, st);
    if (e != hipSuccess) return e;
    e = rok::launch_adj_seed(A, ybar_np1, ybar_n, N, s, tab->b, st);
    if (e != hipSuccess) return e;
    rok::Work Wp = W;      // projection partials of V^T kbar go to the adjoint's buffer
    Wp.partials = A.part;
    for (int i = s - 1; i >= 0; --i) {
        double* kbi = A.kbar + (long)i * N;
        if (M > 0) {
            e = rok::launch_project(Wp, W.V, kbi, N, M, st);
            if (e != hipSuccess) return e;
        }
        double grow[ROK_MAX_STAGES];
        for (int j = 0; j < ROK_MAX_STAGES; ++j) grow[j] = (j < i) ? tab->gam[i * ROK_MAX_STAGES + j] : 0.0;
        if (M > 0) {
            e = rok::launch_small_rev(W, A, Mm, i, grow, h, st);
            if (e != hipSuccess) return e;
        }
        double* Fbar = (i == 0) ? A.Fbar0 : A.FB;
        e = rok::launch_vbar_stage(W, A, Mm, i, h, Fbar, N, i == s - 1, st);
        if (e != hipSuccess) return e;
        if (i > 0) {   // Y_i = y_n + sum_j alpha_ij k_j;  ybar += J(Y_i)^T Fbar, kbar_j += alpha_ij (...)
            const double* arow = tab->alpha + i * ROK_MAX_STAGES;
            e = rok::launch_stage_state(y_n, W.K, arow, i, A.Yt, N, st);
            if (e != hipSuccess) return e;
            e = rok::launch_vjp(c->G, recon, A.Yt, nullptr, A.FB, A.Ybar, nullptr, 0, st);
            if (e != hipSuccess) return e;
            e = rok::launch_scatter(A, A.Ybar, ybar_n, arow, i, N, st);
            if (e != hipSuccess) return e;
        }
    }
    if (M > 0) {
        e = rok::launch_abar_to_hbar(W, A, Mm, h * tab->gamma, st);
        if (e != hipSuccess) return e;
        const bool resident = c->mgs_path != ROK_MGS_PER_PASS && rok::mgs_rev_resident_available(N);
        for (int j = M - 1; j >= 0; --j) {
            const double* vj = W.V + (long)j * N;
            // J v_j is needed only where the final MGS iterate cannot be taken
            // as h_{j+1,j} v_{j+1}: the basis' last column
            e = jvp_into(c, y_n, nullptr, vj, W.w, ROK_JVP_TANGENT, nullptr, 0.0, st, W.ints, j);
            if (e != hipSuccess) return e;
            e = rok::launch_arnoldi_rev_col(W, A, M, j, N, resident, st);
            if (e != hipSuccess) return e;
            // w = J(y) v_j:  vbar_j += J^T wbar,  ybar += d/dt [J(y + t v_j)^T wbar]
            e = rok::launch_vjp(c->G, recon, y_n, vj, A.wbar, A.Vbar + (long)j * N, ybar_n, 1, st, W.ints, j);
            if (e != hipSuccess) return e;
        }
        e = rok::launch_beta_rev(W, A, N, st);
        if (e != hipSuccess) return e;
    }
    // F_1 = f(y_n)
    return rok::launch_vjp(c->G, recon, y_n, nullptr, A.Fbar0, ybar_n, nullptr, 1, st);
}

}  // namespace

extern "C" {

rok_status rok_create(const rok_problem* p, rok_ctx** out) {
    if (!p || !out) return ROK_EINVAL;
    *out = nullptr;
    if (p->ndim != 2 && p->ndim != 3) return ROK_EINVAL;
    long ncell = 1;
    for (int d = 0; d < p->ndim; ++d) {
        if (p->n[d] < 1 || !(p->hi[d] > p->lo[d])) return ROK_EINVAL;
        ncell *= p->n[d];
        if (ncell > (1L << 31)) return ROK_EINVAL;
    }
    if (p->physics != ROK_EULER && p->physics != ROK_NS) return ROK_EINVAL;
    if (p->recon != ROK_FIRST_ORDER && p->recon != ROK_MUSCL_MINMOD) return ROK_EINVAL;
    if (p->flux != ROK_RUSANOV && p->flux != ROK_ROE) return ROK_EINVAL;
    if (p->precision != ROK_FP64 && p->precision != ROK_FP32_RESIDUAL) return ROK_EINVAL;
    if (!(p->gamma > 1.0) || !(p->mu >= 0.0) || !(p->prandtl > 0.0)) return ROK_EINVAL;
    if (!(p->sutherland >= 0.0) || !isfinite(p->sutherland)) return ROK_EINVAL;
    if (p->sutherland > 0.0 && (!(p->t_ref > 0.0) || !isfinite(p->t_ref))) return ROK_EINVAL;
    rok_ctx* c = new (std::nothrow) rok_ctx;
    if (!c) return ROK_EINVAL;
    c->pb = *p;
    c->mgs_path = ROK_MGS_AUTO;
    rok::Geom& G = c->G;
    memset(&G, 0, sizeof(G));
    G.D = p->ndim;
    for (int d = 0; d < 3; ++d) G.n[d] = (d < p->ndim) ? p->n[d] : 1;
    G.nvar = p->ndim + 2;
    G.ncell = ncell;
    G.N = (long)G.nvar * ncell;
    for (int d = 0; d < p->ndim; ++d) {
        double dx = (p->hi[d] - p->lo[d]) / p->n[d];
        G.invdx[d] = 1.0 / dx;
        G.hinv[d] = 0.5 * G.invdx[d];
    }
    G.g = p->gamma;
    G.gm1 = p->gamma - 1.0;
    G.mu = p->physics == ROK_NS ? p->mu : 0.0;
    G.c23mu = (2.0 / 3.0) * G.mu;
    G.kappa = G.mu * p->gamma / ((p->gamma - 1.0) * p->prandtl);
    G.flux = p->flux;
    G.suth = (p->physics == ROK_NS && p->sutherland > 0.0) ? 1 : 0;
    G.suth_s = p->sutherland;
    G.suth_one_s = 1.0 + p->sutherland;
    G.t_ref = p->sutherland > 0.0 ? p->t_ref : 1.0;
    G.kden = (p->gamma - 1.0) * p->prandtl;
    *out = c;
    return ROK_OK;
}

void rok_destroy(rok_ctx* c) { delete c; }

size_t rok_grid_metric_bytes(const rok_ctx* c) {
    if (!c || c->pb.ndim != 2 || c->pb.n[0] < 2 || c->pb.n[1] < 2) return 0;
    return sizeof(double) * 9 * (size_t)c->G.ncell;
}

rok_status rok_set_grid(rok_ctx* c, const double* xn, const double* yn, double* metrics, void* stream) {
    if (!c) return ROK_EINVAL;
    if (!xn && !yn && !metrics) {
        c->G.metric = nullptr;
        c->G.ogrid = 0;
        return ROK_OK;
    }
    if (c->pb.ndim != 2) return ROK_EUNSUPPORTED;
    if (c->pb.n[0] < 2 || c->pb.n[1] < 2) return ROK_EINVAL;
    if (!xn || !yn || !metrics || !aligned(xn, 8) || !aligned(yn, 8) || !aligned(metrics, 8)) return ROK_EINVAL;
    const double Lx = c->pb.hi[0] - c->pb.lo[0], Ly = c->pb.hi[1] - c->pb.lo[1];
    ROK_TRY(rok::launch_metrics(xn, yn, c->pb.n[0], c->pb.n[1], Lx, Ly, metrics, (hipStream_t)stream));
    c->G.metric = metrics;
    c->G.ogrid = 0;
    return ROK_OK;
}

size_t rok_ogrid_metric_bytes(const rok_ctx* c) {
    if (!c || c->pb.ndim != 2 || c->pb.n[0] < 2 || c->pb.n[1] < 2) return 0;
    return sizeof(double) * (9 * (size_t)c->G.ncell + 4 * (size_t)c->pb.n[0]);
}

rok_status rok_set_ogrid(rok_ctx* c, const double* xn, const double* yn, const double* freestream, double t_wall,
                         double* metrics, void* stream) {
    if (!c) return ROK_EINVAL;
    if (c->pb.ndim != 2) return ROK_EUNSUPPORTED;
    if (c->pb.physics == ROK_NS && (!(t_wall > 0.0) || !isfinite(t_wall))) return ROK_EINVAL;
    if (!xn || !yn || !metrics || !freestream || !aligned(xn, 8) || !aligned(yn, 8) || !aligned(metrics, 8))
        return ROK_EINVAL;
    const double r = freestream[0], E = freestream[3];
    const double ke = (freestream[1] * freestream[1] + freestream[2] * freestream[2]) / r;
    if (!(r > 0.0) || !isfinite(E) || !((c->pb.gamma - 1.0) * (E - 0.5 * ke) > 0.0)) return ROK_EINVAL;
    if (c->pb.n[0] < 2 || c->pb.n[1] < 2) return ROK_EINVAL;
    ROK_TRY(rok::launch_metrics_ogrid(xn, yn, c->pb.n[0], c->pb.n[1], metrics, (hipStream_t)stream));
    c->G.metric = metrics;
    c->G.ogrid = 1;
    c->G.t_wall = t_wall;
    for (int m = 0; m < 4; ++m) c->G.uinf[m] = freestream[m];
    return ROK_OK;
}

rok_status rok_set_mgs_path(rok_ctx* c, int path) {
    if (!c || (path != ROK_MGS_AUTO && path != ROK_MGS_PER_PASS && path != ROK_MGS_RESIDENT &&
               path != ROK_MGS_ONE_REDUCE))
        return ROK_EINVAL;
    c->mgs_path = path;
    return ROK_OK;
}

size_t rok_state_size(const rok_ctx* c) { return c ? (size_t)c->G.N : 0; }

size_t rok_workspace_bytes(const rok_ctx* c, int M, int s) {
    if (!c || M < 0 || s < 0 || s > ROK_MAX_STAGES) return 0;
    int Mc = M > ROK_MAX_M ? ROK_MAX_M : M;
    if ((long)Mc > c->G.N) Mc = (int)c->G.N;
    return rok::work_bytes(c->G.N, Mc, s, s > 0);
}

rok_status rok_residual(rok_ctx* c, const double* y, void* F, void* stream) {
    if (!c || !y || !F || !aligned(y, 8) || !aligned(F, fp32(c) ? 4 : 8)) return ROK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    rok::ResArgs A = plain_args(y, F);
    ROK_TRY(rok::launch_residual(c->G, c->pb.recon, c->pb.physics == ROK_NS, fp32(c), 0, !fp32(c), A, st));
    return ROK_OK;
}

rok_status rok_residual_split(rok_ctx* c, const double* y, void* F_inv, void* F_visc, void* stream) {
    const size_t a = fp32(c) ? 4 : 8;
    if (!c || !y || !F_inv || !F_visc || F_inv == F_visc || !aligned(y, 8) || !aligned(F_inv, a) ||
        !aligned(F_visc, a))
        return ROK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // inviscid part: the Euler kernel of the same discretisation
    rok::ResArgs A = plain_args(y, F_inv);
    ROK_TRY(rok::launch_residual(c->G, c->pb.recon, false, fp32(c), 0, !fp32(c), A, st));
    if (c->pb.physics != ROK_NS) {
        ROK_TRY(rok::launch_zero(F_visc, c->G.N * (long)a, st));
        return ROK_OK;
    }
    A.out = F_visc;
    A.viscous_only = 1;
    ROK_TRY(rok::launch_residual(c->G, c->pb.recon, true, fp32(c), 0, !fp32(c), A, st));
    return ROK_OK;
}

namespace {

// Validation shared by rok_jvp and rok_jvp_noalloc.
rok_status jvp_args_ok(const rok_ctx* c, const double* y, const double* fy, const double* v, const void* w,
                       int mode) {
    if (!c || !y || !v || !w || !aligned(y, 8) || !aligned(v, 8) || !aligned(w, fp32(c) ? 4 : 8)) return ROK_EINVAL;
    if (mode != ROK_JVP_FD && mode != ROK_JVP_TANGENT) return ROK_EINVAL;
    if (mode == ROK_JVP_FD) {
        if (fp32(c)) return ROK_EUNSUPPORTED;
        if (!fy || !aligned(fy, 8)) return ROK_EINVAL;
    }
    return ROK_OK;
}

// The launches of rok_jvp once the arguments are valid.  `small` is the
// base of the small workspace layout (header, scalars, reduction
// partials); it is touched only for a finite-difference product with the
// default increment (eps <= 0).
hipError_t jvp_launch(const rok_ctx* c, const double* y, const double* fy, const double* v, void* w, int mode,
                      double eps, void* small, hipStream_t st) {
    rok::ResArgs A{};
    A.y = y;
    A.v = v;
    A.out = w;
    if (mode == ROK_JVP_TANGENT)
        return rok::launch_residual(c->G, c->pb.recon, c->pb.physics == ROK_NS, fp32(c), 2, !fp32(c), A, st);
    A.f0 = fy;
    if (eps > 0.0) {
        A.eps = eps;
    } else {
        rok::Work W = rok::carve(small, 0, 0, 0, false);
        hipError_t e = rok::launch_init(W, 0, 0, st);
        if (e == hipSuccess) e = rok::launch_norm_eps(W, y, v, c->G.N, st);
        if (e != hipSuccess) return e;
        A.eps_dev = W.scal + 1;
    }
    return rok::launch_residual(c->G, c->pb.recon, c->pb.physics == ROK_NS, false, 1, true, A, st);
}

}  // namespace

rok_status rok_jvp(rok_ctx* c, const double* y, const double* fy, const double* v, void* w, int mode, double eps,
                   void* work, size_t wbytes, void* stream) {
    rok_status r = jvp_args_ok(c, y, fy, v, w, mode);
    if (r != ROK_OK) return r;
    if (mode == ROK_JVP_FD && !(eps > 0.0)) {
        size_t need = rok::work_bytes(c->G.N, 0, 0, false);
        if (!work || !aligned(work, 256) || wbytes < need) return ROK_EINVAL;
    }
    ROK_TRY(jvp_launch(c, y, fy, v, w, mode, eps, work, (hipStream_t)stream));
    return ROK_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free rok_jvp.  The default finite-difference increment needs two
// grid-wide norms, whose reduction partials, header and scalars live in a
// caller workspace in rok_jvp; rok_jvp_noalloc keeps them in `scratch`, a
// file-scope device array of fixed size (every device the library runs on
// holds one copy until the process ends).  In host code `scratch` names a
// host-side stand-in, so its device address is looked up once per device,
// with that device current, and only that address is passed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kJvpScratchBytes = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[kJvpScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];   // device address of `scratch` per device (null until looked up)

// The current device's copy of `scratch` (looked up on its first use on that device).
hipError_t current_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

rok_status rok_jvp_noalloc(rok_ctx* c, const double* y, const double* fy, const double* v, void* w, int mode,
                           double eps, void* stream) {
    rok_status r = jvp_args_ok(c, y, fy, v, w, mode);
    if (r != ROK_OK) return r;
    void* base = nullptr;
    if (mode == ROK_JVP_FD && !(eps > 0.0)) {
        if (rok::work_small_bytes(0, 0) > kJvpScratchBytes) return ROK_EINVAL;
        ROK_TRY(current_scratch(&base));
    }
    ROK_TRY(jvp_launch(c, y, fy, v, w, mode, eps, base, (hipStream_t)stream));
    return ROK_OK;
}

rok_status rok_arnoldi(rok_ctx* c, const double* y, const double* fy, int M, int mode, double eps, double* V,
                       double* H, int* M_eff, void* work, size_t wbytes, void* stream) {
    if (!c || !y || !fy || !V || !H || !M_eff) return ROK_EINVAL;
    if (!aligned(y, 8) || !aligned(fy, 8) || !aligned(V, 8) || !aligned(H, 8) || !aligned(M_eff, 4)) return ROK_EINVAL;
    if (mode != ROK_JVP_FD && mode != ROK_JVP_TANGENT) return ROK_EINVAL;
    if (M < 1 || M > ROK_MAX_M) return ROK_EINVAL;
    if ((long)M > c->G.N) M = (int)c->G.N;
    if (mode == ROK_JVP_FD && fp32(c)) return ROK_EUNSUPPORTED;
    size_t need = rok::work_bytes(c->G.N, M, 0, false);
    if (!work || !aligned(work, 256) || wbytes < need) return ROK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    rok::Work W = rok::carve(work, c->G.N, M, 0, false);
    ROK_TRY(rok::launch_init(W, M, 0, st));
    ROK_TRY(arnoldi_core(c, W, y, fy, M, mode, eps, V, st));
    ROK_TRY(rok::launch_copy_h(W, M, H, M_eff, st));
    return ROK_OK;
}

rok_status rok_step(rok_ctx* c, const rok_tableau* tab, int M, int mode, double h, const double* y_n, double* y_np1,
                    void* work, size_t wbytes, void* stream) {
    if (!c || !tab || !y_n || !y_np1 || y_n == y_np1) return ROK_EINVAL;
    if (!aligned(y_n, 8) || !aligned(y_np1, 8)) return ROK_EINVAL;
    if (tab->s < 1 || tab->s > ROK_MAX_STAGES) return ROK_EINVAL;
    if (mode != ROK_JVP_FD && mode != ROK_JVP_TANGENT) return ROK_EINVAL;
    if (M < 0 || M > ROK_MAX_M || !(h == h)) return ROK_EINVAL;
    if ((long)M > c->G.N) M = (int)c->G.N;
    if (M > 0 && mode == ROK_JVP_FD && fp32(c)) return ROK_EUNSUPPORTED;
    size_t need = rok::work_bytes(c->G.N, M, tab->s, true);
    if (!work || !aligned(work, 256) || wbytes < need) return ROK_EINVAL;
    rok::Work W = rok::carve(work, c->G.N, M, tab->s, true);
    ROK_TRY(step_core(c, tab, M, mode, h, y_n, y_np1, W, (hipStream_t)stream));
    return ROK_OK;
}

rok_status rok_error_norm(rok_ctx* c, const double* y_n, const double* y_a, const double* y_b, double rtol,
                          double atol, double scale, double* err, void* work, size_t wbytes, void* stream) {
    if (!c || !y_n || !y_a || !y_b || !err) return ROK_EINVAL;
    if (!aligned(y_n, 8) || !aligned(y_a, 8) || !aligned(y_b, 8) || !aligned(err, 8)) return ROK_EINVAL;
    if (!(rtol >= 0.0) || !(atol >= 0.0) || !(rtol + atol > 0.0) || !isfinite(rtol) || !isfinite(atol))
        return ROK_EINVAL;
    if (!(scale > 0.0) || !isfinite(scale)) return ROK_EINVAL;
    size_t need = rok::work_bytes(c->G.N, 0, 0, false);
    if (!work || !aligned(work, 256) || wbytes < need) return ROK_EINVAL;
    rok::Work W = rok::carve(work, c->G.N, 0, 0, false);
    ROK_TRY(rok::launch_error_norm(W, y_n, y_a, y_b, c->G.N, rtol, atol, scale, err, (hipStream_t)stream));
    return ROK_OK;
}

namespace {
constexpr double kAdaptSafety = 0.9, kAdaptFmin = 0.2, kAdaptFmax = 4.0;

size_t al256h(size_t b) { return (b + 255) & ~(size_t)255; }

// The controller's next macro step (safety * err^(-1/(p+1)), clamped).
double adapt_next(double H, double err, int order, bool after_reject) {
    const double fmax = after_reject ? 1.0 : kAdaptFmax;
    double fac;
    if (err == 0.0) {
        fac = fmax;
    } else {
        fac = kAdaptSafety * pow(err, -1.0 / (double)(order + 1));
        if (fac < kAdaptFmin) fac = kAdaptFmin;
        if (fac > fmax) fac = fmax;
    }
    return H * fac;
}
}  // namespace

size_t rok_adaptive_workspace_bytes(const rok_ctx* c, int M, int s) {
    if (!c || M < 0 || s < 1 || s > ROK_MAX_STAGES) return 0;
    int Mc = M > ROK_MAX_M ? ROK_MAX_M : M;
    if ((long)Mc > c->G.N) Mc = (int)c->G.N;
    return al256h(rok::work_bytes(c->G.N, Mc, s, true)) + 3 * al256h(sizeof(double) * (size_t)c->G.N) + 256;
}

rok_status rok_integrate_adaptive(rok_ctx* c, const rok_tableau* tab, int M, int mode, int order, double T, double H0,
                                  double rtol, double atol, int max_steps, double* y, rok_adaptive_stats* stats,
                                  double* history, int history_cap, void* work, size_t wbytes, void* stream) {
    if (!c || !tab || !y || !stats || !aligned(y, 8)) return ROK_EINVAL;
    if (tab->s < 1 || tab->s > ROK_MAX_STAGES) return ROK_EINVAL;
    if (mode != ROK_JVP_FD && mode != ROK_JVP_TANGENT) return ROK_EINVAL;
    if (M < 0 || M > ROK_MAX_M || order < 1 || order > 16 || max_steps < 0) return ROK_EINVAL;
    if (!(T >= 0.0) || !isfinite(T) || !(H0 > 0.0) || !isfinite(H0)) return ROK_EINVAL;
    if (!(rtol >= 0.0) || !(atol >= 0.0) || !(rtol + atol > 0.0) || !isfinite(rtol) || !isfinite(atol))
        return ROK_EINVAL;
    if (history_cap < 0 || (history_cap > 0 && !history)) return ROK_EINVAL;
    if ((long)M > c->G.N) M = (int)c->G.N;
    if (M > 0 && mode == ROK_JVP_FD && fp32(c)) return ROK_EUNSUPPORTED;
    const long N = c->G.N;
    const size_t step_b = al256h(rok::work_bytes(N, M, tab->s, true));
    const size_t vec = al256h(sizeof(double) * (size_t)N);
    if (!work || !aligned(work, 256) || wbytes < step_b + 3 * vec + 256) return ROK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    char* p = (char*)work;
    rok::Work W = rok::carve(p, N, M, tab->s, true);
    double* buf[3] = {(double*)(p + step_b), (double*)(p + step_b + vec), (double*)(p + step_b + 2 * vec)};
    double* err_dev = (double*)(p + step_b + 3 * vec);
    // cur (the accepted state) and the three trial states always occupy four distinct buffers
    double* cur = y;
    double* y_full = buf[0];
    double* y_mid = buf[1];
    double* y_half = buf[2];
    const double c_scale = (double)((1L << order) - 1);
    double t = 0.0, H = H0;
    bool after_reject = false;
    int acc = 0, rej = 0, rec = 0;
    for (int it = 0; it < max_steps; ++it) {
        if (t >= T || !(t + H > t)) break;   // done, or the step no longer advances t
        const bool last = t + H >= T;
        if (last) H = T - t;
        ROK_TRY(step_core(c, tab, M, mode, H, cur, y_full, W, st));
        ROK_TRY(step_core(c, tab, M, mode, 0.5 * H, cur, y_mid, W, st));
        ROK_TRY(step_core(c, tab, M, mode, 0.5 * H, y_mid, y_half, W, st));
        ROK_TRY(rok::launch_error_norm(W, cur, y_half, y_full, N, rtol, atol, c_scale, err_dev, st));
        double err = 0.0;
        ROK_TRY(hipMemcpyAsync(&err, err_dev, sizeof(double), hipMemcpyDeviceToHost, st));
        ROK_TRY(hipStreamSynchronize(st));
        if (!isfinite(err)) err = INFINITY;
        const bool ok = err <= 1.0;
        if (rec < history_cap) {
            history[4 * rec + 0] = t;
            history[4 * rec + 1] = H;
            history[4 * rec + 2] = err;
            history[4 * rec + 3] = ok ? 1.0 : 0.0;
            ++rec;
        }
        double H_next;
        if (ok) {
            ++acc;
            t = last ? T : t + H;
            // the two-half-step result becomes the state; the old state's buffer takes its role
            double* old = cur;
            cur = y_half;
            y_half = old;
            H_next = adapt_next(H, err, order, after_reject);
            after_reject = false;
        } else {
            ++rej;
            H_next = isfinite(err) ? adapt_next(H, err, order, true) : H * kAdaptFmin;
            after_reject = true;
        }
        H = H_next;
    }
    if (cur != y) ROK_TRY(hipMemcpyAsync(y, cur, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, st));
    ROK_TRY(hipStreamSynchronize(st));
    stats->t = t;
    stats->h_next = H;
    stats->accepted = acc;
    stats->rejected = rej;
    stats->recorded = rec;
    return ROK_OK;
}

namespace {
struct EigLayout {
    size_t work, vec, basis, coef, hb, total;
};

EigLayout eig_layout(long N, int m) {
    EigLayout L;
    L.work = al256h(rok::work_bytes(N, m + 1, 0, false));
    L.vec = al256h(sizeof(double) * (size_t)N);
    L.basis = L.vec * (size_t)(m + 1);
    L.coef = al256h(sizeof(double) * (size_t)(m + 1) * (size_t)(m + 1));
    L.hb = al256h(sizeof(double) * (size_t)(m + 2) * (size_t)(m + 1));
    L.total = L.work + 2 * L.basis + L.coef + L.hb;
    return L;
}

bool eig_args_ok(const rok_ctx* c, int k, int m) {
    return c && m >= 3 && m <= ROK_EIGS_MAX_M && k >= 1 && k + 2 <= m && (long)m + 1 <= c->G.N;
}
}  // namespace

size_t rok_eigs_workspace_bytes(const rok_ctx* c, int k, int m) {
    if (!eig_args_ok(c, k, m)) return 0;
    return eig_layout(c->G.N, m).total;
}

rok_status rok_eigs(rok_ctx* c, const double* y, const double* v0, int k, int m, int max_restarts, double tol,
                    double* re, double* im, double* resid, int* info, void* work, size_t wbytes, void* stream) {
    if (!eig_args_ok(c, k, m) || !y || !v0 || !re || !im || !resid || !info) return ROK_EINVAL;
    if (!aligned(y, 8) || !aligned(v0, 8) || max_restarts < 0 || !(tol > 0.0) || !isfinite(tol)) return ROK_EINVAL;
    const long N = c->G.N;
    const int Mp = m + 1;
    const EigLayout L = eig_layout(N, m);
    if (!work || !aligned(work, 256) || wbytes < L.total) return ROK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    char* p = (char*)work;
    rok::Work W = rok::carve(p, N, Mp, 0, false);
    double* V = (double*)(p + L.work);
    double* Vo = (double*)(p + L.work + L.basis);
    double* Cd = (double*)(p + L.work + 2 * L.basis);
    // a second pass of every Gram-Schmidt column writes its coefficients here
    rok::Work W2 = W;
    W2.H = (double*)(p + L.work + 2 * L.basis + L.coef);
    // the resident kernel holds a column of H in LDS (at most ROK_MAX_M entries): larger bases
    // take the pass-by-pass kernels
    const bool resident = c->mgs_path != ROK_MGS_PER_PASS && Mp <= ROK_MAX_M && rok::mgs_resident_per(N) > 0 &&
                          rok::mgs_resident_available();
    if (c->mgs_path == ROK_MGS_RESIDENT && !resident) return ROK_EUNSUPPORTED;
    auto mgs = [&](const rok::Work& Wx, int j, double* vnext) -> hipError_t {
        return resident ? rok::launch_mgs_resident(Wx, Wx.w, V, N, Mp, j, vnext, st)
                        : rok::launch_mgs_column(Wx, Wx.w, V, N, Mp, j, vnext, st);
    };
    // orthonormalise W.w against V[:, 0..j] into V[:, j+1] by modified Gram-Schmidt,
    // twice (the second pass on the normalised result restores the orthogonality
    // that one pass loses when w is nearly in the span, as near convergence)
    auto orthonormalise = [&](int j) -> hipError_t {
        double* vnext = V + (long)(j + 1) * N;
        hipError_t e = mgs(W, j, vnext);
        if (e == hipSuccess)
            e = hipMemcpyAsync(W.w, vnext, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = mgs(W2, j, vnext);
        return e;
    };
    // column j of the Arnoldi process: w = J v_j (exact product), then orthonormalised
    auto column = [&](int j) -> hipError_t {
        hipError_t e = jvp_into(c, y, nullptr, V + (long)j * N, W.w, ROK_JVP_TANGENT, nullptr, 0.0, st);
        if (e != hipSuccess) return e;
        return orthonormalise(j);
    };
    std::vector<double> Hd((size_t)(Mp + 1) * Mp), Hb((size_t)(Mp + 1) * Mp), Hh((size_t)(m + 1) * m, 0.0);
    int ints[3] = {0, 0, 0};
    // both passes' coefficients and the status words to the host
    auto fetch = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(Hd.data(), W.H, sizeof(double) * Hd.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(Hb.data(), W2.H, sizeof(double) * Hb.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ints, W.ints, sizeof(ints), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    };
    // combined coefficient of column j: w = sum_i (h_ij + b h'_ij) v_i + b b' v_{j+1}
    // (h, b = h_{j+1,j}: first pass; h', b': second pass on w / b)
    auto hd = [&](int i, int j) {
        const double b = Hd[(size_t)(j + 1) * Mp + j];
        const double b2 = Hb[(size_t)(j + 1) * Mp + j];
        if (i == j + 1) return b * b2;
        return Hd[(size_t)i * Mp + j] + b * Hb[(size_t)i * Mp + j];
    };
    auto hh = [&](int i, int j) -> double& { return Hh[(size_t)i * m + j]; };

    ROK_TRY(rok::launch_init(W2, Mp, 0, st));
    ROK_TRY(rok::launch_init(W, Mp, 0, st));
    ROK_TRY(rok::launch_start_basis(W, v0, N, V, st));
    for (int j = 0; j < m; ++j) ROK_TRY(column(j));
    ROK_TRY(fetch());
    if (ints[2] & ROK_FLAG_ZERO_RHS) return ROK_EINVAL;   // v0 = 0
    for (int j = 0; j < m; ++j)
        for (int i = 0; i <= j + 1; ++i) hh(i, j) = hd(i, j);
    int meff = ints[1] ? ints[0] : m;   // a breakdown leaves an invariant subspace of dimension meff

    std::vector<double> wr(m), wi(m), Qacc((size_t)m * m), Hw((size_t)m * m), Cc((size_t)Mp * Mp);
    std::vector<int> idx(m);
    int restarts = 0;
    for (;;) {
        const int n = meff < m ? meff : m;
        if (!rok::dense::hessenberg_eigenvalues(n, Hh.data(), m, wr.data(), wi.data())) return ROK_EHIP;
        for (int i = 0; i < n; ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.begin() + n, [&](int a, int b) {
            return std::hypot(wr[a], wi[a]) > std::hypot(wr[b], wi[b]);
        });
        const double hlast = n < m ? 0.0 : hh(m, m - 1);
        int conv = 0;
        for (int t = 0; t < k; ++t) {
            if (t >= n) {
                re[t] = im[t] = 0.0;
                resid[t] = INFINITY;
                continue;
            }
            const int i = idx[t];
            re[t] = wr[i];
            im[t] = wi[i];
            resid[t] = (n < m) ? 0.0 : rok::dense::ritz_residual(m, Hh.data(), m, hlast, wr[i], wi[i]);
            if (resid[t] <= tol * std::hypot(wr[i], wi[i])) ++conv;
        }
        info[0] = restarts;
        info[1] = conv;
        if (conv == k || n < m || restarts >= max_restarts) break;
        // Ritz values of a real H come in conjugate pairs: pair them up (partner[i] = i for real ones)
        std::vector<int> partner(m);
        for (int i = 0; i < m; ++i) partner[i] = i;
        {
            std::vector<int> pos, neg;
            for (int i = 0; i < m; ++i) {
                if (fabs(wi[i]) <= 1e-12 * std::hypot(wr[i], wi[i])) continue;
                (wi[i] > 0.0 ? pos : neg).push_back(i);
            }
            std::vector<char> taken(m, 0);
            for (int i : pos) {
                int best = -1;
                double bd = INFINITY;
                for (int j : neg) {
                    if (taken[j]) continue;
                    const double dd = std::hypot(wr[j] - wr[i], wi[j] + wi[i]);
                    if (dd < bd) { bd = dd; best = j; }
                }
                if (best >= 0) {
                    taken[best] = 1;
                    partner[i] = best;
                    partner[best] = i;
                }
            }
        }
        // wanted: the k largest and the partners of complex ones among them (kk values);
        // the others are the exact shifts, each real one once and each pair as one double
        // shift, so that the shifts' total degree is m - kk
        std::vector<char> want(m, 0);
        for (int t = 0; t < k; ++t) want[idx[t]] = want[partner[idx[t]]] = 1;
        int kk = 0;
        for (int i = 0; i < m; ++i) kk += want[i];
        if (kk + 2 > m) break;   // no room to restart: keep the current estimate
        std::fill(Qacc.begin(), Qacc.end(), 0.0);
        for (int i = 0; i < m; ++i) Qacc[(size_t)i * m + i] = 1.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Hw[(size_t)i * m + j] = hh(i, j);
        for (int t = 0; t < m; ++t) {
            const int i = idx[t];
            if (want[i]) continue;
            if (partner[i] == i) {
                rok::dense::shift_step(m, Hw.data(), m, Qacc.data(), wr[i], 0.0, false);
            } else if (wi[i] > 0.0) {
                rok::dense::shift_step(m, Hw.data(), m, Qacc.data(), wr[i], wi[i], true);
            }
        }
        // new basis [V Q[:, 0..kk-1], f_kk] with f_kk = (V Q)[:, kk] H+[kk, kk-1] + v_m h[m, m-1] Q[m-1, kk-1]
        std::fill(Cc.begin(), Cc.end(), 0.0);
        for (int cc = 0; cc < kk; ++cc)
            for (int i = 0; i < m; ++i) Cc[(size_t)cc * Mp + i] = Qacc[(size_t)i * m + cc];
        const double hk = Hw[(size_t)kk * m + kk - 1];
        for (int i = 0; i < m; ++i) Cc[(size_t)kk * Mp + i] = hk * Qacc[(size_t)i * m + kk];
        Cc[(size_t)kk * Mp + m] = hh(m, m - 1) * Qacc[(size_t)(m - 1) * m + kk - 1];
        ROK_TRY(hipMemcpyAsync(Cd, Cc.data(), sizeof(double) * (size_t)Mp * (kk + 1), hipMemcpyHostToDevice, st));
        ROK_TRY(rok::launch_combine(V, N, Mp, Cd, kk + 1, Vo, st));
        std::swap(V, Vo);
        // orthonormalise f_kk against the kept vectors (its projections correct column kk-1 of H), then extend
        ROK_TRY(rok::launch_init(W2, Mp, 0, st));
        ROK_TRY(rok::launch_init(W, Mp, 0, st));
        ROK_TRY(hipMemcpyAsync(W.w, V + (long)kk * N, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, st));
        ROK_TRY(orthonormalise(kk - 1));
        for (int j = kk; j < m; ++j) ROK_TRY(column(j));
        ROK_TRY(fetch());
        std::fill(Hh.begin(), Hh.end(), 0.0);
        for (int j = 0; j + 1 < kk; ++j)
            for (int i = 0; i <= j + 1; ++i) hh(i, j) = Hw[(size_t)i * m + j];
        for (int i = 0; i < kk; ++i) hh(i, kk - 1) = Hw[(size_t)i * m + kk - 1] + hd(i, kk - 1);
        hh(kk, kk - 1) = hd(kk, kk - 1);
        for (int j = kk; j < m; ++j)
            for (int i = 0; i <= j + 1; ++i) hh(i, j) = hd(i, j);
        meff = ints[1] ? ints[0] : m;
        ++restarts;
    }
    return ROK_OK;
}

size_t rok_step_vjp_workspace_bytes(const rok_ctx* c, int M, int s) {
    if (!c || M < 0 || s < 1 || s > ROK_MAX_STAGES) return 0;
    int Mc = M > ROK_MAX_M ? ROK_MAX_M : M;
    if ((long)Mc > c->G.N) Mc = (int)c->G.N;
    return rok::work_bytes(c->G.N, Mc, s, true) + rok::adj_bytes(c->G.N, Mc, s);
}

rok_status rok_step_vjp(rok_ctx* c, const rok_tableau* tab, int M, double h, const double* y_n,
                        const double* ybar_np1, double* ybar_n, double* y_np1, void* work, size_t wbytes,
                        void* stream) {
    if (!c || !tab || !y_n || !ybar_np1 || !ybar_n) return ROK_EINVAL;
    if (!aligned(y_n, 8) || !aligned(ybar_np1, 8) || !aligned(ybar_n, 8) || (y_np1 && !aligned(y_np1, 8)))
        return ROK_EINVAL;
    if (ybar_n == y_n || ybar_n == ybar_np1 || (y_np1 && (y_np1 == y_n || y_np1 == ybar_n || y_np1 == ybar_np1)))
        return ROK_EINVAL;
    if (tab->s < 1 || tab->s > ROK_MAX_STAGES) return ROK_EINVAL;
    if (M < 0 || M > ROK_MAX_M || !(h == h)) return ROK_EINVAL;
    if (!adjoint_supported(c)) return ROK_EUNSUPPORTED;
    if ((long)M > c->G.N) M = (int)c->G.N;
    const int s = tab->s;
    const long N = c->G.N;
    const size_t fwd = rok::work_bytes(N, M, s, true);
    if (!work || !aligned(work, 256) || wbytes < fwd + rok::adj_bytes(N, M, s)) return ROK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    rok::Work W = rok::carve(work, N, M, s, true);
    rok::AdjWork A = rok::adj_carve((char*)work + fwd, N, M, s);
    ROK_TRY(step_core(c, tab, M, ROK_JVP_TANGENT, h, y_n, y_np1 ? y_np1 : A.Yt, W, st, true));
    ROK_TRY(step_adjoint(c, tab, M, h, y_n, ybar_np1, ybar_n, W, A, st));
    return ROK_OK;
}

size_t rok_step_vjp_adjoint_bytes(const rok_ctx* c, int M, int s) {
    if (!c || M < 0 || s < 1 || s > ROK_MAX_STAGES) return 0;
    int Mc = M > ROK_MAX_M ? ROK_MAX_M : M;
    if ((long)Mc > c->G.N) Mc = (int)c->G.N;
    return rok::adj_bytes(c->G.N, Mc, s);
}

rok_status rok_step_vjp_stored(rok_ctx* c, const rok_tableau* tab, int M, double h, const double* y_n,
                               const double* ybar_np1, double* ybar_n, void* fwd_work, size_t fwd_bytes,
                               void* adj_work, size_t adj_bytes, void* stream) {
    if (!c || !tab || !y_n || !ybar_np1 || !ybar_n) return ROK_EINVAL;
    if (!aligned(y_n, 8) || !aligned(ybar_np1, 8) || !aligned(ybar_n, 8)) return ROK_EINVAL;
    if (ybar_n == y_n || ybar_n == ybar_np1) return ROK_EINVAL;
    if (tab->s < 1 || tab->s > ROK_MAX_STAGES) return ROK_EINVAL;
    if (M < 0 || M > ROK_MAX_M || !(h == h)) return ROK_EINVAL;
    if (!adjoint_supported(c)) return ROK_EUNSUPPORTED;
    if ((long)M > c->G.N) M = (int)c->G.N;
    const int s = tab->s;
    const long N = c->G.N;
    if (!fwd_work || !aligned(fwd_work, 256) || fwd_bytes < rok::work_bytes(N, M, s, true)) return ROK_EINVAL;
    if (!adj_work || !aligned(adj_work, 256) || adj_bytes < rok::adj_bytes(N, M, s)) return ROK_EINVAL;
    // the forward rok_step of this context orthogonalised its basis by the one-reduce form, whose reverse is not built
    if (M > 0 && pick_ortho(c, M, false) == ORTHO_ONE_REDUCE) return ROK_EUNSUPPORTED;
    rok::Work W = rok::carve(fwd_work, N, M, s, true);
    rok::AdjWork A = rok::adj_carve(adj_work, N, M, s);
    ROK_TRY(step_adjoint(c, tab, M, h, y_n, ybar_np1, ybar_n, W, A, (hipStream_t)stream));
    return ROK_OK;
}

rok_status rok_workspace_init(rok_ctx* c, void* work, size_t wbytes, int M, int s, void* stream) {
    if (!c || !work || !aligned(work, 256) || M < 0 || M > ROK_MAX_M || s < 0 || s > ROK_MAX_STAGES)
        return ROK_EINVAL;
    if ((long)M > c->G.N) M = (int)c->G.N;
    if (wbytes < rok::work_bytes(c->G.N, M, s, s > 0)) return ROK_EINVAL;
    rok::Work W = rok::carve(work, c->G.N, M, s, s > 0);
    ROK_TRY(rok::launch_init(W, M, s, (hipStream_t)stream));
    return ROK_OK;
}

rok_status rok_mgs_column(rok_ctx* c, const double* V, int M, int j, double* w, double* H, double* vnext, void* work,
                          size_t wbytes, void* stream) {
    if (!c || !V || !w || !H || !work || !aligned(V, 8) || !aligned(w, 8) || !aligned(H, 8) || !aligned(work, 256))
        return ROK_EINVAL;
    if (M < 1 || M > ROK_MAX_M || (long)M > c->G.N || j < 0 || j >= M) return ROK_EINVAL;
    if (j + 1 < M && (!vnext || !aligned(vnext, 8))) return ROK_EINVAL;
    if (wbytes < rok::work_bytes(c->G.N, M, 0, false)) return ROK_EINVAL;
    const long N = c->G.N;
    rok::Work W = rok::carve(work, N, M, 0, false);
    W.H = H;
    hipStream_t st = (hipStream_t)stream;
    const int ortho = pick_ortho(c, M, false);   // the orthogonalisation rok_arnoldi takes
    if (ortho < 0) return ROK_EUNSUPPORTED;
    double* vn = (j + 1 < M) ? vnext : nullptr;
    if (ortho == ORTHO_RESIDENT)
        ROK_TRY(rok::launch_mgs_resident(W, w, V, N, M, j, vn, st));
    else if (ortho == ORTHO_ONE_REDUCE)
        ROK_TRY(rok::launch_ls_column(W, w, V, N, M, j, vn, st));
    else
        ROK_TRY(rok::launch_mgs_column(W, w, V, N, M, j, vn, st));
    return ROK_OK;
}

int rok_arnoldi_path(const rok_ctx* c, int M) {
    if (!c || M < 1 || M > ROK_MAX_M) return ROK_EINVAL;
    if ((long)M > c->G.N) M = (int)c->G.N;
    switch (pick_ortho(c, M, false)) {
        case ORTHO_PASS: return ROK_MGS_PER_PASS;
        case ORTHO_RESIDENT: return ROK_MGS_RESIDENT;
        case ORTHO_ONE_REDUCE: return ROK_MGS_ONE_REDUCE;
        default: return ROK_EUNSUPPORTED;
    }
}

rok_status rok_residual_vjp(rok_ctx* c, const double* y, const double* wbar, double* ybar, int accumulate,
                            void* stream) {
    if (!c || !y || !wbar || !ybar || !aligned(y, 8) || !aligned(wbar, 8) || !aligned(ybar, 8)) return ROK_EINVAL;
    if (ybar == y || ybar == wbar) return ROK_EINVAL;
    if (!adjoint_supported(c)) return ROK_EUNSUPPORTED;
    ROK_TRY(rok::launch_vjp(c->G, c->pb.recon, y, nullptr, wbar, ybar, nullptr, accumulate ? 1 : 0,
                            (hipStream_t)stream));
    return ROK_OK;
}

rok_status rok_residual_vjp2(rok_ctx* c, const double* y, const double* v, const double* wbar, double* ybar,
                             double* ybar2, int accumulate, void* stream) {
    if (!c || !y || !v || !wbar || !ybar || !ybar2) return ROK_EINVAL;
    if (!aligned(y, 8) || !aligned(v, 8) || !aligned(wbar, 8) || !aligned(ybar, 8) || !aligned(ybar2, 8))
        return ROK_EINVAL;
    if (ybar == ybar2 || ybar == y || ybar == wbar || ybar == v || ybar2 == y || ybar2 == wbar || ybar2 == v)
        return ROK_EINVAL;
    if (!adjoint_supported(c)) return ROK_EUNSUPPORTED;
    ROK_TRY(rok::launch_vjp(c->G, c->pb.recon, y, v, wbar, ybar, ybar2, accumulate ? 1 : 0, (hipStream_t)stream));
    return ROK_OK;
}

static rok_status read_header(const void* work, int idx, int* out, void* stream) {
    if (!work || !out || !aligned(work, 256)) return ROK_EINVAL;
    int ints[4];
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(ints, work, sizeof(ints), hipMemcpyDeviceToHost, st) != hipSuccess) return ROK_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return ROK_EHIP;
    *out = ints[idx];
    return ROK_OK;
}

rok_status rok_read_status(rok_ctx* c, const void* work, int* host_flags, void* stream) {
    if (!c) return ROK_EINVAL;
    return read_header(work, 2, host_flags, stream);
}

rok_status rok_read_meff(rok_ctx* c, const void* work, int* host_meff, void* stream) {
    if (!c) return ROK_EINVAL;
    return read_header(work, 0, host_meff, stream);
}

const char* rok_strerror(rok_status s) {
    switch (s) {
        case ROK_OK: return "success";
        case ROK_EINVAL: return "invalid argument";
        case ROK_EUNSUPPORTED: return "unsupported option combination";
        case ROK_EHIP: return "HIP launch failure";
        default: return "unknown status";
    }
}

}  // extern "C"
