/*
 * librok -- MI355X (gfx950) implementation of the hot path of the matrix-free
 * Rosenbrock-Krylov (ROK) time integrator for semi-discretised compressible
 * flow, y' = f(y) (Sarshar, Tranquilli, Pickering, McCall, Sandu, Roy,
 * "A numerical investigation of matrix-free implicit time-stepping methods
 * for large CFD simulations", Computers & Fluids 159, 2017).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout.  A state vector has N = nvar * ncell doubles, variable-major,
 * x fastest:  y[((v * nz + k) * ny + j) * nx + i],  nvar = ndim + 2, with the
 * variables [rho, rho*u, rho*v, (rho*w), E] of the conserved form of the
 * Euler / Navier-Stokes equations (Sec. 3.2, eq. 11).
 *
 * Memory.  Every pointer argument of type double* / float* / void* other than
 * the context, the problem and the tableau is DEVICE memory owned by the
 * caller.  The library never allocates or frees device memory and keeps no
 * pointer after a call returns.  Device pointers must be 8-byte aligned;
 * workspaces must be 256-byte aligned.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Every call
 * validates its arguments on the host, enqueues its kernels on `stream` and
 * returns without synchronising; results are ready when the stream is.
 * Calls that share a workspace must not overlap in time.
 *
 * Errors.  A call returns ROK_OK or a negative status:
 *   ROK_EINVAL        bad argument (null / misaligned pointer, size out of
 *                     range, workspace too small); nothing was enqueued;
 *   ROK_EUNSUPPORTED  the combination of options is not built;
 *   ROK_EHIP          a HIP launch failed (hipGetLastError after enqueueing).
 * Numerical events are recorded in a status word inside the workspace and
 * read with rok_read_status (ROK_FLAG_*).
 */
#ifndef ROK_H
#define ROK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rok_ctx rok_ctx;
typedef int rok_status;

enum {
    ROK_OK = 0,
    ROK_EINVAL = -1,
    ROK_EUNSUPPORTED = -2,
    ROK_EHIP = -3
};

enum { ROK_EULER = 0, ROK_NS = 1 };                  /* physics                     */
enum { ROK_FIRST_ORDER = 0, ROK_MUSCL_MINMOD = 1 };  /* reconstruction              */
enum { ROK_RUSANOV = 0, ROK_ROE = 1 };               /* inviscid flux               */
enum { ROK_FP64 = 0, ROK_FP32_RESIDUAL = 1 };        /* precision of f and J v      */
enum { ROK_JVP_FD = 0, ROK_JVP_TANGENT = 1 };        /* Jacobian-vector product     */

/* status-word bits (rok_read_status).  The gas law has no positivity fix
 * (Sec. 3.2: ideal gas, p = (gamma - 1)(E - rho |u|^2 / 2)): a non-physical
 * state is reported, and the arithmetic goes on with it (a square root of a
 * negative pressure gives NaN, which is reported as non-finite). */
enum {
    ROK_FLAG_NONFINITE = 1,   /* a NaN or Inf appeared in a residual or product  */
                              /* output (F_i, J v_j; so also from a NaN in y),    */
                              /* in H, phi or lambda                              */
    ROK_FLAG_BREAKDOWN = 2,   /* Arnoldi stopped early: M_eff < M (invariant space) */
    ROK_FLAG_ZERO_RHS = 4,    /* f(y_n) = 0 exactly: M_eff = 0                       */
    ROK_FLAG_BARRIER = 8,     /* an in-kernel grid barrier timed out (results invalid) */
    ROK_FLAG_NONPHYSICAL = 16 /* a residual or product saw a cell with rho <= 0 or */
                              /* p <= 0 (y_n, a stage state Y_i, or y_n + eps v_j) */
};

/* Orthogonalisation of the Arnoldi columns (rok_set_mgs_path). */
enum { ROK_MGS_AUTO = 0, ROK_MGS_PER_PASS = 1, ROK_MGS_RESIDENT = 2, ROK_MGS_ONE_REDUCE = 3 };

#define ROK_MAX_STAGES 8
#define ROK_MAX_M 64
/* Largest Arnoldi dimension m of the eigenvalue estimate (rok_eigs). */
#define ROK_EIGS_MAX_M 2048

/*
 * The semi-discrete system y' = f(y) of Sec. 2, eq. (1): the compressible
 * Euler (physics = ROK_EULER) or Navier-Stokes (ROK_NS) equations of
 * Sec. 3.2, eq. (11), finite volumes on a periodic cell-centred Cartesian
 * box [lo, hi] with n cells per direction (ndim = 2: n[2] and lo/hi[2] are
 * ignored), first-order or MUSCL (minmod limiter, primitive variables)
 * reconstruction, Rusanov or Roe flux (ROK_ROE: Roe's linearisation with
 * density-weighted averages and Harten's entropy fix, half-width c/8, on the
 * acoustic waves; the paper's residual offers Roe and Van Leer fluxes,
 * Sec. 3.2), viscosity mu, constant or by Sutherland's law
 * mu(T) = mu theta^(3/2) (1 + s) / (theta + s), theta = T / t_ref,
 * s = sutherland, at each face's temperature (T_a + T_b) / 2 with T = p / rho
 * (the paper's cylinder cases set Sutherland's coefficient, Sec. 4.2),
 * conductivity mu(T) gamma / ((gamma - 1) Pr), Prandtl number
 * `prandtl`, ratio of specific heats `gamma`.  With precision =
 * ROK_FP32_RESIDUAL the residual and tangent kernels compute in float while
 * Arnoldi, the reduced solve and all state accumulation stay in double.
 */
typedef struct {
    int ndim;
    int n[3];
    double lo[3];
    double hi[3];
    int physics;
    int recon;
    int flux;
    double gamma;
    double mu;
    double prandtl;
    int precision;
    double sutherland;   /* S / T_ref of Sutherland's law (>= 0; 0: constant mu) */
    double t_ref;        /* temperature p / rho at which the viscosity is mu (> 0 when sutherland > 0) */
} rok_problem;

/*
 * ROK coefficients (Sec. 2.2.2, eq. 9): s stages (1..8); alpha_ij and
 * gamma_ij are stored row-major with leading dimension ROK_MAX_STAGES
 * (alpha[i * ROK_MAX_STAGES + j]) and only the strictly lower triangle
 * j < i < s is read; gamma is the common diagonal; b has s weights.
 * Host memory.
 */
typedef struct {
    int s;
    double alpha[ROK_MAX_STAGES * ROK_MAX_STAGES];
    double gam[ROK_MAX_STAGES * ROK_MAX_STAGES];
    double gamma;
    double b[ROK_MAX_STAGES];
} rok_tableau;

/* Validates *problem and creates a host-only, immutable context.  Allocates
 * no device memory.  ROK_EINVAL on a bad problem (ndim not 2 or 3, n < 1,
 * hi <= lo, gamma <= 1, mu < 0, NS with mu = 0 is allowed). */
rok_status rok_create(const rok_problem* problem, rok_ctx** out);
void rok_destroy(rok_ctx* ctx);

/* Selects how the modified Gram-Schmidt passes of rok_arnoldi / rok_step
 * run: ROK_MGS_PER_PASS launches one kernel per pass (the work vector is
 * streamed through memory); ROK_MGS_RESIDENT runs one cooperative kernel per
 * Arnoldi column with the work vector held in registers (N up to 16 * 2^18 = 4194304);
 * ROK_MGS_AUTO (default) takes the resident kernel when the device and N
 * allow it.  Both produce bit-identical results.  The setting also selects
 * the reverse of the Arnoldi columns in rok_step_vjp: one resident kernel per
 * column for N up to 8 * 2^18 = 2097152 unless ROK_MGS_PER_PASS is set
 * (per-pass kernels otherwise; bit-identical as well).
 * ROK_MGS_ONE_REDUCE (M <= 24) computes the same coefficients from sums
 * against the original work vector, h = (I + L)^{-1} V^T w with L the
 * strictly lower part of V^T V (modified Gram-Schmidt's coefficients in
 * exact arithmetic, written in its inverse compact WY form): two sweeps over
 * the basis per column instead of one per pass, rounded differently (V, H and
 * steps within 1e-12 of modified Gram-Schmidt; with finite-difference
 * products the step is no longer the same bits, since the quotient divides
 * the basis' last-bit differences by eps: see the library's tests for the
 * measured level).  ROK_MGS_AUTO takes it when the resident kernel cannot
 * hold the work vector (N above 4194304) and M <= 24; ROK_MGS_PER_PASS keeps
 * modified Gram-Schmidt pass by pass there (the same bits as the resident
 * kernel and the library's reference arithmetic).  The forward recomputed by
 * rok_step_vjp always takes modified Gram-Schmidt (its reverse is that of
 * modified Gram-Schmidt); rok_step_vjp_stored returns ROK_EUNSUPPORTED where
 * rok_step would have taken the one-reduce form.
 * Changes the context: not to be called while other calls on the same
 * context are being made.  ROK_EINVAL for an unknown path. */
rok_status rok_set_mgs_path(rok_ctx* ctx, int path);

/* The orthogonalisation rok_arnoldi, rok_step and rok_mgs_column take on this
 * context for Krylov dimension M (1..ROK_MAX_M): ROK_MGS_PER_PASS,
 * ROK_MGS_RESIDENT or ROK_MGS_ONE_REDUCE; ROK_EUNSUPPORTED if the path set
 * with rok_set_mgs_path is not available, ROK_EINVAL for a bad argument. */
int rok_arnoldi_path(const rok_ctx* ctx, int M);

/*
 * Curvilinear grids (2-D, n[0], n[1] >= 2): the box [lo, hi] becomes a periodic
 * structured grid with the given nodes (the paper's residual works on
 * curvilinear structured grids, Sec. 3.2).  xn, yn: n[0] * n[1] doubles each,
 * device memory, node (i, j) at j * n[0] + i; node (i + n[0], j) is node (i, j)
 * moved by (hi[0] - lo[0], 0) and node (i, j + n[1]) by (0, hi[1] - lo[1]).
 * Cell (i, j) has the nodes (i, j), (i+1, j), (i+1, j+1), (i, j+1); its faces
 * carry the edge vectors turned by 90 degrees and its area is half the cross
 * product of its diagonals.  The call computes these metrics into `metrics`
 * (rok_grid_metric_bytes(ctx) bytes of device memory owned by the caller, which
 * must stay valid while the context uses it) on `stream`; afterwards the
 * residual, both Jacobian-vector products, rok_arnoldi, rok_step and
 * rok_integrate_adaptive evaluate f on the curvilinear grid: reconstruction in
 * index space, then at each face the states are rotated into the face frame
 * (normal and tangential momentum and velocity), the flux is taken there,
 * rotated back and scaled by the face length, and
 * f_c = sum_d (Fhat_{c-1/2} - Fhat_{c+1/2}) / A_c.  Navier-Stokes physics: face
 * gradients by the chain rule through the face's two grid directions (the
 * index-space difference across the face and the mean of the two cells'
 * central differences along it, with the face vector and the difference of
 * the two cells' centroids, each centroid the mean of its nodes).  All three
 * pointers null: back to the Cartesian grid.  FP64 precision only (the FP32
 * form returns ROK_EUNSUPPORTED); the adjoint entry points return
 * ROK_EUNSUPPORTED.
 */
rok_status rok_set_grid(rok_ctx* ctx, const double* xn, const double* yn, double* metrics, void* stream);

/* Bytes of the metric buffer of rok_set_grid (0 unless 2-D with n[0], n[1] >= 2). */
size_t rok_grid_metric_bytes(const rok_ctx* ctx);

/*
 * An O-grid around a body (2-D, n[0], n[1] >= 2; the paper's cylinder cases use
 * such grids with a wall and a far field, Sec. 4.2): nodes xn, yn of
 * n[0] * (n[1] + 1) doubles each, device memory, node (i, j) at j * n[0] + i for
 * j = 0..n[1] (row 0 on the body, row n[1] on the far-field boundary), periodic
 * in i without offset (node n[0] is node 0).  Cell faces, areas and the flux in
 * the face frame are as for rok_set_grid; along j the face below row 0 is the
 * wall (it carries the first cell's pressure on the wall face vector: a slip
 * wall for ROK_EULER; for ROK_NS also the viscous flux of an isothermal no-slip
 * wall at temperature t_wall, with gradients from the wall values and the
 * first cell through the vector from the wall face's midpoint to that cell's
 * centroid), the face above the last row is the far field (the numerical flux
 * between the last cell's primitive state, in conserved form, and
 * `freestream`; no viscous flux), MUSCL slopes that would reach past either
 * boundary are zero, and index differences along j are one-sided in the
 * boundary rows.
 *   freestream: host, 4 doubles, the conserved free-stream state (rho, rho u,
 *               rho v, E) with rho > 0 and a positive pressure
 *   t_wall:     the wall temperature p / rho (> 0; read for ROK_NS only)
 *   metrics:    rok_ogrid_metric_bytes(ctx) bytes of device memory owned by the
 *               caller (valid while the context uses it)
 * Same restrictions as rok_set_grid; rok_set_grid(ctx, 0, 0, 0, s) returns to
 * the Cartesian grid.
 */
rok_status rok_set_ogrid(rok_ctx* ctx, const double* xn, const double* yn, const double* freestream, double t_wall,
                         double* metrics, void* stream);

/* Bytes of the metric buffer of rok_set_ogrid (0 unless 2-D with n[0], n[1] >= 2). */
size_t rok_ogrid_metric_bytes(const rok_ctx* ctx);

/* N, the length of a state vector. */
size_t rok_state_size(const rok_ctx* ctx);

/* Bytes of workspace needed by rok_jvp / rok_arnoldi (s = 0) or rok_step
 * (s = number of stages) with Krylov dimension M. */
size_t rok_workspace_bytes(const rok_ctx* ctx, int M, int s);

/*
 * F = f(y)  (Sec. 2, eq. 1; Sec. 3.2, eq. 11).  y: N doubles.  F: N doubles,
 * or N floats when the context's precision is ROK_FP32_RESIDUAL.
 */
rok_status rok_residual(rok_ctx* ctx, const double* y, void* F, void* stream);

/*
 * The residual split into its inviscid and viscous parts (eq. 11: the
 * divergence of the inviscid flux and of the viscous stress / heat flux
 * vectors), F_inv + F_visc = f(y) up to the rounding of that one addition:
 *   F_inv  = -sum_d (Fhat_{c+1/2} - Fhat_{c-1/2}) / dx_d  (inviscid flux only)
 *   F_visc =  sum_d (Fv_{c+1/2} - Fv_{c-1/2}) / dx_d      (viscous flux only;
 *            zero for ROK_EULER)
 * Each part is assembled as f is, with the other flux left out.
 *   y: N doubles; F_inv, F_visc: N elements each (double, or float for
 *   ROK_FP32_RESIDUAL), device memory, distinct.
 */
rok_status rok_residual_split(rok_ctx* ctx, const double* y, void* F_inv, void* F_visc, void* stream);

/*
 * w = J(y) v, J = df/dy at y (Sec. 2.3).
 *   mode ROK_JVP_FD:      w = (f(y + eps v) - fy) / eps  (eq. 10); fy = f(y)
 *                         (N doubles); eps > 0 is used as given, eps <= 0
 *                         selects eps = sqrt((1 + ||y||_2) eps_mach) / ||v||_2,
 *                         which needs `work` (rok_workspace_bytes(ctx, 0, 0)).
 *                         FP64 precision only (ROK_EUNSUPPORTED otherwise).
 *   mode ROK_JVP_TANGENT: the exact product (forward-mode derivative of f);
 *                         fy, eps and work are ignored.
 * v: N doubles.  w: N doubles (N floats under ROK_FP32_RESIDUAL).
 */
rok_status rok_jvp(rok_ctx* ctx, const double* y, const double* fy, const double* v, void* w,
                   int mode, double eps, void* work, size_t work_bytes, void* stream);

/*
 * rok_jvp for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same product with the same arguments and
 * results, bit for bit, without `work`.  The default finite-difference
 * increment (mode ROK_JVP_FD, eps <= 0) needs two grid-wide norms; their
 * reduction partials live in a library-owned device array of 64 KiB, one per
 * device, held until the process ends (its need does not grow with N; a
 * layout that outgrew it would return ROK_EINVAL).  The call uses the array
 * of the current device, so `stream` must belong to the current device.  It
 * allocates nothing and clears what it needs with a kernel (no memset).
 * Calls that overlap in time on one device share that array and race: order
 * them on one stream or synchronise between them.
 */
rok_status rok_jvp_noalloc(rok_ctx* ctx, const double* y, const double* fy, const double* v, void* w, int mode,
                           double eps, void* stream);

/*
 * Modified Arnoldi (Sec. 2.2.2): orthonormal basis V of K_M(J(y), fy) and
 * H = V^T J V (upper Hessenberg).
 *   y, fy:  N doubles (fy = f(y) as a double vector)
 *   M:      1..min(ROK_MAX_M, N) requested dimension
 *   mode:   ROK_JVP_FD (eps <= 0: sqrt((1 + ||y||) eps_mach), unit vectors)
 *           or ROK_JVP_TANGENT
 *   V:      N x M doubles, column c at V + c*N (columns >= M_eff untouched)
 *   H:      M x M doubles, row-major, H[i*M + j] = h_ij (zero outside the
 *           leading M_eff x M_eff Hessenberg block)
 *   M_eff:  one device int: the dimension reached (0 when fy = 0; < M on an
 *           invariant subspace, i.e. h_{j+1,j} <= 1e-13 ||(h_1j..h_{j+1,j})||)
 *   work:   rok_workspace_bytes(ctx, M, 0) bytes; its status word
 *           (rok_read_status) reports the products J v_j: ROK_FLAG_NONPHYSICAL
 *           and ROK_FLAG_NONFINITE as for rok_step
 */
rok_status rok_arnoldi(rok_ctx* ctx, const double* y, const double* fy, int M, int mode, double eps,
                       double* V, double* H, int* M_eff, void* work, size_t work_bytes, void* stream);

/*
 * One column of modified Arnoldi (Sec. 2.2.2): orthogonalise w = J v_j
 * against v_0..v_j by modified Gram-Schmidt, h_ij = <v_i, w>, w <- w - h_ij v_i
 * (i = 0..j, in order), then, when j + 1 < M, h_{j+1,j} = ||w|| and
 * v_{j+1} = w / h_{j+1,j} unless the breakdown test of rok_arnoldi holds.
 * The column is orthogonalised the way rok_arnoldi does on this context
 * (rok_arnoldi_path: pass by pass, resident, or the one-reduce form, which
 * keeps the strictly lower Gram part of V^T V in the workspace from one
 * column to the next).  Sums are taken in the library's fixed order, so a
 * sequence of calls j = 0..M-1 on one workspace reproduces rok_arnoldi's V
 * and H bit for bit.
 *   V:      N x M doubles, column c at V + c*N; columns 0..j are read
 *   M, j:   1 <= M <= min(ROK_MAX_M, N), 0 <= j < M
 *   w:      N doubles holding J v_j; its contents are undefined on return
 *   H:      (M + 1) x M doubles, row-major: writes H[i*M + j] (i <= j) and
 *           H[(j+1)*M + j] when j + 1 < M
 *   vnext:  N doubles (may be V + (j+1)*N), written when j + 1 < M and the
 *           column did not break down
 *   work:   rok_workspace_bytes(ctx, M, 0) bytes prepared by
 *           rok_workspace_init(ctx, work, bytes, M, 0, stream); a breakdown
 *           sets M_eff = j + 1 and ROK_FLAG_BREAKDOWN in its status header
 *           (rok_read_meff / rok_read_status), after which later columns
 *           are skipped until the workspace is initialised again.
 * All pointers are device memory.
 */
rok_status rok_mgs_column(rok_ctx* ctx, const double* V, int M, int j, double* w, double* H, double* vnext,
                          void* work, size_t work_bytes, void* stream);

/* Prepare a workspace of rok_workspace_bytes(ctx, M, s) bytes for the
 * column-level calls (status header cleared, M_eff = M).  The other entry
 * points prepare their workspace themselves. */
rok_status rok_workspace_init(rok_ctx* ctx, void* work, size_t work_bytes, int M, int s, void* stream);

/*
 * One ROK step (Sec. 2.2.2, eq. 9): F_i = f(y_n + sum_j alpha_ij k_j),
 * phi_i = V^T F_i, lambda_i = (I - h gamma H)^{-1} (h phi_i + h H sum_j
 * gamma_ij lambda_j), k_i = V lambda_i + h (F_i - V phi_i),
 * y_{n+1} = y_n + sum_i b_i k_i, with (V, H) from rok_arnoldi at y_n (FD
 * products use eps = sqrt((1 + ||y_n||) eps_mach)).  M = 0 gives the explicit
 * Runge-Kutta method (alpha, b).
 *   tab:    host tableau;  M: 0..ROK_MAX_M (clamped to N);  h: step size
 *   y_n, y_np1: N doubles each (may not alias)
 *   work:   rok_workspace_bytes(ctx, M, tab->s) bytes
 * Status word of `work` (rok_read_status), cleared at the start of the call:
 * ROK_FLAG_NONPHYSICAL if any stage residual or product staged a cell with
 * rho <= 0 or p <= 0 (the step is still computed, with no positivity fix),
 * ROK_FLAG_NONFINITE if a stage residual, a product, H, phi or lambda holds
 * a NaN or Inf (a NaN anywhere in y_n reaches F_1), plus the Arnoldi bits.
 * rok_residual and rok_jvp take no status word and report nothing.
 */
rok_status rok_step(rok_ctx* ctx, const rok_tableau* tab, int M, int mode, double h,
                    const double* y_n, double* y_np1, void* work, size_t work_bytes, void* stream);

/*
 * Weighted RMS norm of a local error estimate, for adaptive step-size control
 * (Sec. 4.2 compares the adaptive step sizes of explicit Runge-Kutta and ROK;
 * the estimator is not stated there, and the library's reading is step
 * doubling, see rok_integrate_adaptive):
 *   sc_i = atol + rtol * max(|y_n,i|, |y_a,i|)
 *   q_i  = (y_a,i - y_b,i) / (scale * sc_i)
 *   *err = sqrt( sum_i q_i^2 / N )
 * with the sum taken in the library's fixed order (bitwise reproducible).
 * A NaN in y_n or y_a propagates to *err.
 *   y_n, y_a, y_b: N doubles each, device memory
 *   rtol, atol:    >= 0, finite, not both zero;  scale: > 0, finite
 *   err:           one double, device memory, written on `stream`
 *   work:          rok_workspace_bytes(ctx, 0, 0) bytes (any larger workspace
 *                  works); its status header and reduction scratch are
 *                  overwritten, so a forward kept for rok_step_vjp_stored
 *                  must not be passed
 */
rok_status rok_error_norm(rok_ctx* ctx, const double* y_n, const double* y_a, const double* y_b, double rtol,
                          double atol, double scale, double* err, void* work, size_t work_bytes, void* stream);

typedef struct {
    double t;        /* time reached: T, unless max_steps attempts ran out first */
    double h_next;   /* the controller's proposal for the next macro step       */
    int accepted;    /* accepted macro steps                                    */
    int rejected;    /* rejected macro steps                                    */
    int recorded;    /* entries written to `history`                            */
} rok_adaptive_stats;

/*
 * Integrates y' = f(y) from 0 to T with rok_step under adaptive step-size
 * control by step doubling (reading of Sec. 4.2).  Each macro step of size H
 * takes one step of H (y_full) and two of H/2 (y_half) from the accepted
 * state y_n; err = rok_error_norm(y_n, y_half, y_full; rtol, atol,
 * scale = 2^order - 1).  err <= 1 accepts the step and the integration
 * continues from y_half; the next H is H * min(fmax, max(0.2, 0.9 *
 * err^(-1/(order+1)))) with fmax = 4, or 1 right after a rejection (a
 * non-finite err rejects with factor 0.2).  The last macro step is shortened
 * to end at T.  The control decisions are taken on the host: each macro step
 * synchronises `stream` once to read err.
 *   tab, M, mode: as rok_step (M = 0: the explicit Runge-Kutta method)
 *   order:   1..16, the order p of the method (sets the error scale and the
 *            controller's exponent)
 *   T >= 0, H0 > 0: end time and first attempted macro step
 *   rtol, atol: as rok_error_norm
 *   max_steps: attempts (accepted + rejected) after which the call returns
 *            with stats->t < T; it also returns early, with stats->t < T,
 *            when rejections have shrunk H until t + H == t (every attempt
 *            failed, e.g. on a non-physical state)
 *   y:       N doubles, device memory: y(0) on entry, y(stats->t) on return
 *   stats:   host memory, written on success
 *   history: host memory for history_cap entries of 4 doubles (t, H, err,
 *            accepted ? 1 : 0), one per attempted macro step in order;
 *            attempts beyond history_cap are not recorded (may be null when
 *            history_cap = 0)
 *   work:    rok_adaptive_workspace_bytes(ctx, M, tab->s) bytes, device
 *            memory (a step workspace and three state vectors)
 * Returns when the work is complete (the stream is synchronised).
 */
rok_status rok_integrate_adaptive(rok_ctx* ctx, const rok_tableau* tab, int M, int mode, int order, double T,
                                  double H0, double rtol, double atol, int max_steps, double* y,
                                  rok_adaptive_stats* stats, double* history, int history_cap, void* work,
                                  size_t work_bytes, void* stream);

/* Bytes of device workspace rok_integrate_adaptive needs (0 on invalid arguments). */
size_t rok_adaptive_workspace_bytes(const rok_ctx* ctx, int M, int s);

/*
 * Discrete adjoint of one ROK step (Sec. 2.2.2, eq. 9) taken with exact
 * (tangent) Jacobian-vector products:
 *   ybar_n = (d y_{n+1} / d y_n)^T ybar_np1
 * where y_{n+1} is the step of rok_step with mode ROK_JVP_TANGENT.  The step
 * is recomputed from y_n (checkpoint recomputation); its result is written
 * to y_np1 when that pointer is non-null.  The reverse sweep differentiates
 * every operation of the step, including the dependence of the Krylov basis
 * V and of H on y_n (modified Gram-Schmidt in reverse, the normalisation of
 * the first basis vector and the second-order residual adjoint of each
 * product J(y_n) v_j), so the result is the gradient of the computed step,
 * not of an idealised one (up to the rounding of the rebuilt MGS iterates:
 * the last iterate of column j is taken as h_{j+1,j} v_{j+1} where v_{j+1}
 * exists).  The workspace's status header reports the step (M_eff, flags)
 * and ROK_FLAG_BARRIER if an in-kernel barrier of the reverse timed out.
 *   tab, M, h:  as rok_step
 *   y_n, ybar_np1, ybar_n, y_np1: N doubles each, device memory; ybar_n and
 *               y_np1 may not alias any other argument
 *   work:       rok_step_vjp_workspace_bytes(ctx, M, tab->s) bytes
 * FP64 precision only (ROK_EUNSUPPORTED in FP32); every physics, flux and
 * grid (Cartesian, rok_set_grid, rok_set_ogrid).
 */
rok_status rok_step_vjp(rok_ctx* ctx, const rok_tableau* tab, int M, double h, const double* y_n,
                        const double* ybar_np1, double* ybar_n, double* y_np1, void* work, size_t work_bytes,
                        void* stream);

/* Bytes of device workspace rok_step_vjp needs (0 on invalid arguments). */
size_t rok_step_vjp_workspace_bytes(const rok_ctx* ctx, int M, int s);

/*
 * The reverse sweep of rok_step_vjp without recomputing the step: the same
 * adjoint (Sec. 2.2.2, eq. 9; exact products), taken from the forward
 * quantities (V, H, its LU factors, lambda_i, phi_i, F_i, k_i) that a call
 * rok_step(ctx, tab, M, ROK_JVP_TANGENT, h, y_n, ...) left in `fwd_work`.
 * It trades memory for time: a caller that keeps one forward workspace per
 * step (rok_workspace_bytes(ctx, M, tab->s) bytes, about M + 2 s state
 * vectors) reverses each step in about the time of the reverse sweep alone.
 *   tab, M, h, y_n: exactly those of that rok_step call (not checked: any
 *           other forward, an FD step included, gives a meaningless result)
 *   ybar_np1, ybar_n: N doubles each; ybar_n may not alias y_n or ybar_np1
 *   fwd_work: the forward workspace, device memory, rok_workspace_bytes(ctx,
 *           M, tab->s) bytes; the call writes only its scratch words (work
 *           vector, exchange and status words), so a forward may be reversed
 *           several times
 *   adj_work: rok_step_vjp_adjoint_bytes(ctx, M, tab->s) bytes, device memory
 * Results are bitwise those of rok_step_vjp; the same restrictions.
 */
rok_status rok_step_vjp_stored(rok_ctx* ctx, const rok_tableau* tab, int M, double h, const double* y_n,
                               const double* ybar_np1, double* ybar_n, void* fwd_work, size_t fwd_bytes,
                               void* adj_work, size_t adj_bytes, void* stream);

/* Bytes of adjoint workspace rok_step_vjp_stored needs (0 on invalid arguments). */
size_t rok_step_vjp_adjoint_bytes(const rok_ctx* ctx, int M, int s);

/*
 * Adjoint product of the residual (transposed Jacobian, Sec. 2.3 / eq. 11):
 *   ybar = J(y)^T wbar          (accumulate = 0)
 *   ybar = ybar + J(y)^T wbar   (accumulate = 1)
 * y, wbar, ybar: N doubles (ybar may not alias y or wbar).  FP64 precision
 * only (ROK_EUNSUPPORTED in FP32); every physics (Euler, Navier-Stokes with
 * constant or Sutherland viscosity), flux and grid (Cartesian, periodic
 * curvilinear, O-grid with its wall and far-field faces).
 * Deterministic: each cell gathers its own contributions.
 */
rok_status rok_residual_vjp(rok_ctx* ctx, const double* y, const double* wbar, double* ybar, int accumulate,
                            void* stream);

/*
 * First- and second-order adjoint in one pass: ybar (+)= J(y)^T wbar and
 * ybar2 (+)= d/dt [J(y + t v)^T wbar] at t = 0 (the derivative of the adjoint
 * product along v, needed to differentiate a Krylov basis built from exact
 * products).  All arrays N doubles, device memory; same restrictions as
 * rok_residual_vjp.
 */
rok_status rok_residual_vjp2(rok_ctx* ctx, const double* y, const double* v, const double* wbar, double* ybar,
                             double* ybar2, int accumulate, void* stream);

/*
 * The k eigenvalues of largest magnitude of the Jacobian J(y) of f, matrix
 * free: the stiffness diagnostic of Sec. 4 (an implicitly restarted Arnoldi
 * method on exact products J v).  An Arnoldi factorisation J V_m = V_m H_m +
 * h_{m+1,m} v_{m+1} e_m^T is built from v0 (modified Gram-Schmidt, the
 * library's kernels, applied twice per column); the Ritz values of H_m are its eigenvalues; while
 * fewer than k of the wanted ones have residual estimates
 * |h_{m+1,m}| |e_m^T x| <= tol |theta| (x the unit eigenvector of H_m), the
 * factorisation is compressed to k (k + 1 when a conjugate pair straddles
 * the cut) columns by exact shifted QR steps with the unwanted Ritz values
 * and extended back to m, at most max_restarts times.  The small dense work
 * on H (m x m) runs on the host; the call synchronises `stream`.
 *   y, v0:  N doubles, device memory (v0 != 0: the start vector)
 *   k, m:   1 <= k, k + 2 <= m <= ROK_EIGS_MAX_M, m + 1 <= N (m + 1 > ROK_MAX_M:
 *           the passes of the Gram-Schmidt columns run one launch each,
 *           whatever the context's Gram-Schmidt path; ROK_EUNSUPPORTED if the
 *           context asks for ROK_MGS_RESIDENT)
 *   tol:    > 0;  max_restarts >= 0
 *   re, im, resid: host arrays of k doubles: the wanted Ritz values by
 *           decreasing magnitude and their residual estimates (0 when the
 *           Krylov space became invariant)
 *   info:   host int[2]: restarts used, number of converged values
 *   work:   rok_eigs_workspace_bytes(ctx, k, m) bytes, device memory
 * ROK_EINVAL for a zero start vector; ROK_EHIP if the host QR iteration on
 * H does not converge.
 */
rok_status rok_eigs(rok_ctx* ctx, const double* y, const double* v0, int k, int m, int max_restarts, double tol,
                    double* re, double* im, double* resid, int* info, void* work, size_t work_bytes, void* stream);

/* Bytes of device workspace rok_eigs needs (0 on invalid arguments). */
size_t rok_eigs_workspace_bytes(const rok_ctx* ctx, int k, int m);

/* Copies the status word of `work` (ROK_FLAG_* bits of the last call that
 * used it) to *host_flags; synchronises `stream`. */
rok_status rok_read_status(rok_ctx* ctx, const void* work, int* host_flags, void* stream);

/* Reads M_eff of the last rok_step that used `work`; synchronises `stream`. */
rok_status rok_read_meff(rok_ctx* ctx, const void* work, int* host_meff, void* stream);

const char* rok_strerror(rok_status status);

#ifdef __cplusplus
}
#endif

#endif /* ROK_H */
