// Host-side launch interface of the librok kernels (internal).
#pragma once

#include "rok_device.hpp"

namespace rok {

// Residual family (rok_residual.hip).  kind: 0 = F = f(Y), 1 = FD product,
// 2 = tangent product.  fp32: compute in float.  out_double: write doubles
// even when computing in float (internal FP64 consumers).
// Face vectors and inverse areas of a 2-D curvilinear periodic grid (5 x nx*ny doubles).
hipError_t launch_metrics(const double* xn, const double* yn, int nx, int ny, double Lx, double Ly, double* out,
                          hipStream_t st);
// O-grid metrics (5 x nx*ny doubles, then 2 x nx wall face vectors).
hipError_t launch_metrics_ogrid(const double* xn, const double* yn, int nx, int ny, double* out, hipStream_t st);
// Fills `bytes` bytes (a multiple of 4) at p with zeros (a kernel, not a memset).
hipError_t launch_zero(void* p, long bytes, hipStream_t st);
hipError_t launch_residual(const Geom& G, int recon, bool ns, bool fp32, int kind, bool out_double,
                           const ResArgs& A, hipStream_t st);

// Adjoint products (rok_adjoint.hip): ybar (+)= J^T wbar; with v: ybar2 (+)= d/dt J(y+tv)^T wbar.
// With gate: does nothing when col >= gate[0] (gate = the step's M_eff word).
hipError_t launch_vjp(const Geom& G, int recon, const double* y, const double* v, const double* wbar, double* ybar,
                      double* ybar2, int accumulate, hipStream_t st, const int* gate = nullptr, int col = 0);

// Device scratch layout of the Krylov / step kernels (carved from the
// caller's workspace; 256-byte aligned regions).
struct Work {
    int* ints;        // [0] M_eff, [1] stop, [2] status flags (offset 0 of the workspace)
    double* scal;     // [0] ||y||, [1] eps, [2] beta, [3] ||v||
    double* H;        // (M+1) x M, row-major with leading dimension M
    double* LU;       // M x M
    double* phi;      // s x M
    double* lam;      // s x M
    int* perm;        // M
    double* L;        // M x M: strictly lower Gram part of the one-reduce Gram-Schmidt (leading dimension M)
    double* sig;      // M + 1 basis scales: column c of V holds v_c / sig[c] (1 unless normalisation is deferred)
    double* partials; // npart x kRedBlocks reduction partials
    int npart;
    double* gpart;    // 2 x kRedBlocks partials exchanged inside the resident MGS kernel
    unsigned* bar;    // grid barrier counters (kBarWords unsigned, zeroed by launch_init)
    // full-length vectors (double, N each)
    double* w;        // Arnoldi work vector
    double* V;        // M columns (rok_step only; rok_arnoldi uses the caller's V)
    double* F;        // s stage residuals
    double* K;        // s stage vectors
};

constexpr int kRedBlocks = 1024;   // reduction grid (fixed: it fixes the summation order)
constexpr int kRedThreads = 256;
constexpr int kBarWords = 1024;   // grid-barrier state (4 KiB)

size_t work_small_bytes(int M, int s);
size_t work_bytes(long N, int M, int s, bool step);
Work carve(void* base, long N, int M, int s, bool step);

// Krylov / step kernels (rok_krylov.hip)
hipError_t launch_init(const Work& W, int M, int s, hipStream_t st);
// scal[0] = ||y||, scal[1] = sqrt((1 + ||y||) u) / (v ? ||v|| : 1)  (scal[3] = ||v||)
hipError_t launch_norm_eps(const Work& W, const double* y, const double* v, long n, hipStream_t st);
// *out = sqrt(sum_i q_i^2 / n), q_i = (a_i - b_i) / (c (atol + rtol max(|y_i|, |a_i|)))
hipError_t launch_error_norm(const Work& W, const double* y, const double* a, const double* b, long n, double rtol,
                             double atol, double c, double* out, hipStream_t st);
hipError_t launch_start_basis(const Work& W, const double* f, long n, double* v0, hipStream_t st);
hipError_t launch_mgs_column(const Work& W, double* w, const double* V, long n, int M, int j, double* vnext,
                             hipStream_t st);
// v = w / ||w|| with ||w||^2 finished from `partials`, after the breakdown test of column j (H[j+1][j] = ||w||)
hipError_t launch_normalize(const Work& W, const double* w, const double* partials, int M, int j, double* v, long n,
                            hipStream_t st);
// One-reduce Gram-Schmidt for one Arnoldi column (rok_lowsync.hip); M <= 24.
// deferred: the next column is stored as the orthogonalised w, unnormalised,
// with its scale 1 / ||w|| in W.sig[j + 1]; the columns' scales apply
// throughout (W.sig; products take it as ResArgs.vscale).
bool lowsync_supported(int M);
hipError_t launch_ls_column(const Work& W, const double* w, const double* V, long n, int M, int j, double* vnext,
                            hipStream_t st, bool deferred = false);
// H[j+1][j] = ||w||, finished from `partials`, the breakdown test of column j and sig[j+1] = 1 / ||w|| (one block)
hipError_t launch_norm_scale(const Work& W, const double* partials, int M, int j, hipStream_t st);
// Resident-w MGS for one column (rok_mgs.hip).
int mgs_resident_per(long n);
bool mgs_resident_available();
hipError_t launch_mgs_resident(const Work& W, const double* w, const double* V, long n, int M, int j, double* vnext,
                               hipStream_t st);
// Eigenvalue estimate pieces (rok_eigs.hip)
hipError_t launch_combine(const double* V, long n, int m1, const double* C, int nc, double* Vout, hipStream_t st);
namespace dense {
bool hessenberg_eigenvalues(int n, const double* H, int ldh, double* wr, double* wi);
void shift_step(int m, double* H, int ldh, double* Qacc, double mre, double mim, bool pair);
double ritz_residual(int m, const double* H, int ldh, double hlast, double tre, double tim);
}  // namespace dense
hipError_t launch_copy_h(const Work& W, int M, double* Hout, int* meff_out, hipStream_t st);
hipError_t launch_lu(const Work& W, int M, double hg, hipStream_t st);
hipError_t launch_project(const Work& W, const double* V, const double* F, long n, int M, hipStream_t st);
// phi_1 = beta e_1 (F_1 = f(y_n) = beta v_0) as projection partials, without reading V
hipError_t launch_project_first(const Work& W, int M, hipStream_t st);
// sig: the basis scales (W.sig) when V holds unnormalised columns, else null
hipError_t launch_lambda(const Work& W, int M, int i, const double* gam_row, double h, hipStream_t st,
                         const double* sig = nullptr);
// k_i = V lambda_i + h (F_i - V phi_i) into k; if y is non-null (last stage)
// writes y_{n+1} = y + sum_{q<s} b_q k_q into k instead, K holding k_0..k_{s-2}.
// With ynext (stages i < s - 1; y and K given): also Y_{i+1} = y + sum_{q<=i} arow[q] k_q into ynext.
hipError_t launch_recover(const Work& W, const double* V, const double* F, long n, int M, int i, double h, double* k,
                          const double* y, const double* K, int s, const double* b, hipStream_t st,
                          const double* sig = nullptr, double* ynext = nullptr, const double* arow = nullptr);

// Discrete adjoint of the ROK step (rok_step_adjoint.hip).  Carved after the
// forward step's workspace; lambar, phibar are s x M, Hbar (M+1) x M, Abar
// M x M (leading dimension M, as H and LU).
struct AdjWork {
    double* Hbar;
    double* Abar;
    double* lambar;
    double* phibar;
    double* part;    // (M + 3) x kRedBlocks: projection columns, then three MGS-reverse buffers
    double* Vbar;    // M vectors
    double* kbar;    // s vectors
    double* Fbar0;   // adjoint of F_1 = f(y_n) (stage 0 and the first basis vector)
    double* FB;      // adjoint of the current stage residual
    double* Yt;      // current stage state
    double* Ybar;    // J(Y_i)^T FB
    double* wbar;    // adjoint of the MGS work vector
    int M;
};
size_t adj_bytes(long N, int M, int s);
AdjWork adj_carve(void* base, long N, int M, int s);
hipError_t launch_adj_init(const AdjWork& A, int M, int s, hipStream_t st);
hipError_t launch_adj_seed(const AdjWork& A, const double* ybar_out, double* ybar, long n, int s, const double* b,
                           hipStream_t st);
hipError_t launch_stage_state(const double* y, const double* K, const double* alpha_row, int i, double* Y, long n,
                              hipStream_t st);
hipError_t launch_scatter(const AdjWork& A, const double* Ybar, double* ybar, const double* alpha_row, int i, long n,
                          hipStream_t st);
hipError_t launch_small_rev(const Work& W, const AdjWork& A, int M, int i, const double* gam_row, double h,
                            hipStream_t st);
// first: initialise Vbar (the first stage reversed) instead of accumulating.
hipError_t launch_vbar_stage(const Work& W, const AdjWork& A, int M, int i, double h, double* Fbar, long n,
                             bool first, hipStream_t st);
hipError_t launch_abar_to_hbar(const Work& W, const AdjWork& A, int M, double hg, hipStream_t st);
// resident: one cooperative kernel for the column (mgs_rev_resident_available(n)), else per-pass kernels
hipError_t launch_arnoldi_rev_col(const Work& W, const AdjWork& A, int M, int j, long n, bool resident,
                                  hipStream_t st);
bool mgs_rev_resident_available(long n);
hipError_t launch_mgs_rev_resident(const Work& W, const AdjWork& A, int M, int j, long n, hipStream_t st);
hipError_t launch_beta_rev(const Work& W, const AdjWork& A, long n, hipStream_t st);

}  // namespace rok
