// Host-side launch interface of the librok kernels (internal).
#pragma once

#include "rok_device.hpp"

namespace rok {

// Residual family (rok_residual.hip).  kind: 0 = F = f(Y), 1 = FD product,
// 2 = tangent product.  fp32: compute in float.  out_double: write doubles
// even when computing in float (internal FP64 consumers).
hipError_t launch_residual(const Geom& G, int recon, bool ns, bool fp32, int kind, bool out_double,
                           const ResArgs& A, hipStream_t st);

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
    double* partials; // npart x kRedBlocks reduction partials
    int npart;
    // full-length vectors (double, N each)
    double* w;        // Arnoldi work vector
    double* V;        // M columns (rok_step only; rok_arnoldi uses the caller's V)
    double* F;        // s stage residuals
    double* K;        // s stage vectors
};

constexpr int kRedBlocks = 1024;   // reduction grid (fixed: it fixes the summation order)
constexpr int kRedThreads = 256;

size_t work_small_bytes(int M, int s);
size_t work_bytes(long N, int M, int s, bool step);
Work carve(void* base, long N, int M, int s, bool step);

// Krylov / step kernels (rok_krylov.hip)
hipError_t launch_init(const Work& W, int M, int s, hipStream_t st);
// scal[0] = ||y||, scal[1] = sqrt(u) (1 + ||y||) / (v ? ||v|| : 1)  (scal[3] = ||v||)
hipError_t launch_norm_eps(const Work& W, const double* y, const double* v, long n, hipStream_t st);
hipError_t launch_start_basis(const Work& W, const double* f, long n, double* v0, hipStream_t st);
hipError_t launch_mgs_column(const Work& W, double* w, const double* V, long n, int M, int j, double* vnext,
                             hipStream_t st);
hipError_t launch_copy_h(const Work& W, int M, double* Hout, int* meff_out, hipStream_t st);
hipError_t launch_lu(const Work& W, int M, double hg, hipStream_t st);
hipError_t launch_project(const Work& W, const double* V, const double* F, long n, int M, hipStream_t st);
hipError_t launch_lambda(const Work& W, int M, int i, const double* gam_row, double h, hipStream_t st);
hipError_t launch_recover(const Work& W, const double* V, const double* F, long n, int M, int i, double h, double* k,
                          hipStream_t st);
hipError_t launch_update(const double* y, int s, const double* K, const double* b, long n, double* y1,
                         hipStream_t st);

}  // namespace rok
