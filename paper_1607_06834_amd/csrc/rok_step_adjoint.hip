// Discrete adjoint of one ROK step (Sec. 2.2.2, eq. 9) computed with exact
// (tangent) Jacobian-vector products: given ybar_{n+1} = dL/dy_{n+1}, the
// reverse sweep returns ybar_n = dL/dy_n of the same arithmetic the forward
// step performs.  The forward quantities (V, H, LU, F_i, k_i, lambda_i,
// phi_i) come from a recomputation of the step; the kernels here are the
// transposes of the stage recoveries, of the reduced solve, of the
// projections, of modified Gram-Schmidt (in reverse pass order) and of the
// normalisation of the first basis vector.  Every kernel reads the step's
// M_eff from the status header, so breakdown and zero right-hand sides need
// no host synchronisation.
//
// Reverse rules (x' denotes the result of one forward operation):
//   k = V lam + h (F - V phi):  Vbar += kbar (lam - h phi)^T, lambar += V^T kbar,
//                               phibar -= h V^T kbar, Fbar += h kbar
//   A lam = h phi + h H g:      r = A^{-T} lambar, phibar += h r, Hbar += h r g^T,
//                               gbar = h H^T r, Abar -= r lam^T
//   phi = V^T F:                Vbar += F phibar^T, Fbar += V phibar
//   w' = w - h v, h = <v, w>:   hb = Hbar_h - <w'bar, v>, vbar += hb w - h w'bar,
//                               wbar = w'bar + hb v
//   v = w / rho, rho = ||w||:   wbar = vbar / rho + (Hbar_rho - <vbar, v> / rho) v
// Sums here use a fixed order (deterministic results) that is not tied to
// any other implementation's.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"

namespace rok {

namespace {

constexpr int kT = kRedThreads;  // threads per block of the reduction kernels
constexpr int kB = kRedBlocks;   // reduction grid

__device__ __forceinline__ double bsum(double acc, double* s) {
    __shared__ double s_r;
    double r = tree256(acc, s);
    if (threadIdx.x == 0) s_r = r;
    __syncthreads();
    r = s_r;
    __syncthreads();
    return r;
}

// Sum of kB partials (every thread of a kT block gets it).
__device__ __forceinline__ double finish(const double* part, double* s) {
    double a = 0.0;
    for (int b = threadIdx.x; b < kB; b += kT) a = a + part[b];
    return bsum(a, s);
}

__global__ void k_adj_init(double* Hbar, int nh, double* Abar, int na, double* lambar, double* phibar, int nsm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x, T = gridDim.x * blockDim.x;
    for (int e = t; e < nh; e += T) Hbar[e] = 0.0;
    for (int e = t; e < na; e += T) Abar[e] = 0.0;
    for (int e = t; e < nsm; e += T) {
        lambar[e] = 0.0;
        phibar[e] = 0.0;
    }
}

struct Vecs {
    double* p[kMaxStages];
    double c[kMaxStages];
    int n;
};

// ybar = ybar_out (the direct term of y_{n+1} = y_n + ...), kbar_i = b_i ybar_out.
__global__ void k_adj_seed(const double* ybar_out, double* ybar, Vecs kb, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const double yo = ybar_out[e];
        ybar[e] = yo;
        for (int i = 0; i < kb.n; ++i) kb.p[i][e] = kb.c[i] * yo;
    }
}

struct CVecs {
    const double* p[kMaxStages];
    double c[kMaxStages];
    int n;
};

// Y = y + sum_t c_t x_t (stage state, terms in stage order as in the forward).
__global__ void k_stage_state(const double* y, CVecs xs, double* Y, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double acc = y[e];
        for (int t = 0; t < xs.n; ++t) acc = acc + xs.c[t] * xs.p[t][e];
        Y[e] = acc;
    }
}

// ybar += Ybar; kbar_j += alpha_ij Ybar.
__global__ void k_scatter(const double* Ybar, double* ybar, Vecs kb, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const double yb = Ybar[e];
        ybar[e] = ybar[e] + yb;
        for (int t = 0; t < kb.n; ++t) kb.p[t][e] = kb.p[t][e] + kb.c[t] * yb;
    }
}

struct GRow {
    double g[kMaxStages];
};

// Reduced-space reverse of stage i on one block; P = V^T kbar_i from the
// projection partials (column c at part + c kB).  H, LU and the lambdas are
// staged in LDS; the triangular solves run column by column across threads,
// the rank-one updates of Abar and Hbar entry-parallel.
__global__ __launch_bounds__(kT) void k_small_rev(const double* part, int M, int i, GRow gr, double h,
                                                 const double* H, const double* LU, const int* perm,
                                                 const double* lam, double* lambar, double* phibar, double* Abar,
                                                 double* Hbar, const int* ints) {
    __shared__ double s[kT];
    __shared__ double P[kMaxM], r[kMaxM], z[kMaxM], g[kMaxM], Htr[kMaxM], li[kMaxM];
    __shared__ double sLU[kMaxM * kMaxM], sH[kMaxM * kMaxM];
    const int m = ints[0];
    const int tid = threadIdx.x;
    for (int c = 0; c < m; ++c) {
        double t = finish(part + (long)c * kB, s);
        if (tid == 0) P[c] = t;
    }
    for (int e = tid; e < m * m; e += kT) {
        const int a = e / m, b = e % m;
        sLU[a * kMaxM + b] = LU[a * M + b];
        sH[a * kMaxM + b] = H[a * M + b];
    }
    __syncthreads();
    double* lb = lambar + (long)i * M;
    if (tid < m) {
        const double v = lb[tid] + P[tid];
        lb[tid] = v;
        z[tid] = v;
        li[tid] = lam[(long)i * M + tid];
        double a = 0.0;
        for (int j = 0; j < i; ++j)
            if (gr.g[j] != 0.0) a = a + gr.g[j] * lam[j * M + tid];
        g[tid] = a;
    }
    __syncthreads();
    // A = P^T L U (row permutation perm):  A^T r = lb  <=>  U^T z = lb, L^T u = z, r[perm[q]] = u[q]
    for (int q = 0; q < m; ++q) {          // U^T (lower triangular) forward, column-oriented
        if (tid == 0) z[q] = z[q] / sLU[q * kMaxM + q];
        __syncthreads();
        if (tid > q && tid < m) z[tid] = z[tid] - sLU[q * kMaxM + tid] * z[q];
        __syncthreads();
    }
    for (int q = m - 1; q > 0; --q) {      // L^T (unit upper triangular) backward, column-oriented
        if (tid < q) z[tid] = z[tid] - sLU[q * kMaxM + tid] * z[q];
        __syncthreads();
    }
    if (tid < m) r[perm[tid]] = z[tid];
    __syncthreads();
    if (tid < m) {
        phibar[(long)i * M + tid] = -h * P[tid] + h * r[tid];
        double a = 0.0;                     // (H^T r)_c
        for (int q = 0; q < m; ++q) a = a + sH[q * kMaxM + tid] * r[q];
        Htr[tid] = a;
    }
    for (int e = tid; e < m * m; e += kT) {
        const int a = e / m, b = e % m;
        Abar[a * M + b] = Abar[a * M + b] - r[a] * li[b];
        Hbar[a * M + b] = Hbar[a * M + b] + h * r[a] * g[b];
    }
    __syncthreads();
    if (tid < m)
        for (int j = 0; j < i; ++j)
            if (gr.g[j] != 0.0) lambar[j * M + tid] = lambar[j * M + tid] + gr.g[j] * h * Htr[tid];
}

// Vbar[:, c] += (lam_c - h phi_c) kbar + phibar_c F;  Fbar = h kbar + V phibar.
// first: the last stage, which is reversed first and initialises Vbar.
__global__ void k_vbar_stage(double* Vbar, double* Fbar, const double* V, const double* kbar, const double* F,
                             const double* lam, const double* phi, const double* phibar, double h, long n,
                             const int* ints, int first) {
    const int m = ints[0];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const double kb = kbar[e], fe = F[e];
        double acc = h * kb;
        for (int c = 0; c < m; ++c) {
            const long o = (long)c * n + e;
            const double t = (lam[c] - h * phi[c]) * kb + phibar[c] * fe;
            Vbar[o] = first ? t : Vbar[o] + t;
            acc = acc + phibar[c] * V[o];
        }
        Fbar[e] = acc;
    }
}

// Hbar -= hg Abar  (A = I - hg H).
__global__ void k_abar_to_hbar(const double* Abar, double* Hbar, int M, double hg, const int* ints) {
    const int m = ints[0];
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int a = e / m, b = e % m;
        Hbar[a * M + b] = Hbar[a * M + b] - hg * Abar[a * M + b];
    }
}

// Partials of <a, b>; nothing when col >= M_eff.
__global__ __launch_bounds__(kT) void k_dot(const double* a, const double* b, long n, double* part, const int* ints,
                                           int col) {
    __shared__ double s[kT];
    if (col >= ints[0]) return;
    double acc = 0.0;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < n; e += (long)kB * kT) acc = acc + a[e] * b[e];
    const double t = bsum(acc, s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Start of the reverse of Arnoldi column j (j < M_eff):
//   w    = the forward's last MGS iterate: h_{j+1,j} v_{j+1} when j + 1 < M_eff (equal to it up to the
//          rounding of v_{j+1} = w / h_{j+1,j}), else J v_j - sum_{i<=j} h_ij v_i (w holds J v_j on entry)
//   wbar = adjoint of that iterate: from v_{j+1} = w / h_{j+1,j} when j + 1 < M_eff, else 0
//   part = partials of <wbar, v_j>
__global__ __launch_bounds__(kT) void k_col_start(double* w, const double* V, const double* H, int M, int j,
                                                 const double* Vbar, const double* Hbar, const double* partA,
                                                 double* wbar, double* part, long n, const int* ints) {
    __shared__ double s[kT];
    __shared__ double hc[kMaxM];
    const int m = ints[0];
    if (j >= m) return;
    const bool nrm = j + 1 < m;
    double rho = 1.0, coef = 0.0;
    if (nrm) {
        rho = H[(j + 1) * M + j];
        coef = Hbar[(j + 1) * M + j] - finish(partA, s) / rho;
    }
    for (int i = threadIdx.x; i <= j; i += kT) hc[i] = H[i * M + j];
    __syncthreads();
    const double* vj = V + (long)j * n;
    const double* vn = V + (long)(j + 1) * n;
    const double* vbn = Vbar + (long)(j + 1) * n;
    double acc = 0.0;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < n; e += (long)kB * kT) {
        double wv;
        if (nrm) {
            wv = rho * vn[e];
        } else {
            wv = w[e];
            for (int i = 0; i <= j; ++i) wv = wv - hc[i] * V[(long)i * n + e];
        }
        w[e] = wv;
        const double wb = nrm ? vbn[e] / rho + coef * vn[e] : 0.0;
        wbar[e] = wb;
        acc = acc + wb * vj[e];
    }
    const double t = bsum(acc, s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Reverse of MGS pass i of column j, w' = w - h_ij v_i; on entry w = w',
// wbar = w'bar and pin holds the partials of <w'bar, v_i>.  Restores w,
// updates vbar_i and wbar, and leaves the partials of <wbar, v_{i-1}> in pout.
__global__ __launch_bounds__(kT) void k_mgs_rev(double* w, double* wbar, const double* V, double* Vbar, const double* H,
                                               const double* Hbar, int M, int i, int j, const double* pin,
                                               double* pout, long n, const int* ints) {
    __shared__ double s[kT];
    if (j >= ints[0]) return;
    const double h = H[i * M + j];
    const double hb = Hbar[i * M + j] - finish(pin, s);
    const double* vi = V + (long)i * n;
    const double* vp = V + (long)(i > 0 ? i - 1 : 0) * n;
    double* vbi = Vbar + (long)i * n;
    double acc = 0.0;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < n; e += (long)kB * kT) {
        const double v = vi[e];
        const double wo = w[e] + h * v;
        w[e] = wo;
        const double wb = wbar[e];
        vbi[e] = vbi[e] + hb * wo - h * wb;
        const double wn = wb + hb * v;
        wbar[e] = wn;
        if (i > 0) acc = acc + wn * vp[e];
    }
    if (i > 0) {
        const double t = bsum(acc, s);
        if (threadIdx.x == 0) pout[blockIdx.x] = t;
    }
}

// v_0 = F_0 / beta:  Fbar_0 += vbar_0 / beta - (<vbar_0, v_0> / beta) v_0  (M_eff > 0).
__global__ __launch_bounds__(kT) void k_beta_rev(double* Fbar0, const double* vbar0, const double* v0,
                                                const double* part, const double* scal, long n, const int* ints) {
    __shared__ double s[kT];
    if (ints[0] < 1) return;
    const double beta = scal[2];
    const double coef = finish(part, s) / beta;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        Fbar0[e] = Fbar0[e] + vbar0[e] / beta - coef * v0[e];
}

unsigned grid(long n) {
    long g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

size_t adj_bytes(long N, int M, int s) {
    const int Mm = M > 0 ? M : 1;
    const size_t vec = al(sizeof(double) * (size_t)N);
    size_t b = 0;
    b += al(sizeof(double) * (Mm + 1) * Mm);        // Hbar
    b += al(sizeof(double) * Mm * Mm);              // Abar
    b += 2 * al(sizeof(double) * s * Mm);           // lambar, phibar
    b += al(sizeof(double) * (size_t)(Mm + 3) * kB);  // partials
    b += vec * ((size_t)M + s + 5);                 // Vbar, kbar, Fbar0, FB, Yt, Ybar, wbar
    return b;
}

AdjWork adj_carve(void* base, long N, int M, int s) {
    const int Mm = M > 0 ? M : 1;
    const size_t vec = al(sizeof(double) * (size_t)N);
    char* p = (char*)base;
    AdjWork A{};
    A.Hbar = (double*)p;   p += al(sizeof(double) * (Mm + 1) * Mm);
    A.Abar = (double*)p;   p += al(sizeof(double) * Mm * Mm);
    A.lambar = (double*)p; p += al(sizeof(double) * s * Mm);
    A.phibar = (double*)p; p += al(sizeof(double) * s * Mm);
    A.part = (double*)p;   p += al(sizeof(double) * (size_t)(Mm + 3) * kB);
    A.Vbar = (double*)p;   p += vec * (size_t)M;
    A.kbar = (double*)p;   p += vec * (size_t)s;
    A.Fbar0 = (double*)p;  p += vec;
    A.FB = (double*)p;     p += vec;
    A.Yt = (double*)p;     p += vec;
    A.Ybar = (double*)p;   p += vec;
    A.wbar = (double*)p;   p += vec;
    A.M = Mm;
    return A;
}

hipError_t launch_adj_init(const AdjWork& A, int M, int s, hipStream_t st) {
    const int Mm = M > 0 ? M : 1;
    hipLaunchKernelGGL(k_adj_init, dim3(16), dim3(256), 0, st, A.Hbar, (Mm + 1) * Mm, A.Abar, Mm * Mm, A.lambar,
                       A.phibar, s * Mm);
    return hipGetLastError();
}

hipError_t launch_adj_seed(const AdjWork& A, const double* ybar_out, double* ybar, long n, int s, const double* b,
                           hipStream_t st) {
    Vecs kb{};
    kb.n = s;
    for (int i = 0; i < s; ++i) {
        kb.p[i] = A.kbar + (long)i * n;
        kb.c[i] = b[i];
    }
    hipLaunchKernelGGL(k_adj_seed, dim3(grid(n)), dim3(256), 0, st, ybar_out, ybar, kb, n);
    return hipGetLastError();
}

hipError_t launch_stage_state(const double* y, const double* K, const double* alpha_row, int i, double* Y, long n,
                              hipStream_t st) {
    CVecs xs{};
    int t = 0;
    for (int j = 0; j < i; ++j)
        if (alpha_row[j] != 0.0) {
            xs.p[t] = K + (long)j * n;
            xs.c[t] = alpha_row[j];
            ++t;
        }
    xs.n = t;
    hipLaunchKernelGGL(k_stage_state, dim3(grid(n)), dim3(256), 0, st, y, xs, Y, n);
    return hipGetLastError();
}

hipError_t launch_scatter(const AdjWork& A, const double* Ybar, double* ybar, const double* alpha_row, int i, long n,
                          hipStream_t st) {
    Vecs kb{};
    int t = 0;
    for (int j = 0; j < i; ++j)
        if (alpha_row[j] != 0.0) {
            kb.p[t] = A.kbar + (long)j * n;
            kb.c[t] = alpha_row[j];
            ++t;
        }
    kb.n = t;
    hipLaunchKernelGGL(k_scatter, dim3(grid(n)), dim3(256), 0, st, Ybar, ybar, kb, n);
    return hipGetLastError();
}

hipError_t launch_small_rev(const Work& W, const AdjWork& A, int M, int i, const double* gam_row, double h,
                            hipStream_t st) {
    GRow gr{};
    for (int j = 0; j < kMaxStages; ++j) gr.g[j] = (j < i) ? gam_row[j] : 0.0;
    hipLaunchKernelGGL(k_small_rev, dim3(1), dim3(kT), 0, st, A.part, M, i, gr, h, W.H, W.LU, W.perm, W.lam,
                       A.lambar, A.phibar, A.Abar, A.Hbar, W.ints);
    return hipGetLastError();
}

hipError_t launch_vbar_stage(const Work& W, const AdjWork& A, int M, int i, double h, double* Fbar, long n,
                             bool first, hipStream_t st) {
    hipLaunchKernelGGL(k_vbar_stage, dim3(grid(n)), dim3(256), 0, st, A.Vbar, Fbar, W.V, A.kbar + (long)i * n,
                       W.F + (long)i * n, W.lam + (long)i * M, W.phi + (long)i * M, A.phibar + (long)i * M, h, n,
                       W.ints, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_abar_to_hbar(const Work& W, const AdjWork& A, int M, double hg, hipStream_t st) {
    hipLaunchKernelGGL(k_abar_to_hbar, dim3(1), dim3(256), 0, st, A.Abar, A.Hbar, M, hg, W.ints);
    return hipGetLastError();
}

// Partial buffers: projection columns [0, M), then three for the MGS reverse.
static double* ap(const AdjWork& A, int k) { return A.part + (size_t)(A.M + k) * kB; }

hipError_t launch_arnoldi_rev_col(const Work& W, const AdjWork& A, int M, int j, long n, bool resident,
                                  hipStream_t st) {
    // W.w holds J v_j on entry (where the column needs it).
    if (resident) return launch_mgs_rev_resident(W, A, M, j, n, st);
    if (j + 1 < M)
        hipLaunchKernelGGL(k_dot, dim3(kB), dim3(kT), 0, st, A.Vbar + (long)(j + 1) * n, W.V + (long)(j + 1) * n, n,
                           ap(A, 0), W.ints, j + 1);
    hipLaunchKernelGGL(k_col_start, dim3(kB), dim3(kT), 0, st, W.w, W.V, W.H, M, j, A.Vbar, A.Hbar, ap(A, 0), A.wbar,
                       ap(A, 1), n, W.ints);
    for (int i = j; i >= 0; --i)
        hipLaunchKernelGGL(k_mgs_rev, dim3(kB), dim3(kT), 0, st, W.w, A.wbar, W.V, A.Vbar, W.H, A.Hbar, M, i, j,
                           ap(A, 1 + ((j - i) & 1)), ap(A, 1 + ((j - i + 1) & 1)), n, W.ints);
    return hipGetLastError();
}

hipError_t launch_beta_rev(const Work& W, const AdjWork& A, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_dot, dim3(kB), dim3(kT), 0, st, A.Vbar, W.V, n, ap(A, 0), W.ints, 0);
    hipLaunchKernelGGL(k_beta_rev, dim3(grid(n)), dim3(256), 0, st, A.Fbar0, A.Vbar, W.V, ap(A, 0), W.scal, n,
                       W.ints);
    return hipGetLastError();
}

}  // namespace rok
