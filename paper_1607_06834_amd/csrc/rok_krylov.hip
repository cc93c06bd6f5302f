// Krylov and stage kernels of the ROK step (Sec. 2.2.2, eq. 9): canonical
// reductions, modified Gram-Schmidt Arnoldi passes, the reduced (M x M) LU
// solve, projections V^T F, recoveries k = V lambda + h (F - V phi) and the
// state update.
//
// Reductions follow one canonical order (the same order the CPU oracle
// writes out): a fixed grid of kRedBlocks x kRedThreads lanes, lane t adds
// the elements t, t + T, t + 2T, ... (T = kRedBlocks * kRedThreads) in index
// order, each block combines its lanes by a pairwise halving tree into one
// partial, and the consumer finishes the sum (lane t adds partials t, t+256,
// t+512, t+768, then the tree).  There is no inter-block communication
// inside a kernel: the kernel boundary publishes the partials, so no memory
// fence or atomic is needed, and every block that finishes a sum obtains the
// same bits.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"

namespace rok {

constexpr double kBreakdownTol = 1e-13;
constexpr double kSqrtEps = 1.4901161193847656e-08;  // sqrt(2^-52) = 2^-26

__device__ __forceinline__ double block_sum(double acc, double* s) {
    const int tid = threadIdx.x;
    s[tid] = acc;
    __syncthreads();
#pragma unroll
    for (int st = kRedThreads / 2; st > 0; st >>= 1) {
        if (tid < st) s[tid] = s[tid] + s[tid + st];
        __syncthreads();
    }
    double r = s[0];
    __syncthreads();
    return r;
}

// Final stage of the canonical sum (every thread of a kRedThreads block calls it).
__device__ __forceinline__ double final_sum(const double* partials, double* s) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += kRedThreads) acc = acc + partials[b];
    return block_sum(acc, s);
}

__device__ __forceinline__ bool nonfinite(double x) { return !(x == x) || fabs(x) == __builtin_inf(); }

// Per-lane sums in index order, block tree, one partial per block.
//   UPD:  first w <- w - h vprev, h = finished sum of hpart (block 0 stores
//         it to *hstore); w is written back
//   SELF: sum of w.w, else of vcur.w
template <bool UPD, bool SELF>
__global__ __launch_bounds__(kRedThreads) void k_red(double* w, const double* vprev, const double* hpart,
                                                    double* hstore, const double* vcur, long n,
                                                    const int* ints, double* partials) {
    __shared__ double s[kRedThreads];
    if (ints && ints[1]) return;
    double h = 0.0;
    if constexpr (UPD) {
        h = final_sum(hpart, s);
        if (blockIdx.x == 0 && threadIdx.x == 0) *hstore = h;
    }
    double acc = 0.0;
    const long stride = (long)kRedBlocks * kRedThreads;
    long e = (long)blockIdx.x * kRedThreads + threadIdx.x;
    for (; e + stride < n; e += 2 * stride) {
        double w0 = w[e], w1 = w[e + stride];
        if constexpr (UPD) {
            double a0 = vprev[e], a1 = vprev[e + stride];
            w0 = w0 - h * a0;
            w1 = w1 - h * a1;
            w[e] = w0;
            w[e + stride] = w1;
        }
        double b0, b1;
        if constexpr (SELF) {
            b0 = w0;
            b1 = w1;
        } else {
            b0 = vcur[e];
            b1 = vcur[e + stride];
        }
        acc = acc + b0 * w0;
        acc = acc + b1 * w1;
    }
    if (e < n) {
        double we = w[e];
        if constexpr (UPD) {
            we = we - h * vprev[e];
            w[e] = we;
        }
        if constexpr (SELF) acc = acc + we * we;
        else acc = acc + vcur[e] * we;
    }
    double bs = block_sum(acc, s);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

enum { FIN_SQRT_TO = 0, FIN_STORE = 1, FIN_BETA = 2, FIN_EPS = 3 };

// One block: finishes a sum and applies the bookkeeping of `op`.
__global__ __launch_bounds__(kRedThreads) void k_finish(const double* partials, int op, double* out, double* scal,
                                                       int* ints, int has_v) {
    __shared__ double s[kRedThreads];
    if ((op == FIN_STORE || op == FIN_BETA) && ints[1]) return;
    double tot = final_sum(partials, s);
    if (threadIdx.x != 0) return;
    if (op == FIN_SQRT_TO) {
        *out = sqrt(tot);
    } else if (op == FIN_STORE) {
        *out = tot;
        if (nonfinite(tot)) ints[2] |= ROK_FLAG_NONFINITE;
    } else if (op == FIN_BETA) {
        double beta = sqrt(tot);
        scal[2] = beta;
        if (beta == 0.0) {
            ints[0] = 0;
            ints[1] = 1;
            ints[2] |= ROK_FLAG_ZERO_RHS;
        }
        if (nonfinite(beta)) ints[2] |= ROK_FLAG_NONFINITE;
    } else {  // FIN_EPS: eps = sqrt(u) (1 + ||y||) [/ ||v||]
        double ny = sqrt(tot);
        scal[0] = ny;
        double e = kSqrtEps * (1.0 + ny);
        if (has_v) e = e / scal[3];
        scal[1] = e;
    }
}

// v_{j+1} = w / h_{j+1,j}, h_{j+1,j} = sqrt(w.w) finished from `partials`,
// after the breakdown test h_{j+1,j} <= tol ||(h_1j, ..., h_{j+1,j})||;
// for j < 0: v_0 = w / beta (scal[2]).
__global__ __launch_bounds__(kRedThreads) void k_normalize(const double* w, const double* partials, double* H, int M,
                                                          int j, double* v, long n, int* ints, const double* scal) {
    __shared__ double s[kRedThreads];
    if (ints[1]) return;
    double hn;
    if (j < 0) {
        hn = scal[2];
    } else {
        hn = sqrt(final_sum(partials, s));
        double c = 0.0;
        for (int i = 0; i <= j; ++i) c = c + H[i * M + j] * H[i * M + j];
        c = c + hn * hn;
        bool brk = hn <= kBreakdownTol * sqrt(c);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            H[(j + 1) * M + j] = hn;
            if (brk) {
                ints[0] = j + 1;
                ints[1] = 1;
                ints[2] |= ROK_FLAG_BREAKDOWN;
            }
            if (nonfinite(hn)) ints[2] |= ROK_FLAG_NONFINITE;
        }
        if (brk) return;
    }
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) v[e] = w[e] / hn;
}

__global__ void k_init(double* H, int nh, double* phi, double* lam, int nsm, double* scal, int* ints, int meff0) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int e = t; e < nh; e += gridDim.x * blockDim.x) H[e] = 0.0;
    for (int e = t; e < nsm; e += gridDim.x * blockDim.x) {
        phi[e] = 0.0;
        lam[e] = 0.0;
    }
    if (t < 16) scal[t] = 0.0;
    if (t == 0) {
        ints[0] = meff0;
        ints[1] = 0;
        ints[2] = 0;
    }
}

__global__ void k_copy_h(const double* H, int M, double* Hout, const int* ints, int* meff_out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int m = ints[0];
    for (int e = t; e < M * M; e += gridDim.x * blockDim.x) {
        int i = e / M, j = e % M;
        Hout[e] = (i < m && j < m) ? H[i * M + j] : 0.0;
    }
    if (t == 0 && meff_out) *meff_out = m;
}

// LU with partial pivoting of A = I - hg H (M_eff x M_eff), one thread.
__global__ void k_lu(const double* H, int M, double hg, double* LU, int* perm, const int* ints) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int m = ints[0];
    for (int i = 0; i < m; ++i) {
        perm[i] = i;
        for (int j = 0; j < m; ++j) LU[i * M + j] = (i == j ? 1.0 : 0.0) - hg * H[i * M + j];
    }
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int r = k + 1; r < m; ++r)
            if (fabs(LU[r * M + k]) > fabs(LU[piv * M + k])) piv = r;
        if (piv != k) {
            for (int c = 0; c < m; ++c) {
                double t = LU[k * M + c];
                LU[k * M + c] = LU[piv * M + c];
                LU[piv * M + c] = t;
            }
            int t = perm[k];
            perm[k] = perm[piv];
            perm[piv] = t;
        }
        for (int r = k + 1; r < m; ++r) {
            LU[r * M + k] = LU[r * M + k] / LU[k * M + k];
            for (int c = k + 1; c < m; ++c) LU[r * M + c] = LU[r * M + c] - LU[r * M + k] * LU[k * M + c];
        }
    }
}

struct GamRow {
    double g[kMaxStages];
};

// phi_i = V^T F_i finished from the projection partials, then
// lambda_i = LU^{-1} (h phi_i + h H sum_{j<i} gamma_ij lambda_j) on one thread.
__global__ __launch_bounds__(kRedThreads) void k_lambda(const double* H, const double* LU, const int* perm, int M,
                                                       int i, GamRow gr, double h, const double* partials,
                                                       double* phi, double* lam, int* ints) {
    __shared__ double s[kRedThreads];
    const int m = ints[0];
    for (int c = 0; c < m; ++c) {
        double t = final_sum(partials + (long)c * kRedBlocks, s);
        if (threadIdx.x == 0) phi[i * M + c] = t;
    }
    if (threadIdx.x != 0) return;
    double g[kMaxM], x[kMaxM], rhs[kMaxM];
    for (int c = 0; c < m; ++c) g[c] = 0.0;
    for (int j = 0; j < i; ++j) {
        if (gr.g[j] != 0.0)
            for (int c = 0; c < m; ++c) g[c] = g[c] + gr.g[j] * lam[j * M + c];
    }
    for (int r = 0; r < m; ++r) {
        double hg = 0.0;
        for (int c = 0; c < m; ++c) hg = hg + H[r * M + c] * g[c];
        rhs[r] = h * phi[i * M + r] + h * hg;
    }
    for (int r = 0; r < m; ++r) x[r] = rhs[perm[r]];
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < r; ++c) x[r] = x[r] - LU[r * M + c] * x[c];
    for (int r = m - 1; r >= 0; --r) {
        for (int c = r + 1; c < m; ++c) x[r] = x[r] - LU[r * M + c] * x[c];
        x[r] = x[r] / LU[r * M + r];
    }
    bool bad = false;
    for (int r = 0; r < m; ++r) {
        lam[i * M + r] = x[r];
        bad = bad || nonfinite(x[r]);
    }
    if (bad) ints[2] |= ROK_FLAG_NONFINITE;
}

// Projection partials: for c < M_eff, canonical per-block partial sums of
// V[:, c] . F (finished by k_lambda).  MB >= M.
template <int MB>
__global__ __launch_bounds__(kRedThreads) void k_project(const double* V, const double* F, long n, const int* ints,
                                                        double* partials) {
    __shared__ double s[kRedThreads];
    const int m = ints[0];
    double acc[MB];
#pragma unroll
    for (int c = 0; c < MB; ++c) acc[c] = 0.0;
    const long stride = (long)kRedBlocks * kRedThreads;
    for (long e = (long)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += stride) {
        double fe = F[e];
#pragma unroll
        for (int c = 0; c < MB; ++c)
            if (c < m) acc[c] = acc[c] + V[(long)c * n + e] * fe;
    }
#pragma unroll
    for (int c = 0; c < MB; ++c) {
        if (c < m) {
            double bs = block_sum(acc[c], s);
            if (threadIdx.x == 0) partials[(long)c * kRedBlocks + blockIdx.x] = bs;
        }
    }
}

// k = V lambda + h (F - V phi), column sums in order from zero.
__global__ void k_recover(const double* V, const double* F, long n, const int* ints, const double* lam,
                          const double* phi, double h, double* k) {
    const int m = ints[0];
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double a = 0.0, b = 0.0;
        for (int c = 0; c < m; ++c) {
            double vc = V[(long)c * n + e];
            a = a + vc * lam[c];
            b = b + vc * phi[c];
        }
        k[e] = a + h * (F[e] - b);
    }
}

struct BRow {
    double b[kMaxStages];
};

__global__ void k_update(const double* y, int s, const double* K, BRow br, long n, double* y1) {
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double acc = y[e];
        for (int i = 0; i < s; ++i)
            if (br.b[i] != 0.0) acc = acc + br.b[i] * K[(long)i * n + e];
        y1[e] = acc;
    }
}

// ---------------------------------------------------------------------------
// Workspace: a 256-byte header (status ints, scalars) at offset 0 for every M
// and s, then the small matrices, the reduction partials and the vectors.
// ---------------------------------------------------------------------------

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static int npart(int M) { return (M > 0 ? M : 1) + 3; }  // projection columns + three MGS buffers

size_t work_small_bytes(int M, int s) {
    int Mm = M > 0 ? M : 1;
    int ss = s > 0 ? s : 1;
    size_t b = 256;
    b += al256(sizeof(double) * (Mm + 1) * Mm);                  // H
    b += al256(sizeof(double) * Mm * Mm);                        // LU
    b += al256(sizeof(double) * ss * Mm);                        // phi
    b += al256(sizeof(double) * ss * Mm);                        // lam
    b += al256(sizeof(int) * Mm);                                // perm
    b += al256(sizeof(double) * (size_t)npart(M) * kRedBlocks);  // partials
    return b;
}

size_t work_bytes(long N, int M, int s, bool step) {
    size_t b = work_small_bytes(M, s);
    size_t vec = al256(sizeof(double) * (size_t)N);
    b += vec;                                          // w
    if (step) b += vec * ((size_t)M + 2 * (size_t)s);  // V, F, K
    return b;
}

Work carve(void* base, long N, int M, int s, bool step) {
    int Mm = M > 0 ? M : 1;
    int ss = s > 0 ? s : 1;
    char* p = (char*)base;
    Work W{};
    W.ints = (int*)p;
    W.scal = (double*)(p + 128);
    p += 256;
    W.H = (double*)p;        p += al256(sizeof(double) * (Mm + 1) * Mm);
    W.LU = (double*)p;       p += al256(sizeof(double) * Mm * Mm);
    W.phi = (double*)p;      p += al256(sizeof(double) * ss * Mm);
    W.lam = (double*)p;      p += al256(sizeof(double) * ss * Mm);
    W.perm = (int*)p;        p += al256(sizeof(int) * Mm);
    W.partials = (double*)p; p += al256(sizeof(double) * (size_t)npart(M) * kRedBlocks);
    W.npart = npart(M);
    size_t vec = al256(sizeof(double) * (size_t)N);
    W.w = (double*)p;        p += vec;
    if (step) {
        W.V = (double*)p;    p += vec * (size_t)M;
        W.F = (double*)p;    p += vec * (size_t)s;
        W.K = (double*)p;    p += vec * (size_t)s;
    }
    return W;
}

// Partial buffers: [0, Mm) projection columns, then three rotating MGS buffers.
static double* mgs_part(const Work& W, int k) { return W.partials + (size_t)(W.npart - 3 + (k % 3)) * kRedBlocks; }

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline unsigned grid_for(long n, int threads) {
    long g = (n + threads - 1) / threads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

#define ROK_RED(UPD, SELF, ...) \
    hipLaunchKernelGGL((k_red<UPD, SELF>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, __VA_ARGS__)

hipError_t launch_init(const Work& W, int M, int s, hipStream_t st) {
    int Mm = M > 0 ? M : 1;
    int ss = s > 0 ? s : 1;
    hipLaunchKernelGGL(k_init, dim3(16), dim3(256), 0, st, W.H, (Mm + 1) * Mm, W.phi, W.lam, ss * Mm, W.scal, W.ints,
                       M);
    return hipGetLastError();
}

hipError_t launch_norm_eps(const Work& W, const double* y, const double* v, long n, hipStream_t st) {
    if (v) {
        ROK_RED(false, true, (double*)v, nullptr, nullptr, nullptr, nullptr, n, nullptr, mgs_part(W, 1));
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, st, mgs_part(W, 1), (int)FIN_SQRT_TO, W.scal + 3,
                           W.scal, W.ints, 0);
    }
    ROK_RED(false, true, (double*)y, nullptr, nullptr, nullptr, nullptr, n, nullptr, mgs_part(W, 0));
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, st, mgs_part(W, 0), (int)FIN_EPS, nullptr, W.scal,
                       W.ints, v ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_start_basis(const Work& W, const double* f, long n, double* v0, hipStream_t st) {
    ROK_RED(false, true, (double*)f, nullptr, nullptr, nullptr, nullptr, n, W.ints, mgs_part(W, 0));
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, st, mgs_part(W, 0), (int)FIN_BETA, nullptr, W.scal,
                       W.ints, 0);
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(n, kRedThreads)), dim3(kRedThreads), 0, st, f, nullptr, W.H, 1, -1,
                       v0, n, W.ints, W.scal);
    return hipGetLastError();
}

// Orthogonalise w (= J v_j) against V[:, 0..j] by modified Gram-Schmidt;
// writes H[0..j, j] and, if j + 1 < M, H[j+1, j] and v_{j+1}.
hipError_t launch_mgs_column(const Work& W, double* w, const double* V, long n, int M, int j, double* vnext,
                             hipStream_t st) {
    for (int i = 0; i <= j; ++i) {
        const double* vcur = V + (long)i * n;
        if (i == 0) {
            ROK_RED(false, false, w, nullptr, nullptr, nullptr, vcur, n, W.ints, mgs_part(W, 0));
        } else {
            ROK_RED(true, false, w, V + (long)(i - 1) * n, mgs_part(W, i - 1), W.H + (long)(i - 1) * M + j, vcur, n,
                    W.ints, mgs_part(W, i));
        }
    }
    if (j + 1 < M) {
        ROK_RED(true, true, w, V + (long)j * n, mgs_part(W, j), W.H + (long)j * M + j, nullptr, n, W.ints,
                mgs_part(W, j + 1));
        hipLaunchKernelGGL(k_normalize, dim3(grid_for(n, kRedThreads)), dim3(kRedThreads), 0, st, w,
                           mgs_part(W, j + 1), W.H, M, j, vnext, n, W.ints, W.scal);
    } else {
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, st, mgs_part(W, j), (int)FIN_STORE,
                           W.H + (long)j * M + j, W.scal, W.ints, 0);
    }
    return hipGetLastError();
}

hipError_t launch_copy_h(const Work& W, int M, double* Hout, int* meff_out, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_h, dim3(grid_for((long)M * M, 256)), dim3(256), 0, st, W.H, M, Hout, W.ints, meff_out);
    return hipGetLastError();
}

hipError_t launch_lu(const Work& W, int M, double hg, hipStream_t st) {
    hipLaunchKernelGGL(k_lu, dim3(1), dim3(64), 0, st, W.H, M, hg, W.LU, W.perm, W.ints);
    return hipGetLastError();
}

hipError_t launch_project(const Work& W, const double* V, const double* F, long n, int M, hipStream_t st) {
#define ROK_PROJ(MB) \
    hipLaunchKernelGGL((k_project<MB>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, F, n, W.ints, W.partials)
    if (M <= 8) ROK_PROJ(8);
    else if (M <= 16) ROK_PROJ(16);
    else if (M <= 32) ROK_PROJ(32);
    else ROK_PROJ(64);
#undef ROK_PROJ
    return hipGetLastError();
}

hipError_t launch_lambda(const Work& W, int M, int i, const double* gam_row, double h, hipStream_t st) {
    GamRow gr{};
    for (int j = 0; j < kMaxStages; ++j) gr.g[j] = (j < i) ? gam_row[j] : 0.0;
    hipLaunchKernelGGL(k_lambda, dim3(1), dim3(kRedThreads), 0, st, W.H, W.LU, W.perm, M, i, gr, h, W.partials,
                       W.phi, W.lam, W.ints);
    return hipGetLastError();
}

hipError_t launch_recover(const Work& W, const double* V, const double* F, long n, int M, int i, double h, double* k,
                          hipStream_t st) {
    int Mm = M > 0 ? M : 1;
    hipLaunchKernelGGL(k_recover, dim3(grid_for(n, 256)), dim3(256), 0, st, V, F, n, W.ints, W.lam + (long)i * Mm,
                       W.phi + (long)i * Mm, h, k);
    return hipGetLastError();
}

hipError_t launch_update(const double* y, int s, const double* K, const double* b, long n, double* y1,
                         hipStream_t st) {
    BRow br{};
    for (int i = 0; i < kMaxStages; ++i) br.b[i] = (i < s) ? b[i] : 0.0;
    hipLaunchKernelGGL(k_update, dim3(grid_for(n, 256)), dim3(256), 0, st, y, s, K, br, n, y1);
    return hipGetLastError();
}

}  // namespace rok
