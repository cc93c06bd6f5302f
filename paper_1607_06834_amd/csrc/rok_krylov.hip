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
constexpr double kEpsMach = 2.220446049250313e-16;   // 2^-52

// Block of kRedThreads threads: the halving tree; every thread gets the sum.
__device__ __forceinline__ double block_sum(double acc, double* s) {
    __shared__ double s_r;
    double r = tree256(acc, s);
    if (threadIdx.x == 0) s_r = r;
    __syncthreads();
    r = s_r;
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
        double w0 = ld_stream(w + e), w1 = ld_stream(w + e + stride);
        if constexpr (UPD) {
            double a0 = ld_stream(vprev + e), a1 = ld_stream(vprev + e + stride);
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
            b0 = ld_stream(vcur + e);
            b1 = ld_stream(vcur + e + stride);
        }
        acc = acc + b0 * w0;
        acc = acc + b1 * w1;
    }
    if (e < n) {
        double we = ld_stream(w + e);
        if constexpr (UPD) {
            we = we - h * ld_stream(vprev + e);
            w[e] = we;
        }
        if constexpr (SELF) acc = acc + we * we;
        else acc = acc + ld_stream(vcur + e) * we;
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
    } else {  // FIN_EPS: eps = sqrt((1 + ||y||) u) [/ ||v||]
        double ny = sqrt(tot);
        scal[0] = ny;
        double e = sqrt((1.0 + ny) * kEpsMach);
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
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) v[e] = ld_stream(w + e) / hn;
}

// The normalisation's bookkeeping without the division: h_{j+1,j} = sqrt(w.w)
// from `partials`, the breakdown test of k_normalize, and sig[j+1] =
// 1 / h_{j+1,j}, the scale of the unnormalised column (one block).
__global__ __launch_bounds__(kRedThreads) void k_norm_scale(const double* partials, double* H, int M, int j,
                                                           int* ints, double* sig) {
    __shared__ double s[kRedThreads];
    if (ints[1]) return;
    const double hn = sqrt(final_sum(partials, s));
    if (threadIdx.x != 0) return;
    double c = 0.0;
    for (int i = 0; i <= j; ++i) c = c + H[i * M + j] * H[i * M + j];
    c = c + hn * hn;
    H[(j + 1) * M + j] = hn;
    if (hn <= kBreakdownTol * sqrt(c)) {
        ints[0] = j + 1;
        ints[1] = 1;
        ints[2] |= ROK_FLAG_BREAKDOWN;
    } else {
        sig[j + 1] = 1.0 / hn;
    }
    if (nonfinite(hn)) ints[2] |= ROK_FLAG_NONFINITE;
}

__global__ void k_init(double* H, int nh, double* phi, double* lam, int nsm, double* scal, int* ints, int meff0,
                       unsigned* bar, double* sig, int nsig) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int e = t; e < kBarWords; e += gridDim.x * blockDim.x) bar[e] = 0u;
    for (int e = t; e < nsig; e += gridDim.x * blockDim.x) sig[e] = 1.0;
    for (int e = t; e < nh; e += gridDim.x * blockDim.x) H[e] = 0.0;
    for (int e = t; e < nsm; e += gridDim.x * blockDim.x) {
        phi[e] = 0.0;
        lam[e] = 0.0;
    }
    if (t < 16) scal[t] = 0.0;
    if (t < 32) ints[t] = (t == 0) ? meff0 : 0;   // M_eff, stop, flags, barrier words
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

// LU with partial pivoting of A = I - hg H (M_eff x M_eff) in LDS, one block.
// Each entry sees the same sequence of operations as the textbook
// right-looking elimination; rows (and columns) are updated in parallel.
__global__ __launch_bounds__(kRedThreads) void k_lu(const double* H, int M, double hg, double* LU, int* perm,
                                                   const int* ints) {
    __shared__ double A[kMaxM * kMaxM];
    __shared__ int P[kMaxM];
    __shared__ int s_piv;
    const int m = ints[0];
    const int tid = threadIdx.x;
    for (int e = tid; e < m * m; e += blockDim.x) {
        int i = e / m, j = e % m;
        A[i * kMaxM + j] = (i == j ? 1.0 : 0.0) - hg * H[i * M + j];
    }
    for (int i = tid; i < m; i += blockDim.x) P[i] = i;
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (tid == 0) {
            int piv = k;
            for (int r = k + 1; r < m; ++r)
                if (fabs(A[r * kMaxM + k]) > fabs(A[piv * kMaxM + k])) piv = r;
            s_piv = piv;
            if (piv != k) {
                int t = P[k];
                P[k] = P[piv];
                P[piv] = t;
            }
        }
        __syncthreads();
        const int piv = s_piv;
        if (piv != k) {
            for (int c = tid; c < m; c += blockDim.x) {
                double t = A[k * kMaxM + c];
                A[k * kMaxM + c] = A[piv * kMaxM + c];
                A[piv * kMaxM + c] = t;
            }
        }
        __syncthreads();
        for (int r = k + 1 + tid; r < m; r += blockDim.x) A[r * kMaxM + k] = A[r * kMaxM + k] / A[k * kMaxM + k];
        __syncthreads();
        const int w = m - k - 1;
        for (int e = tid; e < w * w; e += blockDim.x) {
            int r = k + 1 + e / w, c = k + 1 + e % w;
            A[r * kMaxM + c] = A[r * kMaxM + c] - A[r * kMaxM + k] * A[k * kMaxM + c];
        }
        __syncthreads();
    }
    for (int e = tid; e < m * m; e += blockDim.x) {
        int i = e / m, j = e % m;
        LU[i * M + j] = A[i * kMaxM + j];
    }
    for (int i = tid; i < m; i += blockDim.x) perm[i] = P[i];
}

struct GamRow {
    double g[kMaxStages];
};

// The value of v held by lane `lane` (uniform across the wave) of the calling wave.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// phi_i = V^T F_i finished from the projection partials (all columns at once,
// canonical order per column), then
// lambda_i = LU^{-1} (h phi_i + h H sum_{j<i} gamma_ij lambda_j) on the same block.
__global__ __launch_bounds__(kRedThreads) void k_lambda(const double* H, const double* LU, const int* perm, int M,
                                                       int i, GamRow gr, double h, const double* partials,
                                                       double* phi, double* lam, int* ints, const double* sig) {
    __shared__ double s[16][kRedThreads];
    __shared__ double sphi[kMaxM];
    __shared__ double sLU[kMaxM * kMaxM], sH[kMaxM * kMaxM];
    __shared__ double g[kMaxM];
    __shared__ int sperm[kMaxM];
    const int tid = threadIdx.x;
    // Every load whose address does not depend on M_eff is issued first, for the
    // compiled size M (entries past M_eff are loaded and never used): the first
    // 16 columns' partials (lane tid adds partials tid, tid + 256, tid + 512,
    // tid + 768 of each column in order), then LU, H, the pivots and the earlier
    // lambdas, staged in LDS; one round trip to memory instead of three.
    static_assert(kRedBlocks == 4 * kRedThreads, "four partials per lane");
    const int n16 = M < 16 ? M : 16;
    double pv[16][4];
#pragma unroll
    for (int c = 0; c < 16; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) pv[c][q] = (c < n16) ? partials[(long)c * kRedBlocks + tid + q * kRedThreads] : 0.0;
    for (int e = tid; e < M * M; e += kRedThreads) {
        const int r = e / M, c = e % M;
        sLU[r * kMaxM + c] = LU[e];
        sH[r * kMaxM + c] = H[e];
    }
    if (tid < M) {
        sperm[tid] = perm[tid];
        double a = 0.0;
        for (int j = 0; j < i; ++j)
            if (gr.g[j] != 0.0) a = a + gr.g[j] * lam[j * M + tid];
        g[tid] = a;
    }
    const int m = ints[0];
    for (int c0 = 0; c0 < m; c0 += 16) {
        const int nc = (m - c0) < 16 ? (m - c0) : 16;
        if (c0 > 0) {   // columns past the first 16 (M > 16)
#pragma unroll
            for (int c = 0; c < 16; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    pv[c][q] = (c < nc) ? partials[(long)(c0 + c) * kRedBlocks + tid + q * kRedThreads] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (c < nc) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc = acc + pv[c][q];
                s[c][tid] = acc;
            }
        }
        __syncthreads();
        for (int st = kRedThreads / 2; st > 0; st >>= 1) {
            if (tid < st)
                for (int c = 0; c < nc; ++c) s[c][tid] = s[c][tid] + s[c][tid + st];
            __syncthreads();
        }
        // a column stored unnormalised: <v_c, F> = sig_c <V_c, F>
        if (tid < nc) sphi[c0 + tid] = sig ? s[tid][0] * sig[c0 + tid] : s[tid][0];
        __syncthreads();
    }
    if (tid < m) phi[i * M + tid] = sphi[tid];
    // The reduced solve: the right-hand side row-parallel, the forward substitution
    // column-parallel (each entry still sees its updates in increasing column order),
    // the back substitution one row at a time (each row's sum in increasing column
    // order) with the finished entries broadcast from their lanes.
    // From here on wave 0 alone (m <= kMaxM = 64: row r on lane r), with no block barrier:
    // lane values move by lane shuffles and broadcasts.
    if (tid >= 64) return;
    double x = 0.0;
    if (tid < m) {   // x_r = h phi_r + h (H g)_r
        double hg = 0.0;
        for (int c = 0; c < m; ++c) hg = hg + sH[tid * kMaxM + c] * g[c];
        x = h * sphi[tid] + h * hg;
    }
    double yr = __shfl(x, tid < m ? sperm[tid] : tid, 64);   // placed at its pivoted position
    for (int c = 0; c + 1 < m; ++c) {   // forward substitution with the unit lower factor
        const double yc = lane_value(yr, c);
        if (tid > c && tid < m) yr = yr - sLU[tid * kMaxM + c] * yc;
    }
    for (int r = m - 1; r >= 0; --r) {   // back substitution: row r's sum in increasing column order
        double a = lane_value(yr, r);
        for (int c = r + 1; c < m; ++c) a = a - sLU[r * kMaxM + c] * lane_value(yr, c);
        a = a / sLU[r * kMaxM + r];
        if (tid == r) yr = a;
    }
    if (tid < m) lam[i * M + tid] = yr;
    const bool bad = __any(tid < m && nonfinite(yr));
    if (tid == 0 && bad) ints[2] |= ROK_FLAG_NONFINITE;
}

// Projection partials: for c < M_eff, canonical per-block partial sums of
// V[:, c] . F (finished by k_lambda).  MB >= M; the common case M_eff == MB
// runs a branch-free loop so all loads of an element are in flight together.
template <int MB>
__global__ __launch_bounds__(kRedThreads) void k_project(const double* V, const double* F, long n, const int* ints,
                                                        double* partials) {
    const int m = ints[0];
    double acc[MB];
#pragma unroll
    for (int c = 0; c < MB; ++c) acc[c] = 0.0;
    const long stride = (long)kRedBlocks * kRedThreads;
    if (m == MB) {
        for (long e = (long)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += stride) {
            double fe = ld_stream(F + e);
            double vc[MB];
#pragma unroll
            for (int c = 0; c < MB; ++c) vc[c] = ld_stream(V + (long)c * n + e);
#pragma unroll
            for (int c = 0; c < MB; ++c) acc[c] = acc[c] + vc[c] * fe;
        }
    } else {
        for (long e = (long)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += stride) {
            double fe = ld_stream(F + e);
#pragma unroll
            for (int c = 0; c < MB; ++c)
                if (c < m) acc[c] = acc[c] + ld_stream(V + (long)c * n + e) * fe;
        }
    }
    __shared__ double sm[16][kRedThreads];
    tree256_chunks<0, MB>(acc, m, sm, [&](int c, double b) { partials[(long)c * kRedBlocks + blockIdx.x] = b; });
}

struct BRow {
    double b[kMaxStages];
};

// k = V lambda + h (F - V phi), column sums in order from zero.  FINAL: the
// last stage, which writes y_{n+1} = y + sum_i b_i k_i instead of k.  Other
// stages i with ynext: also the next stage's input Y_{i+1} = y + sum_{q<=i}
// a_q k_q (a = row i + 1 of alpha; terms with a_q = 0 skipped, k_i from
// registers), in the order the residual forms it from y and the k_q
// (sum in stage order, terms with b_i = 0 skipped).
template <int MB, bool FINAL>
__global__ __launch_bounds__(256) void k_recover(const double* __restrict__ V, const double* __restrict__ F, long n,
                                                const int* ints, const double* lam, const double* phi, double h,
                                                double* __restrict__ k, const double* __restrict__ y,
                                                const double* __restrict__ K, int s, BRow br, const double* sig,
                                                double* __restrict__ ynext, int stage, BRow ar) {
    const int m = ints[0];
    // columns stored unnormalised (v_c = sig_c V_c): the scales go into the coefficients
    auto lamc = [&](int c) { return sig ? lam[c] * sig[c] : lam[c]; };
    auto phic = [&](int c) { return sig ? phi[c] * sig[c] : phi[c]; };
    double lm[MB], ph[MB];
    if (m == MB) {
#pragma unroll
        for (int c = 0; c < MB; ++c) {
            lm[c] = lamc(c);
            ph[c] = phic(c);
        }
    }
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double a = 0.0, b = 0.0;
        if (m == MB) {
            double vc[MB];
#pragma unroll
            for (int c = 0; c < MB; ++c) vc[c] = ld_stream(V + (long)c * n + e);
#pragma unroll
            for (int c = 0; c < MB; ++c) {
                a = a + vc[c] * lm[c];
                b = b + vc[c] * ph[c];
            }
        } else {
            for (int c = 0; c < m; ++c) {
                double vc = ld_stream(V + (long)c * n + e);
                a = a + vc * lamc(c);
                b = b + vc * phic(c);
            }
        }
        double ke = a + h * (ld_stream(F + e) - b);
        if constexpr (FINAL) {
            double acc = ld_stream(y + e);
            for (int i = 0; i < s - 1; ++i)
                if (br.b[i] != 0.0) acc = acc + br.b[i] * ld_stream(K + (long)i * n + e);
            if (br.b[s - 1] != 0.0) acc = acc + br.b[s - 1] * ke;
            k[e] = acc;
        } else {
            k[e] = ke;
            if (ynext) {
                double acc = ld_stream(y + e);
                for (int q = 0; q < stage; ++q)
                    if (ar.b[q] != 0.0) acc = acc + ar.b[q] * ld_stream(K + (long)q * n + e);
                if (ar.b[stage] != 0.0) acc = acc + ar.b[stage] * ke;
                ynext[e] = acc;
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Workspace: a 256-byte header (status ints, scalars) at offset 0 for every M
// and s, then the small matrices, the reduction partials and the vectors.
// ---------------------------------------------------------------------------

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Partial columns: the projections (M) and three rotating MGS buffers, or the one-reduce Gram-Schmidt's
// r and s columns (twice the compiled width of its widest column) and its norm column, whichever is more.
static int npart(int M) {
    const int Mm = M > 0 ? M : 1;
    int ls = 0;
    if (lowsync_supported(Mm)) {
        static const int b[] = {1, 2, 4, 8, 12, 16, 20, 24};
        for (int x : b)
            if (Mm <= x) {
                ls = 2 * x + 1;
                break;
            }
    }
    return Mm + 3 > ls ? Mm + 3 : ls;
}

size_t work_small_bytes(int M, int s) {
    int Mm = M > 0 ? M : 1;
    int ss = s > 0 ? s : 1;
    size_t b = 256;
    b += al256(sizeof(double) * (Mm + 1) * Mm);                  // H
    b += al256(sizeof(double) * Mm * Mm);                        // LU
    b += al256(sizeof(double) * ss * Mm);                        // phi
    b += al256(sizeof(double) * ss * Mm);                        // lam
    b += al256(sizeof(int) * Mm);                                // perm
    b += al256(sizeof(double) * Mm * Mm);                        // L
    b += al256(sizeof(double) * (Mm + 1));                       // sig
    b += al256(sizeof(double) * (size_t)npart(M) * kRedBlocks);  // partials
    b += al256(sizeof(double) * 2 * kRedBlocks);                 // gpart
    b += al256(sizeof(unsigned) * kBarWords);                    // barrier
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
    W.L = (double*)p;        p += al256(sizeof(double) * Mm * Mm);
    W.sig = (double*)p;      p += al256(sizeof(double) * (Mm + 1));
    W.partials = (double*)p; p += al256(sizeof(double) * (size_t)npart(M) * kRedBlocks);
    W.npart = npart(M);
    W.gpart = (double*)p;    p += al256(sizeof(double) * 2 * kRedBlocks);
    W.bar = (unsigned*)p;    p += al256(sizeof(unsigned) * kBarWords);
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

// Weighted RMS norm of a step-doubling error estimate: lane sums of q_i^2 in
// the canonical order, q_i = (a_i - b_i) / (c (atol + rtol max(|y_i|, |a_i|))).
// The maximum propagates a NaN of either operand.
__global__ __launch_bounds__(kRedThreads) void k_err_partials(const double* y, const double* a, const double* b,
                                                             long n, double rtol, double atol, double c,
                                                             double* partials) {
    __shared__ double s[kRedThreads];
    double acc = 0.0;
    const long stride = (long)kRedBlocks * kRedThreads;
    for (long e = (long)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += stride) {
        const double ay = fabs(y[e]), aa = fabs(a[e]);
        const double m = (ay != ay || ay > aa) ? ay : aa;
        const double sc = atol + rtol * m;
        const double q = (a[e] - b[e]) / (c * sc);
        acc = acc + q * q;
    }
    double bs = block_sum(acc, s);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// *out = sqrt(sum / n) from the partials.
__global__ __launch_bounds__(kRedThreads) void k_err_finish(const double* partials, double n, double* out) {
    __shared__ double s[kRedThreads];
    double tot = final_sum(partials, s);
    if (threadIdx.x == 0) *out = sqrt(tot / n);
}

#define ROK_RED(UPD, SELF, ...) \
    hipLaunchKernelGGL((k_red<UPD, SELF>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, __VA_ARGS__)

hipError_t launch_init(const Work& W, int M, int s, hipStream_t st) {
    int Mm = M > 0 ? M : 1;
    int ss = s > 0 ? s : 1;
    hipLaunchKernelGGL(k_init, dim3(16), dim3(256), 0, st, W.H, (Mm + 1) * Mm, W.phi, W.lam, ss * Mm, W.scal, W.ints,
                       M, W.bar, W.sig, Mm + 1);
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

hipError_t launch_error_norm(const Work& W, const double* y, const double* a, const double* b, long n, double rtol,
                             double atol, double c, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_err_partials, dim3(kRedBlocks), dim3(kRedThreads), 0, st, y, a, b, n, rtol, atol, c,
                       mgs_part(W, 0));
    hipLaunchKernelGGL(k_err_finish, dim3(1), dim3(kRedThreads), 0, st, mgs_part(W, 0), (double)n, out);
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

hipError_t launch_normalize(const Work& W, const double* w, const double* partials, int M, int j, double* v, long n,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(n, kRedThreads)), dim3(kRedThreads), 0, st, w, partials, W.H, M, j,
                       v, n, W.ints, W.scal);
    return hipGetLastError();
}

hipError_t launch_norm_scale(const Work& W, const double* partials, int M, int j, hipStream_t st) {
    hipLaunchKernelGGL(k_norm_scale, dim3(1), dim3(kRedThreads), 0, st, partials, W.H, M, j, W.ints, W.sig);
    return hipGetLastError();
}

hipError_t launch_copy_h(const Work& W, int M, double* Hout, int* meff_out, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_h, dim3(grid_for((long)M * M, 256)), dim3(256), 0, st, W.H, M, Hout, W.ints, meff_out);
    return hipGetLastError();
}

hipError_t launch_lu(const Work& W, int M, double hg, hipStream_t st) {
    hipLaunchKernelGGL(k_lu, dim3(1), dim3(kRedThreads), 0, st, W.H, M, hg, W.LU, W.perm, W.ints);
    return hipGetLastError();
}

// Smallest compiled column count >= M.
static int mbucket(int M) {
    static const int b[] = {1, 2, 4, 8, 12, 16, 20, 24, 32, 48, 64};
    for (int x : b)
        if (M <= x) return x;
    return 64;
}

#define ROK_MB_SWITCH(MBV, CALL)       \
    switch (MBV) {                     \
        case 1: CALL(1); break;        \
        case 2: CALL(2); break;        \
        case 4: CALL(4); break;        \
        case 8: CALL(8); break;        \
        case 12: CALL(12); break;      \
        case 16: CALL(16); break;      \
        case 20: CALL(20); break;      \
        case 24: CALL(24); break;      \
        case 32: CALL(32); break;      \
        case 48: CALL(48); break;      \
        default: CALL(64); break;      \
    }

// The first stage's projection without a pass over the basis: F_1 = f(y_n) =
// beta v_0 (the basis starts from it), so phi_1 = V^T F_1 = beta e_1 in exact
// arithmetic.  Leaves partials that k_lambda finishes to exactly that:
// column 0 holds beta in its first partial, every other partial is zero.
__global__ __launch_bounds__(kRedThreads) void k_project_first(int M, const double* scal, double* partials) {
    const long t = (long)blockIdx.x * kRedThreads + threadIdx.x;
    if (t < (long)M * kRedBlocks) partials[t] = (t == 0) ? scal[2] : 0.0;
}

hipError_t launch_project_first(const Work& W, int M, hipStream_t st) {
    const long n = (long)(M > 0 ? M : 1) * kRedBlocks;
    hipLaunchKernelGGL(k_project_first, dim3((unsigned)((n + kRedThreads - 1) / kRedThreads)), dim3(kRedThreads), 0,
                       st, M, W.scal, W.partials);
    return hipGetLastError();
}

hipError_t launch_project(const Work& W, const double* V, const double* F, long n, int M, hipStream_t st) {
#define ROK_PROJ(MB) \
    hipLaunchKernelGGL((k_project<MB>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, F, n, W.ints, W.partials)
    ROK_MB_SWITCH(mbucket(M), ROK_PROJ)
#undef ROK_PROJ
    return hipGetLastError();
}

hipError_t launch_lambda(const Work& W, int M, int i, const double* gam_row, double h, hipStream_t st,
                         const double* sig) {
    GamRow gr{};
    for (int j = 0; j < kMaxStages; ++j) gr.g[j] = (j < i) ? gam_row[j] : 0.0;
    hipLaunchKernelGGL(k_lambda, dim3(1), dim3(kRedThreads), 0, st, W.H, W.LU, W.perm, M, i, gr, h, W.partials,
                       W.phi, W.lam, W.ints, sig);
    return hipGetLastError();
}

hipError_t launch_recover(const Work& W, const double* V, const double* F, long n, int M, int i, double h, double* k,
                          const double* y, const double* K, int s, const double* b, hipStream_t st,
                          const double* sig, double* ynext, const double* arow) {
    int Mm = M > 0 ? M : 1;
    BRow br{}, ar{};
    for (int q = 0; q < kMaxStages; ++q) br.b[q] = (b && q < s) ? b[q] : 0.0;
    for (int q = 0; q < kMaxStages; ++q) ar.b[q] = (arow && q <= i) ? arow[q] : 0.0;
    if (ynext && (!y || !K)) return hipErrorInvalidValue;
    const bool fin = y && !ynext;   // the last stage: y_{n+1} into k
    const double* lam = W.lam + (long)i * Mm;
    const double* phi = W.phi + (long)i * Mm;
    const unsigned g = grid_for(n, 256);
#define ROK_REC(MB)                                                                                             \
    if (fin) hipLaunchKernelGGL((k_recover<MB, true>), dim3(g), dim3(256), 0, st, V, F, n, W.ints, lam, phi, h,  \
                                k, y, K, s, br, sig, nullptr, 0, ar);                                         \
    else hipLaunchKernelGGL((k_recover<MB, false>), dim3(g), dim3(256), 0, st, V, F, n, W.ints, lam, phi, h, k,  \
                            y, K, s, br, sig, ynext, i, ar)
    ROK_MB_SWITCH(mbucket(M > 0 ? M : 1), ROK_REC)
#undef ROK_REC
    return hipGetLastError();
}

}  // namespace rok
