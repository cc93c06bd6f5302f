// One-reduce modified Gram-Schmidt for the Arnoldi columns (Sec. 2.2.2,
// modified Arnoldi), for exact (tangent) products when the work vector does
// not fit on chip.
//
// Modified Gram-Schmidt computes h_i = <q_i, w_i>, w_{i+1} = w_i - h_i q_i for
// i = 0..j, one dependent grid-wide sum per pass.  Written against the
// original w, the same coefficients are
//     h_i = <q_i, w> - sum_{l<i} <q_i, q_l> h_l,   i.e.  (I + L) h = r,
// with r = Q^T w and L the strictly lower part of Q^T Q (the inverse compact
// WY form of modified Gram-Schmidt): in exact arithmetic the same h, and the
// Gram correction gives the same loss of orthogonality as the pass-by-pass
// form.  A column then needs two sweeps over the basis instead of j + 1:
//   sweep A (k_ls_dots):   r_i = <q_i, w> (i <= j) and the new Gram row
//                          s_l = <q_j, q_l> (l < j), all partial sums at once
//   k_ls_solve (1 block):  finish the sums, L[j][l] = s_l, forward
//                          substitution (I + L) h = r, H[i][j] = h_i
//   sweep B (k_ls_update): w' = w - h_0 q_0 - h_1 q_1 - ... - h_j q_j (in that
//                          order), written as the next basis column, and the
//                          partial sums of ||w'||^2
// and the normalisation kernel of the pass-by-pass path finishes ||w'||, takes
// the breakdown decision and divides.  The last column (j = M - 1) needs only
// H's column: sweep A and the solve.
//
// Deferred normalisation (the basis a ROK step keeps for itself): the division
// pass is dropped.  Column j + 1 stays w' and its scale sig_{j+1} = 1 / ||w'||
// is kept on the device; the product J v_{j+1} takes the scale on its
// direction, the sums of sweep A are scaled after summation and sweep B, the
// projection and the recovery fold the scales into their coefficients.  In
// exact arithmetic nothing changes; one pass over a state vector less per
// column.
//
// Sums follow the canonical lane order of the other reductions (lane t of
// kRedBlocks x kRedThreads adds the elements t, t + T, ... in order, block
// trees, finished in order by one block), so results are deterministic; they
// round differently from the pass-by-pass form, whose finite-difference path
// stays the bitwise one.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"

namespace rok {

// Sweep A of column j over the MB-column bucket: partials of r_c = <q_c, w>
// (c = 0..j) at columns c and of s_c = <q_j, q_c> (c < j) at columns
// (MB + c) of `partials` (kRedBlocks each).
template <int MB>
__global__ __launch_bounds__(kRedThreads) void k_ls_dots(const double* V, const double* w, long n, int j,
                                                        const int* ints, double* partials) {
    if (ints[1]) return;
    double ar[MB], as[MB];
#pragma unroll
    for (int c = 0; c < MB; ++c) {
        ar[c] = 0.0;
        as[c] = 0.0;
    }
    const long stride = (long)kRedBlocks * kRedThreads;
    for (long e = (long)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += stride) {
        const double we = ld_stream(w + e);
        double q[MB];
#pragma unroll
        for (int c = 0; c < MB; ++c) q[c] = (c <= j) ? ld_stream(V + (long)c * n + e) : 0.0;
        double qj = 0.0;
#pragma unroll
        for (int c = 0; c < MB; ++c) qj = (c == j) ? q[c] : qj;
#pragma unroll
        for (int c = 0; c < MB; ++c) {
            if (c <= j) ar[c] = ar[c] + q[c] * we;
            if (c < j) as[c] = as[c] + qj * q[c];
        }
    }
    // the block's sums of every column at once (the canonical tree of each)
    __shared__ double sm[16][kRedThreads];
    tree256_chunks<0, MB>(ar, j + 1, sm, [&](int c, double b) { partials[(long)c * kRedBlocks + blockIdx.x] = b; });
    tree256_chunks<0, MB>(as, j, sm, [&](int c, double b) { partials[(long)(MB + c) * kRedBlocks + blockIdx.x] = b; });
}

constexpr int kSolveThreads = 4 * kRedThreads;   // four of the column's sums finished at once

// One block: finish r and s (canonical final sums), store the Gram row in L
// (row j, leading dimension M), solve (I + L) h = r by forward substitution in
// index order and write h into column j of H.  NONFINITE on a non-finite h.
// sig (non-null): the columns are stored unnormalised, q_c = sig_c V_c, and the
// sums over the stored columns are scaled: r_c = sig_c <V_c, w>,
// s_c = (sig_j sig_c) <V_j, V_c>.
__global__ __launch_bounds__(kSolveThreads) void k_ls_solve(const double* partials, int MB, int j, int M, double* L,
                                                           double* H, int* ints, const double* sig) {
    constexpr int kW = 24;   // widest compiled column
    __shared__ double s[kSolveThreads];
    __shared__ double sr[kMaxM], ss[kMaxM];
    __shared__ double sL[kW * kW], sh[kW];
    const int tid = threadIdx.x;
    const int grp = tid / kRedThreads, lane = tid % kRedThreads;
    // sums q = 0..j are r_q (partial column q), q = j+1..2j are s_{q-j-1}
    // (partial column MB + q - j - 1); each 256-thread group finishes one in
    // the canonical order
    const int nsum = 2 * j + 1;
    constexpr int G = kSolveThreads / kRedThreads;            // sums per round
    constexpr int R = (2 * kW - 1 + G - 1) / G;              // rounds for the widest column (M <= 24)
    static_assert(kRedBlocks == 4 * kRedThreads, "four partials per lane");
    // every partial this lane adds, loaded before any sum waits, and rows 0..j-1 of L
    // staged in LDS meanwhile: one memory round trip before the sums
    double pv[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = r * G + grp;
        const long col = (q <= j) ? q : MB + (q - j - 1);
#pragma unroll
        for (int u = 0; u < 4; ++u) pv[r][u] = (q < nsum) ? partials[col * kRedBlocks + lane + u * kRedThreads] : 0.0;
    }
    for (int e = tid; e < j * j; e += kSolveThreads) {
        const int r = e / j, c = e % j;
        if (c < r) sL[r * kW + c] = L[r * M + c];
    }
    if (ints[1]) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q0 = r * G;
        if (q0 >= nsum) break;
        const int q = q0 + grp;
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) a = a + pv[r][u];
        const double t = tree256(a, s);
        if (lane == 0 && q < nsum) {
            if (q <= j) {
                sr[q] = sig ? t * sig[q] : t;
            } else {
                const int c = q - j - 1;
                ss[c] = sig ? t * (sig[j] * sig[c]) : t;
            }
        }
        __syncthreads();
    }
    if (tid != 0) return;
    // (I + L) h = r by forward substitution, row j of L being the new s row
    for (int c = 0; c < j; ++c) L[j * M + c] = ss[c];
    bool bad = false;
    for (int i = 0; i <= j; ++i) {
        double hi = sr[i];
        for (int l = 0; l < i; ++l) hi = hi - (i < j ? sL[i * kW + l] : ss[l]) * sh[l];
        sh[i] = hi;
        H[i * M + j] = hi;
        bad = bad || !(hi == hi) || fabs(hi) == __builtin_inf();
    }
    if (bad) ints[2] |= ROK_FLAG_NONFINITE;
}

// Sweep B of column j: w' = w - h_0 q_0 - ... - h_j q_j into `out` (the next
// basis column, distinct from V's columns 0..j and from w), partials of
// ||w'||^2 at `partials`.  Two elements of a lane per iteration, both loaded
// before either is stored (the lane's sum keeps index order).  With sig, the
// coefficient of stored column c is h_c sig_c.  The column is stored with the
// non-temporal hint (it is read again only by the next product, from HBM).
template <int MB>
__global__ __launch_bounds__(kRedThreads) void k_ls_update(const double* __restrict__ V,
                                                          const double* __restrict__ w, const double* H, long n,
                                                          int j, int M, double* __restrict__ out, const int* ints,
                                                          double* partials, const double* sig) {
    __shared__ double s[kRedThreads];
    __shared__ double sh[MB];
    if (ints[1]) return;
    if (threadIdx.x < MB) {
        const int c = threadIdx.x;
        sh[c] = (c <= j) ? (sig ? H[c * M + j] * sig[c] : H[c * M + j]) : 0.0;
    }
    __syncthreads();
    double h[MB];
#pragma unroll
    for (int c = 0; c < MB; ++c) h[c] = sh[c];
    double acc = 0.0;
    const long stride = (long)kRedBlocks * kRedThreads;
    long e = (long)blockIdx.x * kRedThreads + threadIdx.x;
    for (; e + stride < n; e += 2 * stride) {
        double q0[MB], q1[MB];
#pragma unroll
        for (int c = 0; c < MB; ++c) {
            q0[c] = (c <= j) ? ld_stream(V + (long)c * n + e) : 0.0;
            q1[c] = (c <= j) ? ld_stream(V + (long)c * n + e + stride) : 0.0;
        }
        double x0 = ld_stream(w + e), x1 = ld_stream(w + e + stride);
#pragma unroll
        for (int c = 0; c < MB; ++c)
            if (c <= j) {
                x0 = x0 - h[c] * q0[c];
                x1 = x1 - h[c] * q1[c];
            }
        __builtin_nontemporal_store(x0, out + e);
        __builtin_nontemporal_store(x1, out + e + stride);
        acc = acc + x0 * x0;
        acc = acc + x1 * x1;
    }
    if (e < n) {
        double x = ld_stream(w + e);
#pragma unroll
        for (int c = 0; c < MB; ++c)
            if (c <= j) x = x - h[c] * ld_stream(V + (long)c * n + e);
        __builtin_nontemporal_store(x, out + e);
        acc = acc + x * x;
    }
    const double b = tree256(acc, s);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// Smallest compiled column count >= j + 1 (0 if the column is too wide for the register arrays).
static int ls_bucket(int cols) {
    static const int b[] = {1, 2, 4, 8, 12, 16, 20, 24};
    for (int x : b)
        if (cols <= x) return x;
    return 0;
}

bool lowsync_supported(int M) { return M >= 1 && ls_bucket(M) > 0; }

hipError_t launch_ls_column(const Work& W, const double* w, const double* V, long n, int M, int j, double* vnext,
                            hipStream_t st, bool deferred) {
    const double* sig = deferred ? W.sig : nullptr;
    const int MB = ls_bucket(j + 1);
    if (MB == 0 || 2 * MB + 1 > W.npart) return hipErrorInvalidValue;   // r, s and the norm's partial columns
    double* part = W.partials;
#define ROK_LS_DOTS(B)                                                                                          \
    hipLaunchKernelGGL((k_ls_dots<B>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, w, n, j, W.ints, part)
    switch (MB) {
        case 1: ROK_LS_DOTS(1); break;
        case 2: ROK_LS_DOTS(2); break;
        case 4: ROK_LS_DOTS(4); break;
        case 8: ROK_LS_DOTS(8); break;
        case 12: ROK_LS_DOTS(12); break;
        case 16: ROK_LS_DOTS(16); break;
        case 20: ROK_LS_DOTS(20); break;
        default: ROK_LS_DOTS(24); break;
    }
#undef ROK_LS_DOTS
    hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(kSolveThreads), 0, st, part, MB, j, M, W.L, W.H, W.ints, sig);
    if (j + 1 < M) {
        double* npart = W.partials + (long)(W.npart - 1) * kRedBlocks;   // the last partial column
#define ROK_LS_UPD(B)                                                                                            \
    hipLaunchKernelGGL((k_ls_update<B>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, w, W.H, n, j, M, vnext, \
                       W.ints, npart, sig)
        switch (MB) {
            case 1: ROK_LS_UPD(1); break;
            case 2: ROK_LS_UPD(2); break;
            case 4: ROK_LS_UPD(4); break;
            case 8: ROK_LS_UPD(8); break;
            case 12: ROK_LS_UPD(12); break;
            case 16: ROK_LS_UPD(16); break;
            case 20: ROK_LS_UPD(20); break;
            default: ROK_LS_UPD(24); break;
        }
#undef ROK_LS_UPD
        if (deferred)   // ||w'||, breakdown test, sig_{j+1} = 1 / ||w'||; the column stays w'
            launch_norm_scale(W, npart, M, j, st);
        else            // ||w'|| finished in every block, breakdown test, v_{j+1} = w' / ||w'|| in place
            launch_normalize(W, vnext, npart, M, j, vnext, n, st);
    }
    return hipGetLastError();
}

}  // namespace rok
