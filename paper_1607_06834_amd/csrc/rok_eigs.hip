// Pieces of the matrix-free eigenvalue estimate of J (the stiffness
// diagnostic of Sec. 4, by implicitly restarted Arnoldi): the basis
// recombination kernel V_out = V C, and the small dense host routines on the
// Hessenberg matrix (its eigenvalues, the shifted QR steps of a restart, and
// the residual estimate of a Ritz value).  The driver is rok_eigs in
// rok_api.hip.
#include <math.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "rok_device.hpp"
#include "rok_kernels.hpp"

namespace rok {

// ---------------------------------------------------------------------------
// V_out[:, c] = sum_i V[:, i] C[i, c]   (i = 0..m1-1 in order, c = 0..nc-1)
// V and V_out are column-major with leading dimension n; C is m1 x nc
// column-major.  Each thread owns one row e and accumulates kChunk outputs at
// a time, so V is read ceil(nc / kChunk) times.
// ---------------------------------------------------------------------------
constexpr int kChunk = 8;

__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ V, long n, int m1,
                                                 const double* __restrict__ C, int nc, double* __restrict__ Vout) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    for (int c0 = 0; c0 < nc; c0 += kChunk) {
        double acc[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) acc[q] = 0.0;
        for (int i = 0; i < m1; ++i) {
            const double v = V[(long)i * n + e];
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
                if (c0 + q < nc) acc[q] = acc[q] + v * C[(long)(c0 + q) * m1 + i];
        }
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
            if (c0 + q < nc) Vout[(long)(c0 + q) * n + e] = acc[q];
    }
}

hipError_t launch_combine(const double* V, long n, int m1, const double* C, int nc, double* Vout, hipStream_t st) {
    if (n <= 0 || m1 <= 0 || nc <= 0) return hipSuccess;
    const long nb = (n + 255) / 256;
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_combine, dim3((unsigned)nb), dim3(256), 0, st, V, n, m1, C, nc, Vout);
    return hipGetLastError();
}

namespace dense {

using cd = std::complex<double>;
constexpr double kEps = 2.220446049250313e-16;

// Eigenvalues of the leading n x n block of the real upper Hessenberg H
// (row-major, leading dimension ldh) by shifted QR iteration in complex
// arithmetic: Givens rotations, Wilkinson shifts from the trailing 2 x 2
// block of the active window, deflation where a subdiagonal entry falls
// below eps (|h_ii| + |h_{i-1,i-1}|), an exceptional shift every eleventh
// iteration without deflation.  Returns false if it did not converge.
bool hessenberg_eigenvalues(int n, const double* H, int ldh, double* wr, double* wi) {
    std::vector<cd> A((size_t)n * n, cd(0.0, 0.0));
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - 1); j < n; ++j) {
            A[(size_t)i * n + j] = cd(H[(size_t)i * ldh + j], 0.0);
            anorm = std::max(anorm, fabs(H[(size_t)i * ldh + j]));
        }
    if (anorm == 0.0) anorm = 1.0;
    auto a = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
    std::vector<cd> gc(n), gs(n);
    int hi = n - 1, iter = 0;
    while (hi >= 0) {
        if (hi == 0) {
            wr[0] = a(0, 0).real();
            wi[0] = a(0, 0).imag();
            --hi;
            continue;
        }
        int l = hi;
        while (l > 0) {
            double s = std::abs(a(l, l)) + std::abs(a(l - 1, l - 1));
            if (s == 0.0) s = anorm;
            if (std::abs(a(l, l - 1)) <= kEps * s) {
                a(l, l - 1) = 0.0;
                break;
            }
            --l;
        }
        if (l == hi) {
            wr[hi] = a(hi, hi).real();
            wi[hi] = a(hi, hi).imag();
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 60 * n) return false;
        const cd p = a(hi - 1, hi - 1), q = a(hi - 1, hi), r = a(hi, hi - 1), d = a(hi, hi);
        cd mu;
        if (iter % 11 == 10) {
            mu = d + cd(0.75 * std::abs(r), 0.0);
        } else {
            const cd half_tr = 0.5 * (p + d);
            const cd disc = std::sqrt(half_tr * half_tr - (p * d - q * r));
            const cd m1 = half_tr + disc, m2 = half_tr - disc;
            mu = (std::abs(m1 - d) <= std::abs(m2 - d)) ? m1 : m2;
        }
        for (int i = l; i <= hi; ++i) a(i, i) -= mu;
        for (int i = l; i < hi; ++i) {
            const cd x = a(i, i), y = a(i + 1, i);
            const double nr = std::sqrt(std::norm(x) + std::norm(y));
            cd c(1.0, 0.0), s(0.0, 0.0);
            if (nr > 0.0) {
                c = x / nr;
                s = y / nr;
            }
            gc[i] = c;
            gs[i] = s;
            for (int j = i; j <= hi; ++j) {   // rows i, i+1 <- G [row i; row i+1], G = [c* s*; -s c]
                const cd t1 = a(i, j), t2 = a(i + 1, j);
                a(i, j) = std::conj(c) * t1 + std::conj(s) * t2;
                a(i + 1, j) = -s * t1 + c * t2;
            }
        }
        for (int i = l; i < hi; ++i) {        // columns i, i+1 <- [col i, col i+1] G^H
            const cd c = gc[i], s = gs[i];
            const int rmax = std::min(i + 2, hi);
            for (int rr = l; rr <= rmax; ++rr) {
                const cd t1 = a(rr, i), t2 = a(rr, i + 1);
                a(rr, i) = t1 * c + t2 * s;
                a(rr, i + 1) = -t1 * std::conj(s) + t2 * std::conj(c);
            }
        }
        for (int i = l; i <= hi; ++i) a(i, i) += mu;
    }
    return true;
}

// Reflector I - beta v v^T (v of length len at rows/columns r..r+len-1)
// applied as H <- P H P (left on columns c0..m-1, right on rows 0..rmax) and
// Qacc <- Qacc P.
static void reflect(int m, double* H, int ldh, double* Q, int r, int len, const double* v, double beta, int c0,
                    int rmax) {
    for (int c = c0; c < m; ++c) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += v[i] * H[(size_t)(r + i) * ldh + c];
        s *= beta;
        for (int i = 0; i < len; ++i) H[(size_t)(r + i) * ldh + c] -= s * v[i];
    }
    for (int rr = 0; rr <= rmax; ++rr) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += H[(size_t)rr * ldh + r + i] * v[i];
        s *= beta;
        for (int i = 0; i < len; ++i) H[(size_t)rr * ldh + r + i] -= s * v[i];
    }
    for (int rr = 0; rr < m; ++rr) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += Q[(size_t)rr * m + r + i] * v[i];
        s *= beta;
        for (int i = 0; i < len; ++i) Q[(size_t)rr * m + r + i] -= s * v[i];
    }
}

// Householder vector of u (length len): (I - beta v v^T) u = alpha e_1.
static double householder(const double* u, int len, double* v) {
    double nu = 0.0;
    for (int i = 0; i < len; ++i) nu += u[i] * u[i];
    nu = std::sqrt(nu);
    for (int i = 0; i < len; ++i) v[i] = u[i];
    if (nu == 0.0) return 0.0;
    const double alpha = u[0] >= 0.0 ? -nu : nu;
    v[0] = u[0] - alpha;
    double vv = 0.0;
    for (int i = 0; i < len; ++i) vv += v[i] * v[i];
    return vv == 0.0 ? 0.0 : 2.0 / vv;
}

// One exact-shift QR step of a restart on the m x m Hessenberg H (row-major,
// leading dimension ldh), done implicitly (bulge chasing) so that the result
// stays Hessenberg: H <- Q^T H Q with Q the orthogonal factor of
// H - mu I (real shift) or of H^2 - 2 Re(mu) H + |mu|^2 I (a complex
// conjugate pair, Francis' double shift); Qacc <- Qacc Q (m x m, row-major).
void shift_step(int m, double* H, int ldh, double* Qacc, double mre, double mim, bool pair) {
    auto h = [&](int i, int j) -> double& { return H[(size_t)i * ldh + j]; };
    double u[3], v[3];
    if (!pair || m < 3) {
        u[0] = h(0, 0) - mre;
        u[1] = h(1, 0);
        for (int k = 0; k + 1 < m; ++k) {
            const double beta = householder(u, 2, v);
            if (beta != 0.0) reflect(m, H, ldh, Qacc, k, 2, v, beta, k > 0 ? k - 1 : 0, std::min(k + 2, m - 1));
            if (k > 0) h(k + 1, k - 1) = 0.0;
            if (k + 2 < m) {
                u[0] = h(k + 1, k);
                u[1] = h(k + 2, k);
            }
        }
        return;
    }
    const double sh = 2.0 * mre, t = mre * mre + mim * mim;
    u[0] = h(0, 0) * h(0, 0) + h(0, 1) * h(1, 0) - sh * h(0, 0) + t;
    u[1] = h(1, 0) * (h(0, 0) + h(1, 1) - sh);
    u[2] = h(1, 0) * h(2, 1);
    for (int k = 0; k + 2 < m; ++k) {
        const double beta = householder(u, 3, v);
        if (beta != 0.0) reflect(m, H, ldh, Qacc, k, 3, v, beta, k > 0 ? k - 1 : 0, std::min(k + 3, m - 1));
        if (k > 0) h(k + 1, k - 1) = h(k + 2, k - 1) = 0.0;
        u[0] = h(k + 1, k);
        u[1] = h(k + 2, k);
        if (k + 3 < m) u[2] = h(k + 3, k);
    }
    const int k = m - 2;
    const double beta = householder(u, 2, v);
    if (beta != 0.0) reflect(m, H, ldh, Qacc, k, 2, v, beta, k - 1, m - 1);
    h(k + 1, k - 1) = 0.0;
}

// Residual estimate of the Ritz pair for theta: |h_{m,m-1}| |x_{m-1}| / ||x||
// with x the eigenvector of the m x m Hessenberg H for theta, by two steps of
// inverse iteration (complex LU with partial pivoting of H - theta' I,
// theta' = theta slightly perturbed so that the matrix is not singular).
// H - theta' I is upper Hessenberg: below the diagonal of column k only row
// k + 1 is nonzero, so the pivot is chosen between rows k and k + 1, the
// elimination touches row k + 1 only and L is unit lower bidiagonal: O(m^2)
// per value.
double ritz_residual(int m, const double* H, int ldh, double hlast, double tre, double tim) {
    const cd th(tre, tim);
    const double pert = 1e-10 * std::max(1.0, std::abs(th));
    const cd shift = th + cd(pert, pert);
    std::vector<cd> A((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = cd(H[(size_t)i * ldh + j], 0.0) - (i == j ? shift : cd(0.0));
    std::vector<int> piv(m);
    std::vector<cd> lsub(m, cd(0.0));   // the multiplier of column k (row k + 1)
    for (int k = 0; k < m; ++k) {
        int p = k;
        if (k + 1 < m && std::abs(A[(size_t)(k + 1) * m + k]) > std::abs(A[(size_t)k * m + k])) p = k + 1;
        piv[k] = p;
        if (p != k)
            for (int j = k; j < m; ++j) std::swap(A[(size_t)k * m + j], A[(size_t)p * m + j]);
        cd d = A[(size_t)k * m + k];
        if (d == cd(0.0)) d = A[(size_t)k * m + k] = cd(kEps * pert, 0.0);
        if (k + 1 < m) {
            const cd f = A[(size_t)(k + 1) * m + k] / d;
            lsub[k] = f;
            A[(size_t)(k + 1) * m + k] = cd(0.0);
            for (int j = k + 1; j < m; ++j) A[(size_t)(k + 1) * m + j] -= f * A[(size_t)k * m + j];
        }
    }
    std::vector<cd> x(m, cd(1.0, 0.0));
    for (int it = 0; it < 2; ++it) {
        // forward: apply each row exchange and elimination in the order of the factorisation
        for (int k = 0; k + 1 < m; ++k) {
            std::swap(x[k], x[piv[k]]);
            x[k + 1] -= lsub[k] * x[k];
        }
        for (int i = m - 1; i >= 0; --i) {
            for (int j = i + 1; j < m; ++j) x[i] -= A[(size_t)i * m + j] * x[j];
            x[i] /= A[(size_t)i * m + i];
        }
        double nx = 0.0;
        for (int i = 0; i < m; ++i) nx += std::norm(x[i]);
        nx = std::sqrt(nx);
        if (!(nx > 0.0) || !std::isfinite(nx)) return INFINITY;
        for (int i = 0; i < m; ++i) x[i] /= nx;
    }
    return fabs(hlast) * std::abs(x[m - 1]);
}

}  // namespace dense
}  // namespace rok
