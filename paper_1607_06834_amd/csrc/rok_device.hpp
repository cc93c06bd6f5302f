// Device-side building blocks shared by the librok kernels: kernel parameter
// blocks, the dual-number type used for exact Jacobian-vector products and
// the periodic index helpers.
//
// Floating-point contract: every file is compiled with -ffp-contract=off and
// evaluates each formula in one fixed, left-to-right operation order, so a
// double-precision result is reproducible bit for bit (FP64 division and
// square root are correctly rounded on gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rok {

constexpr int kMaxStages = 8;
constexpr int kMaxM = 64;

// Geometry and physics constants of one problem (host-computed, passed by value).
struct Geom {
    int D;          // 2 or 3
    int n[3];       // cells per direction (n[2] = 1 in 2-D)
    int nvar;       // D + 2
    long ncell;     // n0 * n1 * n2
    long N;         // nvar * ncell
    double invdx[3];  // 1 / dx, rounded once
    double hinv[3];   // 0.5 / dx (central differences)
    double g, gm1;    // gamma, gamma - 1
    double mu, c23mu, kappa;  // mu, (2/3) mu, mu gamma / ((gamma-1) Pr)
    int flux;                 // inviscid flux: 0 Rusanov, 1 Roe
    int suth;                 // Sutherland's law (else constant mu)
    double suth_s, suth_one_s, t_ref, kden;   // S / T_ref, 1 + S / T_ref, T_ref, (gamma - 1) Pr
    const double* metric;     // 2-D curvilinear grid: Sx_e, Sy_e, Sx_n, Sy_n, 1/A (ncell each), else null
    int ogrid;                // the curvilinear grid is an O-grid (wall at j = 0, far field past j = n1 - 1):
    double uinf[4];           //   then metric also holds the wall face vectors, and uinf is the free stream
    double t_wall;            //   and (Navier-Stokes) t_wall the isothermal wall's temperature
};

// Residual-kernel inputs: the stage state Y = y + sum_t cs[t] xs[t]
// (PLAIN), or y + eps v (FD), or the pair (y, v) (TANGENT).
struct ResArgs {
    const double* y;
    const double* v;
    const double* f0;          // FD: f(y)
    const double* eps_dev;     // FD: if non-null, eps is read from here
    double eps;
    int nterm;
    const double* xs[kMaxStages];
    double cs[kMaxStages];
    void* out;
    // optional: skip the launch unless gate_col + 1 >= *gate (gate: a
    // device-side basis size, e.g. M_eff of the Arnoldi process)
    const int* gate;
    int gate_col;
    // Navier-Stokes kernels: assemble the viscous part of f only
    int viscous_only;
    // optional status word: ROK_FLAG_NONPHYSICAL is or-ed in when a staged
    // cell has rho <= 0 or p <= 0, ROK_FLAG_NONFINITE when an output is NaN or Inf
    int* status;
    // optional: do nothing once *stop is set (a finished Arnoldi process: the
    // basis column this product would read was never written)
    const int* stop;
    // optional (products): the direction is (*vscale) v, for a basis column
    // stored before its normalisation (FD: the increment eps (*vscale) is
    // applied to v; tangent: the tangent is v (*vscale))
    const double* vscale;
};

// ---------------------------------------------------------------------------
// Dual numbers (value, tangent): exact forward-mode derivative of f.
// ---------------------------------------------------------------------------
template <typename T>
struct Dual {
    T v, d;
};

template <typename T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
    T q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
// products and quotients with a plain floating-point constant (any nesting depth)
template <typename T, typename R, typename = typename std::enable_if<std::is_floating_point<R>::value>::type>
__device__ __forceinline__ Dual<T> operator*(R a, Dual<T> b) { return {a * b.v, a * b.d}; }
template <typename T, typename R, typename = typename std::enable_if<std::is_floating_point<R>::value>::type>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, R b) { return {a.v * b, a.d * b}; }
template <typename T, typename R, typename = typename std::enable_if<std::is_floating_point<R>::value>::type>
__device__ __forceinline__ Dual<T> operator/(Dual<T> a, R b) { return {a.v / b, a.d / b}; }
template <typename T, typename R, typename = typename std::enable_if<std::is_floating_point<R>::value>::type>
__device__ __forceinline__ Dual<T> operator+(R a, Dual<T> b) { return {a + b.v, b.d}; }
template <typename T, typename R, typename = typename std::enable_if<std::is_floating_point<R>::value>::type>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, R b) { return {a.v + b, a.d}; }
template <typename T, typename R, typename = typename std::enable_if<std::is_floating_point<R>::value>::type>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, R b) { return {a.v - b, a.d}; }

// Scalar traits: value part (for branch decisions), construction, sqrt.
template <typename S> struct Sc;
template <> struct Sc<double> {
    using R = double;
    static __device__ __forceinline__ double val(double x) { return x; }
    static __device__ __forceinline__ double make(double x) { return x; }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
};
template <> struct Sc<float> {
    using R = float;
    static __device__ __forceinline__ float val(float x) { return x; }
    static __device__ __forceinline__ float make(double x) { return (float)x; }
    static __device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
};
template <typename T> struct Sc<Dual<T>> {
    using R = typename Sc<T>::R;
    static __device__ __forceinline__ R val(Dual<T> x) { return Sc<T>::val(x.v); }
    static __device__ __forceinline__ Dual<T> make(double x) { return {Sc<T>::make(x), Sc<T>::make(0.0)}; }
    static __device__ __forceinline__ Dual<T> sqrt_(Dual<T> x) {
        T s = Sc<T>::sqrt_(x.v);
        return {s, x.d / (s + s)};
    }
};

// The FP64 counterpart of a scalar type (double for float, Dual<double> for
// Dual<float>) and rounding from it.
template <typename S> struct Wide { using type = S; };
template <> struct Wide<float> { using type = double; };
template <typename T> struct Wide<Dual<T>> { using type = Dual<typename Wide<T>::type>; };
template <typename S> __device__ __forceinline__ S narrow(typename Wide<S>::type x) {
    if constexpr (std::is_floating_point<S>::value) return (S)x;
    else return S{narrow<decltype(S{}.v)>(x.v), narrow<decltype(S{}.d)>(x.d)};
}

// Streaming load: for the vector sweeps of the Krylov kernels, which read each
// element of vectors far larger than L2 and the last-level cache once per
// sweep.  The non-temporal hint keeps these lines from displacing reusable
// ones and raises the sweep rate (about 6.3 to 7.1 TB/s for a pure read sweep
// of 17 vectors of 84 M doubles).  Not for stencil staging, whose halos hit in L2.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }

// Pairwise halving tree over groups of 256 consecutive threads of a block:
// with x_i the value of lane i of a group, computes s_i <- s_i + s_{i+h} for
// h = 128, 64, ..., 1 (i < h) and returns s_0 in lane 0 of each group (other
// lanes return partial values).  The two cross-wave levels go through LDS
// (`s`, one double per thread), the six in-wave levels through lane
// shuffles; the additions and their order are those of the LDS tree.
__device__ __forceinline__ double tree256(double v, double* s) {
    const int tid = threadIdx.x;
    const int lane = tid & 255;
    s[tid] = v;
    __syncthreads();
    if (lane < 128) {
        v = v + s[tid + 128];
        s[tid] = v;
    }
    __syncthreads();
    if (lane < 64) {
        v = v + s[tid + 64];
#pragma unroll
        for (int h = 32; h > 0; h >>= 1) v = v + __shfl_down(v, h, 64);
    }
    return v;
}

// tree256 for many values of every thread of a 256-thread block at once:
// values v[C0 .. C0 + 16) (those below nact) go through the tree of tree256
// together, the two LDS levels shared by all of them (three block barriers
// per 16 values, the last before `s` is reused), with the same additions in
// the same order for each; thread 0 passes each sum to store(index, sum).
// `s` holds 16 x 256 doubles of LDS.  nact must be the same in every thread.
template <int C0, int N, typename F>
__device__ __forceinline__ void tree256_chunks(const double (&v)[N], int nact, double (*s)[256], F store) {
    if constexpr (C0 < N) {
        if (C0 >= nact) return;
        const int tid = threadIdx.x;
        constexpr int K = (N - C0) < 16 ? (N - C0) : 16;
        double x[K];
#pragma unroll
        for (int c = 0; c < K; ++c) s[c][tid] = v[C0 + c];
        __syncthreads();
        if (tid < 128) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                x[c] = v[C0 + c] + s[c][tid + 128];
                s[c][tid] = x[c];
            }
        }
        __syncthreads();
        if (tid < 64) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                x[c] = x[c] + s[c][tid + 64];
#pragma unroll
                for (int h = 32; h > 0; h >>= 1) x[c] = x[c] + __shfl_down(x[c], h, 64);
            }
        }
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < K; ++c)
                if (C0 + c < nact) store(C0 + c, x[c]);
        }
        __syncthreads();
        tree256_chunks<C0 + 16, N>(v, nact, s, store);
    }
}

// Periodic wrap of an index that may lie anywhere in [-n, 2n) (fast path) or
// beyond (small grids).
__device__ __forceinline__ int wrap(int i, int n) {
    if (i >= 0 && i < n) return i;
    int r = i % n;
    return r < 0 ? r + n : r;
}

}  // namespace rok
