// Finite-volume residual kernels: F = f(Y), the finite-difference product
// (f(y + eps v) - f(y)) / eps and the exact (tangent) product J(y) v.
//
// f is the semi-discrete compressible Euler / Navier-Stokes operator of
// Sec. 3.2, eq. (11) on a periodic Cartesian grid: primitive variables per
// cell, first-order or MUSCL-minmod face states, Rusanov or Roe flux, central
// viscous fluxes (Stokes stress, Fourier conduction), and the assembly
// f_c = sum_d (Fhat_{c-1/2} - Fhat_{c+1/2}) / dx_d.
//
// Design (one workgroup = one tile of cells):
//   1. the tile plus a halo of two cells on every side is loaded once from
//      HBM (coalesced along x, structure-of-arrays), converted to primitive
//      variables and staged in LDS;
//   2. for each direction every face flux of the tile is computed exactly
//      once from LDS and stored in an LDS face buffer;
//   3. each thread assembles the flux differences of its cells in registers
//      and writes them out once.
// The same code is instantiated with a dual-number scalar for the exact
// Jacobian-vector product and with float for the FP32 form.  The FP32
// instantiations stage primitive perturbations about a reference state (the
// tile's centre cell, taken in FP64) and use the reference-state flux, so
// the large constant part of pressure and energy never enters FP32 sums.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"
#include "rok_flux.hpp"

#include <algorithm>

namespace rok {

enum { MODE_PLAIN = 0, MODE_FD = 1, MODE_TAN = 2 };

// Conserved state of one cell of the stage input.
template <int MODE, int NV, typename S>
__device__ __forceinline__ void load_state(const ResArgs& A, long ncell, long gi, double eps, S* U, double vs = 1.0) {
    using R = typename Sc<S>::R;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        long k = (long)m * ncell + gi;
        if constexpr (MODE == MODE_PLAIN) {
            double acc = A.y[k];
            for (int t = 0; t < A.nterm; ++t) acc = acc + A.cs[t] * A.xs[t][k];
            U[m] = Sc<S>::make(acc);
        } else if constexpr (MODE == MODE_FD) {
            U[m] = Sc<S>::make(A.y[k] + eps * A.v[k]);
        } else {
            U[m] = S{(R)A.y[k], (R)(A.vscale ? A.v[k] * vs : A.v[k])};
        }
    }
}

// Tile shapes.  Box = tile + HW halo cells on each side: 2 for MUSCL (the
// reconstruction reaches two cells past a face), 1 for first order (the face
// and, for viscous terms, the tangential neighbours).
template <int D, int TX, int TY, int TZ, int HW>
struct Tile {
    static constexpr int H = HW;
    static constexpr int TZe = (D == 3) ? TZ : 1;
    static constexpr int BX = TX + 2 * HW, BY = TY + 2 * HW, BZ = (D == 3) ? TZ + 2 * HW : 1;
    static constexpr int BOX = BX * BY * BZ;
    static constexpr int CELLS = TX * TY * TZe;
    static constexpr int NF0 = (TX + 1) * TY * TZe;
    static constexpr int NF1 = TX * (TY + 1) * TZe;
    static constexpr int NF2 = (D == 3) ? TX * TY * (TZ + 1) : 0;
    static constexpr int NFMAX = NF0 > NF1 ? (NF0 > NF2 ? NF0 : NF2) : (NF1 > NF2 ? NF1 : NF2);
    static constexpr int stride(int d) { return d == 0 ? 1 : (d == 1 ? BX : BX * BY); }
};

constexpr int kThreads = 256;
constexpr int kBandY = 4;   // 3-D tile order: rows of tiles along y per band

// The box cells a tile reads: up to HW cells past the tile along one axis
// (the reconstruction stencil of a face), and, for the viscous terms, one
// cell past along two axes (the tangential neighbours of a face's two
// cells).  In 3-D the rest of the box, its far edges and corners, is never
// read: only the listed cells are staged (928 of the 1280 cells of a
// 16x4x4 MUSCL tile with viscous terms).  2-D tiles stage the whole box.
template <int D, int TX, int TY, int TZ, int HW, bool NSV>
struct Stage {
    using T = Tile<D, TX, TY, TZ, HW>;
    static constexpr int out(int b, int t) { return b < HW ? HW - b : (b >= t + HW ? b - t - HW + 1 : 0); }
    static constexpr bool read(int c) {
        const int o0 = out(c % T::BX, TX), o1 = out((c / T::BX) % T::BY, TY);
        const int o2 = (D == 3) ? out(c / (T::BX * T::BY), TZ) : 0;
        const int n = (o0 > 0) + (o1 > 0) + (o2 > 0);
        return n <= 1 || (NSV && n == 2 && o0 <= 1 && o1 <= 1 && o2 <= 1);
    }
    static constexpr bool LIST = (D == 3);
    static constexpr int count() {
        int k = 0;
        for (int c = 0; c < T::BOX; ++c) k += (!LIST || read(c)) ? 1 : 0;
        return k;
    }
    static constexpr int N = count();
    struct Cells { unsigned short c[N]; };
    static constexpr Cells make() {
        Cells a{};
        int k = 0;
        for (int c = 0; c < T::BOX; ++c)
            if (!LIST || read(c)) a.c[k++] = (unsigned short)c;
        return a;
    }
};
template <int D, int TX, int TY, int TZ, int HW, bool NSV>
__device__ constexpr typename Stage<D, TX, TY, TZ, HW, NSV>::Cells kStageCells = Stage<D, TX, TY, TZ, HW, NSV>::make();

// 1 / r (one division; the dual number's tangent by the chain rule)
__device__ __forceinline__ double recip(double r) { return 1.0 / r; }
__device__ __forceinline__ Dual<double> recip(Dual<double> r) {
    const double iv = 1.0 / r.v;
    return {iv, -(r.d * iv) * iv};
}

// XCD-aware block order: workgroups are dispatched round-robin over the 8
// XCDs; give each XCD a contiguous range of tiles so halos hit in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <int D, int RECON, bool NSV, int FLUX, int GEO, typename S, int MODE, typename OUT, int TX, int TY, int TZ>
__global__ __launch_bounds__(kThreads) void k_residual(Geom G, ResArgs A, int nt0, int nt1) {
    using T = Tile<D, TX, TY, TZ, (RECON == 0 ? 1 : 2)>;
    using R = typename Sc<S>::R;
    constexpr int NV = D + 2;
    constexpr bool FO = (RECON == 0);
    constexpr bool PERT = sizeof(R) == 4;              // FP32: reference-state form
    constexpr bool CONS = FO && !PERT;                 // conserved states staged as well
    constexpr int OFF_VEL = CONS ? NV : 1;
    constexpr int OFF_P = OFF_VEL + D;
    constexpr int OFF_T = OFF_P + 1;
    constexpr int CPT = T::CELLS / kThreads;
    static_assert(T::CELLS % kThreads == 0, "tile must be a multiple of the block size");
    using ST = Stage<D, TX, TY, TZ, T::H, NSV>;
    const auto& cells = kStageCells<D, TX, TY, TZ, T::H, NSV>;
    // 3-D: only the box cells the stencil reads are staged, packed in the order
    // of the staging list (s_slot maps a box cell to its slot), which keeps the
    // LDS of a block small enough for three blocks per CU
    constexpr bool PACKED = ST::LIST;
    // the temperature p / rho is staged, except in packed (3-D) boxes: there it
    // is formed where a face needs it, in FP64 as the same division of the same
    // staged values (the same bits), in the FP32 form as the perturbation
    // T - T0 = (r0 p' - p0 rho') / (r0 (r0 + rho')) of the staged perturbations.
    // The FP32 form keeps staging it in 2-D, where LDS allows: the two
    // products nearly cancel for near-isentropic perturbations, which costs
    // about half a bit (a transonic 2-D Roe state: 2.9e-6 against 2.0e-6)
    constexpr bool TSTAGED = NSV && !PACKED;
    constexpr int NP = OFF_P + 1 + (TSTAGED ? 1 : 0);
    constexpr int NSLOT = PACKED ? ST::N : T::BOX;
    constexpr int kFaceUnroll = (D == 2 && sizeof(S) == 8 && !PERT && FLUX == 0) ? 2 : 1;

    __shared__ S sq[NP][NSLOT];
    __shared__ S fb[NV][T::NFMAX];
    __shared__ unsigned short s_slot[PACKED ? T::BOX : 1];
    // FP32 form: the tile's reference state (float, and as doubles)
    __shared__ RefState<D, R> s_ref;
    __shared__ double s_refd[D + 3];   // r0, u0[D], p0, T0 = p0 / r0
    // staged slot of box cell c (every cell the stencil reads is staged)
    auto slot = [&](int c) -> int {
        if constexpr (PACKED) return (int)s_slot[c];
        else return c;
    };
    // temperature of the cell in slot q
    auto temp = [&](int q) -> S {
        if constexpr (TSTAGED) {
            return sq[OFF_T][q];
        } else if constexpr (PERT) {
            const S rp = sq[0][q], pp = sq[OFF_P][q];
            return (s_ref.r0 * pp - s_ref.p0 * rp) / (s_ref.r0 * (s_ref.r0 + rp));
        } else {
            return sq[OFF_P][q] / sq[0][q];
        }
    };

    if (A.gate && A.gate_col + 1 < *A.gate) return;
    if (A.stop && *A.stop) return;
    const int tid = threadIdx.x;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int x0, y0, z0;
    if (D == 3 && nt1 % kBandY == 0) {
        // bands of kBandY tile rows along y, z running inside a band: the tiles
        // above and below a tile (its z halo) are read about nt0 * kBandY tiles
        // apart, within an XCD's L2, instead of a whole tile layer apart
        const int nt2 = gridDim.x / (nt0 * nt1);
        int r = b / nt0;
        x0 = (b % nt0) * TX;
        const int ty = r % kBandY;
        r /= kBandY;
        z0 = (r % nt2) * TZ;
        y0 = ((r / nt2) * kBandY + ty) * TY;
    } else {
        x0 = (b % nt0) * TX;
        y0 = ((b / nt0) % nt1) * TY;
        z0 = (D == 3) ? (b / (nt0 * nt1)) * TZ : 0;
    }
    const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];

    double eps = 0.0;
    if constexpr (MODE == MODE_FD) eps = A.eps_dev ? *A.eps_dev : A.eps;
    // a stored (not yet normalised) basis column: direction vs v
    double vs = 1.0;
    if constexpr (MODE != MODE_PLAIN) {
        if (A.vscale) vs = *A.vscale;
    }
    const double eps_st = (MODE == MODE_FD && A.vscale) ? eps * vs : eps;   // increment applied to v

    // FP32: reference state = the primitive state of the box's centre cell,
    // rounded to float; the same float values (as doubles) are subtracted in
    // FP64 below, so q0 + q' is consistent.
    if constexpr (PERT) {
        if (tid == 0) {
            const int gx = wrap(x0 - T::H + T::BX / 2, n0);
            const int gy = wrap(y0 - T::H + T::BY / 2, n1);
            const int gz = (D == 3) ? wrap(z0 - T::H + T::BZ / 2, n2) : 0;
            const long gi = ((long)gz * n1 + gy) * n0 + gx;
            double U[NV];
            load_state<MODE_PLAIN, NV, double>(MODE == MODE_PLAIN ? A : ResArgs{A.y}, G.ncell, gi, 0.0, U);
            const double r0 = U[0];
            double ke = 0.0, u0[D];
#pragma unroll
            for (int e = 0; e < D; ++e) {
                u0[e] = U[1 + e] / r0;
                ke = ke + u0[e] * u0[e];
            }
            const double p0 = G.gm1 * (U[D + 1] - (0.5 * r0) * ke);
            const R r0f = (R)r0, p0f = (R)p0;
            s_ref.r0 = r0f;
            s_ref.p0 = p0f;
            s_refd[0] = (double)r0f;
            s_refd[D + 1] = (double)p0f;
            s_refd[D + 2] = (double)p0f / (double)r0f;
            double keff = 0.0;
#pragma unroll
            for (int e = 0; e < D; ++e) {
                const R uf = (R)u0[e];
                s_ref.u0[e] = uf;
                s_ref.m0[e] = r0f * uf;
                s_refd[1 + e] = (double)uf;
                keff = keff + (double)uf * (double)uf;
            }
            s_ref.H0 = (R)(G.g * (double)p0f / G.gm1 + 0.5 * (double)r0f * keff);
        }
        __syncthreads();
    }

    // 1. stage the box in LDS as primitive variables.  All loads of this
    // thread's box cells are issued first, then converted: the loads overlap
    // instead of waiting one cell at a time.  `np` records a staged cell with
    // rho <= 0 or p <= 0 (no positivity fix: the arithmetic goes on).
    int np = 0;
    if constexpr (!PERT) {
        constexpr int NIT = (ST::N + kThreads - 1) / kThreads;
        S Ub[NIT][NV];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = tid + it * kThreads;
            if (it + 1 < NIT || i < ST::N) {
                const int c = ST::LIST ? (int)cells.c[i] : i;
                int bx = c % T::BX;
                int by = (c / T::BX) % T::BY;
                int bz = c / (T::BX * T::BY);
                int gx = wrap(x0 - T::H + bx, n0);
                int gy = wrap(y0 - T::H + by, n1);
                int gz = (D == 3) ? wrap(z0 - T::H + bz, n2) : 0;
                long gi = ((long)gz * n1 + gy) * n0 + gx;
                load_state<MODE, NV, S>(A, G.ncell, gi, eps_st, Ub[it], vs);
            }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = tid + it * kThreads;
            if (it + 1 < NIT || i < ST::N) {
                const int c = ST::LIST ? (int)cells.c[i] : i;
                const int q = PACKED ? i : c;
                if constexpr (PACKED) s_slot[c] = (unsigned short)i;
                S* U = Ub[it];
                const R gm1 = (R)G.gm1;
                const R half = (R)0.5;
                S r = U[0];
                S vel[D];
#pragma unroll
                for (int d = 0; d < D; ++d) vel[d] = U[1 + d] / r;
                S ke = vel[0] * vel[0];
#pragma unroll
                for (int d = 1; d < D; ++d) ke = ke + vel[d] * vel[d];
                S p = gm1 * (U[D + 1] - (half * r) * ke);
                np |= (Sc<S>::val(r) <= (R)0 || Sc<S>::val(p) <= (R)0) ? 1 : 0;
                if constexpr (CONS) {
#pragma unroll
                    for (int m = 0; m < NV; ++m) sq[m][q] = U[m];
                } else {
                    sq[0][q] = r;
                }
#pragma unroll
                for (int d = 0; d < D; ++d) sq[OFF_VEL + d][q] = vel[d];
                sq[OFF_P][q] = p;
                if constexpr (TSTAGED) sq[OFF_T][q] = p / r;
            }
        }
        __syncthreads();
    } else {
        // FP32 reference-state form: the state is converted in FP64 (one
        // reciprocal of the density) and the perturbation about the tile's
        // reference state is rounded to float
        for (int i = tid; i < ST::N; i += kThreads) {
            const int c = ST::LIST ? (int)cells.c[i] : i;
            const int q = PACKED ? i : c;
            if constexpr (PACKED) s_slot[c] = (unsigned short)i;
            int bx = c % T::BX;
            int by = (c / T::BX) % T::BY;
            int bz = c / (T::BX * T::BY);
            int gx = wrap(x0 - T::H + bx, n0);
            int gy = wrap(y0 - T::H + by, n1);
            int gz = (D == 3) ? wrap(z0 - T::H + bz, n2) : 0;
            long gi = ((long)gz * n1 + gy) * n0 + gx;
            using SD = typename Wide<S>::type;
            SD U[NV];
            load_state<MODE, NV, SD>(A, G.ncell, gi, eps_st, U, vs);
            const SD r = U[0];
            const SD inv = recip(r);
            SD vel[D];
#pragma unroll
            for (int d = 0; d < D; ++d) vel[d] = U[1 + d] * inv;
            SD ke = vel[0] * vel[0];
#pragma unroll
            for (int d = 1; d < D; ++d) ke = ke + vel[d] * vel[d];
            SD p = G.gm1 * (U[D + 1] - (0.5 * r) * ke);
            np |= (Sc<SD>::val(r) <= 0.0 || Sc<SD>::val(p) <= 0.0) ? 1 : 0;
            sq[0][q] = narrow<S>(r - s_refd[0]);
#pragma unroll
            for (int d = 0; d < D; ++d) sq[1 + d][q] = narrow<S>(vel[d] - s_refd[1 + d]);
            sq[OFF_P][q] = narrow<S>(p - s_refd[D + 1]);
            if constexpr (TSTAGED) sq[OFF_T][q] = narrow<S>(p * inv - s_refd[D + 2]);
        }
        __syncthreads();
    }

    // FD: the loads of f(y) at this thread's output cells are issued here and
    // complete behind the face loops; they are needed only at the write-out
    double f0pre[CPT][NV];
    if constexpr (MODE == MODE_FD) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int cell = tid + k * kThreads;
            const int gx = x0 + cell % TX, gy = y0 + (cell / TX) % TY, gz = z0 + cell / (TX * TY);
            const bool in = gx < n0 && gy < n1 && (D != 3 || gz < n2);
            const long gi = in ? ((long)gz * n1 + gy) * n0 + gx : 0;
#pragma unroll
            for (int m = 0; m < NV; ++m) f0pre[k][m] = in ? A.f0[(long)m * G.ncell + gi] : 0.0;
        }
    }

    S res[CPT][NV];

#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int FX = TX + (d == 0), FY = TY + (d == 1);
        const int NF = (d == 0) ? T::NF0 : (d == 1 ? T::NF1 : T::NF2);
        const int sd = T::stride(d);
        // 2. every face flux of the tile along d, once (plain FP64: two faces
        // interleaved per thread, which hides the latency of their long chains
        // of divisions and square roots)
#pragma unroll(kFaceUnroll)
        for (int f = tid; f < NF; f += kThreads) {
            int fx = f % FX;
            int fy = (f / FX) % FY;
            int fz = f / (FX * FY);
            int cb = ((fz + ((D == 3) ? T::H : 0)) * T::BY + (fy + T::H)) * T::BX + (fx + T::H);
            int ca = cb - sd;
            const int ia = slot(ca), ib = slot(cb);   // staged slots of the face's two cells
            S Fh[NV];
            S UL[NV], UR[NV], vL[D], vR[D];
            S rL, rR, pL, pR;
            if constexpr (PERT) {
                S qL[NV], qR[NV];
                if constexpr (FO) {
#pragma unroll
                    for (int k = 0; k < NV; ++k) { qL[k] = sq[k][ia]; qR[k] = sq[k][ib]; }
                } else {
                    const R half = (R)0.5;
                    const int im = slot(ca - sd), ip = slot(cb + sd);
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        S am1 = sq[k][im], a0 = sq[k][ia], ap1 = sq[k][ib], ap2 = sq[k][ip];
                        qL[k] = a0 + half * minmod(a0 - am1, ap1 - a0);
                        qR[k] = ap1 - half * minmod(ap1 - a0, ap2 - ap1);
                    }
                }
                num_flux_ref<D, FLUX>(G, s_ref, d, qL, qR, Fh);
            } else if constexpr (FO) {
#pragma unroll
                for (int m = 0; m < NV; ++m) { UL[m] = sq[m][ia]; UR[m] = sq[m][ib]; }
                rL = UL[0];
                rR = UR[0];
#pragma unroll
                for (int e = 0; e < D; ++e) { vL[e] = sq[OFF_VEL + e][ia]; vR[e] = sq[OFF_VEL + e][ib]; }
                pL = sq[OFF_P][ia];
                pR = sq[OFF_P][ib];
            } else {
                const R half = (R)0.5;
                S qL[NV], qR[NV];
                // O-grid: no slope across the wall (row 0) or the far field (row n1 - 1)
                bool flatL = false, flatR = false;
                if constexpr (GEO == 2) {
                    if (d == 1) {
                        flatL = (y0 + fy - 1 == 0);
                        flatR = (y0 + fy == n1 - 1);
                    }
                }
                const int im = slot(ca - sd), ip = slot(cb + sd);
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    S am1 = sq[k][im], a0 = sq[k][ia], ap1 = sq[k][ib], ap2 = sq[k][ip];
                    const S sl = flatL ? Sc<S>::make(0.0) : minmod(a0 - am1, ap1 - a0);
                    const S sr = flatR ? Sc<S>::make(0.0) : minmod(ap1 - a0, ap2 - ap1);
                    qL[k] = a0 + half * sl;
                    qR[k] = ap1 - half * sr;
                }
                rL = qL[0];
                rR = qR[0];
#pragma unroll
                for (int e = 0; e < D; ++e) { vL[e] = qL[1 + e]; vR[e] = qR[1 + e]; }
                pL = qL[D + 1];
                pR = qR[D + 1];
                to_conserved<D>(G, rL, vL, pL, UL);
                to_conserved<D>(G, rR, vR, pR, UR);
            }
            int bface = 0;   // O-grid faces along j: 1 wall, 2 far field, 3 outside the grid
            if constexpr (GEO == 2) {
                if (d == 1) {
                    const int gy = y0 + fy;
                    bface = gy == 0 ? 1 : (gy == n1 ? 2 : (gy > n1 ? 3 : 0));
                }
            }
            if constexpr (GEO == 2) {
                if (bface == 2) {
                    // far field: the last cell's primitive state against the free stream
                    rL = sq[0][ca];
#pragma unroll
                    for (int e = 0; e < D; ++e) vL[e] = sq[OFF_VEL + e][ca];
                    pL = sq[OFF_P][ca];
                    to_conserved<D>(G, rL, vL, pL, UL);
#pragma unroll
                    for (int m = 0; m < NV; ++m) UR[m] = Sc<S>::make(G.uinf[m]);
                    primitives<D>(G, UR, rR, vR, pR);
                }
            }
            if constexpr (GEO >= 1) {
                // curvilinear: the flux in the face frame n = S / |S|, rotated back, times |S|
                const int ga = wrap(y0 + fy - (d == 1), n1) * n0 + wrap(x0 + fx - (d == 0), n0);
                const double sx = G.metric[(long)(2 * d) * G.ncell + ga];
                const double sy = G.metric[(long)(2 * d + 1) * G.ncell + ga];
                const double ln = sqrt(sx * sx + sy * sy);
                const double nx = sx / ln, ny = sy / ln;
                S vLr[D], vRr[D], ULr[NV], URr[NV], Fr[NV];
                vLr[0] = vL[0] * nx + vL[1] * ny;
                vLr[1] = vL[1] * nx - vL[0] * ny;
                vRr[0] = vR[0] * nx + vR[1] * ny;
                vRr[1] = vR[1] * nx - vR[0] * ny;
                ULr[0] = UL[0];
                ULr[1] = UL[1] * nx + UL[2] * ny;
                ULr[2] = UL[2] * nx - UL[1] * ny;
                ULr[3] = UL[3];
                URr[0] = UR[0];
                URr[1] = UR[1] * nx + UR[2] * ny;
                URr[2] = UR[2] * nx - UR[1] * ny;
                URr[3] = UR[3];
                num_flux<D, FLUX>(G, 0, ULr, rL, vLr, pL, URr, rR, vRr, pR, Fr);
                Fh[0] = Fr[0] * ln;
                Fh[1] = (Fr[1] * nx - Fr[2] * ny) * ln;
                Fh[2] = (Fr[1] * ny + Fr[2] * nx) * ln;
                Fh[3] = Fr[3] * ln;
                if constexpr (GEO == 2) {
                    if (bface == 1) {
                        // slip wall: the pressure of the first cell on the wall face vector
                        const int gi = wrap(x0 + fx, n0);
                        const double wx = G.metric[9L * G.ncell + gi], wy = G.metric[9L * G.ncell + n0 + gi];
                        const S pw = sq[OFF_P][cb];
                        Fh[0] = Sc<S>::make(0.0);
                        Fh[1] = pw * wx;
                        Fh[2] = pw * wy;
                        Fh[3] = Sc<S>::make(0.0);
                    } else if (bface == 3) {
#pragma unroll
                        for (int m = 0; m < NV; ++m) Fh[m] = Sc<S>::make(0.0);
                    }
                }
            } else if constexpr (!PERT) {
                num_flux<D, FLUX>(G, d, UL, rL, vL, pL, UR, rR, vR, pR, Fh);
            }
            if constexpr (NSV && GEO >= 1) {
                if (A.viscous_only) {
#pragma unroll
                    for (int m = 0; m < NV; ++m) Fh[m] = Sc<S>::make(0.0);
                }
                if (bface != 2 && bface != 3) {   // no viscous flux through the far field
                    const R half = (R)0.5;
                    const int gy = y0 + fy;
                    const int ga = wrap(gy - (d == 1), n1) * n0 + wrap(x0 + fx - (d == 0), n0);
                    const S zero = Sc<S>::make(0.0);
                    double sx, sy, dcx, dcy;
                    S nu, nv, nT, tu, tv, tT, ufx, ufy, Tf;
                    if (bface == 1) {
                        // isothermal no-slip wall: velocity 0 and temperature t_wall on the wall
                        const int gi = wrap(x0 + fx, n0);
                        sx = G.metric[9L * G.ncell + gi];
                        sy = G.metric[9L * G.ncell + n0 + gi];
                        dcx = G.metric[9L * G.ncell + 2 * n0 + gi];
                        dcy = G.metric[9L * G.ncell + 3 * n0 + gi];
                        nu = sq[OFF_VEL][cb] - 0.0;
                        nv = sq[OFF_VEL + 1][cb] - 0.0;
                        nT = sq[OFF_T][cb] - G.t_wall;
                        tu = tv = tT = zero;
                        ufx = ufy = zero;
                        Tf = half * (sq[OFF_T][cb] + G.t_wall);
                    } else {
                        sx = G.metric[(long)(2 * d) * G.ncell + ga];
                        sy = G.metric[(long)(2 * d + 1) * G.ncell + ga];
                        dcx = G.metric[(long)(5 + 2 * d) * G.ncell + ga];
                        dcy = G.metric[(long)(6 + 2 * d) * G.ncell + ga];
                        nu = sq[OFF_VEL][cb] - sq[OFF_VEL][ca];
                        nv = sq[OFF_VEL + 1][cb] - sq[OFF_VEL + 1][ca];
                        nT = sq[OFF_T][cb] - sq[OFF_T][ca];
                        // index-space central differences along the face of both cells, averaged
                        // (O-grid rows next to the wall or the far field: one-sided)
                        const int st = T::stride(1 - d);
                        int side = 0;
                        if constexpr (GEO == 2) {
                            if (d == 0) side = (gy == 0) ? 1 : (gy == n1 - 1 ? 2 : 0);
                        }
                        auto gc = [&](int k, int c) -> S {
                            if (side == 1) return sq[k][c + st] - sq[k][c];
                            if (side == 2) return sq[k][c] - sq[k][c - st];
                            return (sq[k][c + st] - sq[k][c - st]) * half;
                        };
                        tu = half * (gc(OFF_VEL, ca) + gc(OFF_VEL, cb));
                        tv = half * (gc(OFF_VEL + 1, ca) + gc(OFF_VEL + 1, cb));
                        tT = half * (gc(OFF_T, ca) + gc(OFF_T, cb));
                        ufx = half * (sq[OFF_VEL][ca] + sq[OFF_VEL][cb]);
                        ufy = half * (sq[OFF_VEL + 1][ca] + sq[OFF_VEL + 1][cb]);
                        Tf = half * (sq[OFF_T][ca] + sq[OFF_T][cb]);
                    }
                    // chain rule through the face's two grid directions
                    const double J = dcx * sx + dcy * sy;
                    S ux, uy, vx, vy, Tx, Ty;
                    if (d == 0) {
                        ux = (nu * sx - tu * dcy) / J;
                        uy = (nu * sy + tu * dcx) / J;
                        vx = (nv * sx - tv * dcy) / J;
                        vy = (nv * sy + tv * dcx) / J;
                        Tx = (nT * sx - tT * dcy) / J;
                        Ty = (nT * sy + tT * dcx) / J;
                    } else {
                        ux = (nu * sx + tu * dcy) / J;
                        uy = (nu * sy - tu * dcx) / J;
                        vx = (nv * sx + tv * dcy) / J;
                        vy = (nv * sy - tv * dcx) / J;
                        Tx = (nT * sx + tT * dcy) / J;
                        Ty = (nT * sy - tT * dcx) / J;
                    }
                    auto vflux = [&](auto mu_, auto c23_, auto kap_) {
                        const S div = ux + vy;
                        const S txx = mu_ * (ux + ux) - c23_ * div;
                        const S tyy = mu_ * (vy + vy) - c23_ * div;
                        const S txy = mu_ * (uy + vx);
                        const S fx = txx * sx + txy * sy;
                        const S fy = txy * sx + tyy * sy;
                        const S en = (ufx * txx + ufy * txy + kap_ * Tx) * sx + (ufx * txy + ufy * tyy + kap_ * Ty) * sy;
                        Fh[1] = Fh[1] - fx;
                        Fh[2] = Fh[2] - fy;
                        Fh[3] = Fh[3] - en;
                    };
                    if (G.suth) {
                        const S th = Tf / (R)G.t_ref;
                        const S muf = (R)G.mu * th * Sc<S>::sqrt_(th) * (R)G.suth_one_s / (th + (R)G.suth_s);
                        vflux(muf, (R)(2.0 / 3.0) * muf, muf * (R)G.g / (R)G.kden);
                    } else {
                        vflux((R)G.mu, (R)G.c23mu, (R)G.kappa);
                    }
                }
            }
            if constexpr (NSV && GEO == 0) {
                if (A.viscous_only) {
#pragma unroll
                    for (int m = 0; m < NV; ++m) Fh[m] = Sc<S>::make(0.0);
                }
                const R half = (R)0.5;
                const R mu = (R)G.mu, c23mu = (R)G.c23mu, kappa = (R)G.kappa;
                // staged slots of the tangential neighbours of both cells, per direction
                int tap[D], tam[D], tbp[D], tbm[D];
#pragma unroll
                for (int bb = 0; bb < D; ++bb) {
                    if (bb != d) {
                        const int st = T::stride(bb);
                        tap[bb] = slot(ca + st);
                        tam[bb] = slot(ca - st);
                        tbp[bb] = slot(cb + st);
                        tbm[bb] = slot(cb - st);
                    }
                }
                S Gr[D][D];
#pragma unroll
                for (int a = 0; a < D; ++a) {
#pragma unroll
                    for (int bb = 0; bb < D; ++bb) {
                        if (bb == d) {
                            Gr[a][bb] = (sq[OFF_VEL + a][ib] - sq[OFF_VEL + a][ia]) * (R)G.invdx[d];
                        } else {
                            const R h = (R)G.hinv[bb];
                            S gca = (sq[OFF_VEL + a][tap[bb]] - sq[OFF_VEL + a][tam[bb]]) * h;
                            S gcb = (sq[OFF_VEL + a][tbp[bb]] - sq[OFF_VEL + a][tbm[bb]]) * h;
                            Gr[a][bb] = half * (gca + gcb);
                        }
                    }
                }
                S div = Gr[0][0];
#pragma unroll
                for (int a = 1; a < D; ++a) div = div + Gr[a][a];
                // stress, work and conduction for viscosity mu_, (2/3) mu_ and conductivity kappa_
                auto viscous = [&](auto mu_, auto c23mu_, auto kappa_) {
                    S work;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        S tau = (a == d) ? mu_ * (Gr[a][d] + Gr[d][a]) - c23mu_ * div : mu_ * (Gr[a][d] + Gr[d][a]);
                        S uf = half * (sq[OFF_VEL + a][ia] + sq[OFF_VEL + a][ib]);
                        if constexpr (PERT) uf = s_ref.u0[a] + uf;   // perturbations staged: add the reference
                        work = (a == 0) ? uf * tau : work + uf * tau;
                        Fh[1 + a] = Fh[1 + a] - tau;
                    }
                    S dTdn = (temp(ib) - temp(ia)) * (R)G.invdx[d];
                    Fh[D + 1] = Fh[D + 1] - (work + kappa_ * dTdn);
                };
                if (G.suth) {
                    // Sutherland's law at the face temperature (T_a + T_b) / 2
                    S Tf = half * (temp(ia) + temp(ib));
                    if constexpr (PERT) Tf = (R)s_refd[D + 2] + Tf;
                    const S th = Tf / (R)G.t_ref;
                    const S muf = mu * th * Sc<S>::sqrt_(th) * (R)G.suth_one_s / (th + (R)G.suth_s);
                    viscous(muf, (R)(2.0 / 3.0) * muf, muf * (R)G.g / (R)G.kden);
                } else {
                    viscous(mu, c23mu, kappa);
                }
            }
#pragma unroll
            for (int m = 0; m < NV; ++m) fb[m][f] = Fh[m];
        }
        __syncthreads();
        // 3. flux differences of this thread's cells
        const int fs = (d == 0) ? 1 : (d == 1 ? FX : FX * FY);
        const R inv = (R)G.invdx[d];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            int cell = tid + k * kThreads;
            int cx = cell % TX;
            int cy = (cell / TX) % TY;
            int cz = cell / (TX * TY);
            int fl = (cz * FY + cy) * FX + cx;
            R icell = inv;
            if constexpr (GEO >= 1) icell = G.metric[4L * G.ncell + wrap(y0 + cy, n1) * n0 + wrap(x0 + cx, n0)];
#pragma unroll
            for (int m = 0; m < NV; ++m) {
                S term = (fb[m][fl] - fb[m][fl + fs]) * icell;
                res[k][m] = (d == 0) ? term : res[k][m] + term;
            }
        }
        __syncthreads();
    }

    // 4. write out (and note a NaN or Inf in the output)
    bool nonfin = false;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        int cell = tid + k * kThreads;
        int gx = x0 + cell % TX;
        int gy = y0 + (cell / TX) % TY;
        int gz = z0 + cell / (TX * TY);
        if (gx >= n0 || gy >= n1 || (D == 3 && gz >= n2)) continue;
        long gi = ((long)gz * n1 + gy) * n0 + gx;
        OUT* out = (OUT*)A.out;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            long o = (long)m * G.ncell + gi;
            OUT x;
            if constexpr (MODE == MODE_PLAIN) {
                x = (OUT)res[k][m];
            } else if constexpr (MODE == MODE_FD) {
                x = (OUT)((res[k][m] - f0pre[k][m]) / eps);
            } else {
                x = (OUT)res[k][m].d;
            }
            out[o] = x;
            nonfin = nonfin || !(fabs((double)x) < __builtin_inf());
        }
    }
    // rare: only a thread that saw a non-physical cell or a non-finite output touches the status word
    if (A.status && (np || nonfin))
        atomicOr(A.status, (np ? (int)ROK_FLAG_NONPHYSICAL : 0) | (nonfin ? (int)ROK_FLAG_NONFINITE : 0));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// 3-D MUSCL residual and FD product, FP64, Cartesian grid: column-marching form.
// A block owns a 16 x 16 column of cells over a range of planes and walks up
// z.  Three staged planes (z - 1, z, z + 1: primitive variables over the
// 20 x 20 halo'd region) sit in LDS; the block's own cells of plane z + 2 come
// straight from HBM into registers (the z face's reconstruction needs them
// one plane early) and are staged from there one plane later, with the 144
// halo cells, so every cell is loaded once per range.  Each thread computes
// the x face and the y face on the low side of its cell and the z face above
// it, and exchanges fluxes with its neighbours by lane shuffles; the faces on
// the column's +x and +y edges are computed by two waves and passed through a
// small LDS buffer.  LDS per block stays under a third of the CU's, so three
// blocks (12 waves) share a CU.  Every face flux and every cell sum is the
// same sequence of operations on the same values as in k_residual (the same
// bits).
// ---------------------------------------------------------------------------
constexpr int kZW = 20;              // staged plane width (16 + 2 + 2)
constexpr int kZR = kZW * kZW;       // cells of a staged plane
constexpr int kZHalo = kZR - 256;    // its halo cells
constexpr int kZBlocks = 1536;       // two rounds of three resident blocks on each of 256 CUs

struct ZRef {
    int s, c;   // LDS slot, index in the staged plane
};

// primitive variables (rho, u, v, w, p) of a conserved state, in the staging
// order of k_residual; returns whether rho <= 0 or p <= 0
__device__ __forceinline__ bool zprim(const Geom& G, const double* U, double* q) {
    const double gm1 = G.gm1;
    const double half = 0.5;
    const double r = U[0];
    double vel[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) vel[e] = U[1 + e] / r;
    double ke = vel[0] * vel[0];
#pragma unroll
    for (int e = 1; e < 3; ++e) ke = ke + vel[e] * vel[e];
    const double p = gm1 * (U[4] - (half * r) * ke);
    q[0] = r;
#pragma unroll
    for (int e = 0; e < 3; ++e) q[1 + e] = vel[e];
    q[4] = p;
    return r <= 0.0 || p <= 0.0;
}

// The flux through one face along d between cells a and b = a + e_d:
// MUSCL-minmod reconstruction from the primitive states (qm, qa, qb, qp) of
// the cells a - e_d, a, b, b + e_d, the inviscid flux and, with NSV, the
// central viscous flux with the tangential derivatives from the neighbours
// ta / tb (+/- along each direction bb != d, read from the staged planes).
template <int d, bool NSV, int FLUX>
__device__ __forceinline__ void zface(const Geom& G, int viscous_only, const double (*ring)[5][kZR],
                                      const double (&qm)[5], const double (&qa)[5], const double (&qb)[5],
                                      const double (&qp)[5], const ZRef (&tap)[3], const ZRef (&tam)[3],
                                      const ZRef (&tbp)[3], const ZRef (&tbm)[3], double* Fh) {
    auto V = [&](ZRef r, int k) -> double { return ring[r.s][k][r.c]; };
    const double half = 0.5;
    double qL[5], qR[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double am1 = qm[k], a0 = qa[k], ap1 = qb[k], ap2 = qp[k];
        const double sl = minmod(a0 - am1, ap1 - a0);
        const double sr = minmod(ap1 - a0, ap2 - ap1);
        qL[k] = a0 + half * sl;
        qR[k] = ap1 - half * sr;
    }
    double UL[5], UR[5], vL[3], vR[3];
    const double rL = qL[0], rR = qR[0];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        vL[e] = qL[1 + e];
        vR[e] = qR[1 + e];
    }
    const double pL = qL[4], pR = qR[4];
    to_conserved<3>(G, rL, vL, pL, UL);
    to_conserved<3>(G, rR, vR, pR, UR);
    num_flux<3, FLUX>(G, d, UL, rL, vL, pL, UR, rR, vR, pR, Fh);
    if constexpr (NSV) {
        if (viscous_only) {
#pragma unroll
            for (int m = 0; m < 5; ++m) Fh[m] = 0.0;
        }
        const double mu = G.mu, c23mu = G.c23mu, kappa = G.kappa;
        double Gr[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                if (bb == d) {
                    Gr[a][bb] = (qb[1 + a] - qa[1 + a]) * G.invdx[d];
                } else {
                    const double h = G.hinv[bb];
                    double gca = (V(tap[bb], 1 + a) - V(tam[bb], 1 + a)) * h;
                    double gcb = (V(tbp[bb], 1 + a) - V(tbm[bb], 1 + a)) * h;
                    Gr[a][bb] = half * (gca + gcb);
                }
            }
        }
        double div = Gr[0][0];
#pragma unroll
        for (int a = 1; a < 3; ++a) div = div + Gr[a][a];
        const double Ta = qa[4] / qa[0], Tb = qb[4] / qb[0];
        auto viscous = [&](double mu_, double c23mu_, double kappa_) {
            double work;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double tau = (a == d) ? mu_ * (Gr[a][d] + Gr[d][a]) - c23mu_ * div : mu_ * (Gr[a][d] + Gr[d][a]);
                double uf = half * (qa[1 + a] + qb[1 + a]);
                work = (a == 0) ? uf * tau : work + uf * tau;
                Fh[1 + a] = Fh[1 + a] - tau;
            }
            double dTdn = (Tb - Ta) * G.invdx[d];
            Fh[4] = Fh[4] - (work + kappa_ * dTdn);
        };
        if (G.suth) {
            double Tf = half * (Ta + Tb);
            const double th = Tf / G.t_ref;
            const double muf = mu * th * sqrt(th) * G.suth_one_s / (th + G.suth_s);
            viscous(muf, (2.0 / 3.0) * muf, muf * G.g / G.kden);
        } else {
            viscous(mu, c23mu, kappa);
        }
    }
}

// index in the staged plane of halo cell h (0 <= h < kZHalo): rows 0, 1, 18,
// 19 whole, then columns 0, 1, 18, 19 of rows 2 .. 17
__device__ __forceinline__ int zhalo(int h) {
    if (h < 2 * kZW) return h;
    if (h < 4 * kZW) return 16 * kZW + h;
    const int k = h - 4 * kZW, c = k & 3;
    return (2 + (k >> 2)) * kZW + (c < 2 ? c : c + 16);
}

template <bool NSV, int FLUX, int MODE>
__global__ __launch_bounds__(kThreads, (NSV && FLUX == 1) ? 2 : 3) void k_res3z(Geom G, ResArgs A, int nbx, int nby, int nch) {
    __shared__ double ring[3][5][kZR];
    __shared__ double fedge_x[5][16];      // x faces on the column's +x edge, by row
    __shared__ double frow_y[5][5][16];    // y faces below rows 0, 4, 8, 12 and above row 15
    if (A.gate && A.gate_col + 1 < *A.gate) return;
    if (A.stop && *A.stop) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4, wv = tid >> 6, lane = tid & 63;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int ncol = nbx * nby, col = b % ncol, ch = b / ncol;
    const int x0 = (col % nbx) * 16, y0 = (col / nbx) * 16;
    const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
    const int zs = (int)((long)ch * n2 / nch), ze = (int)((long)(ch + 1) * n2 / nch);
    double eps = 0.0;
    if constexpr (MODE == MODE_FD) eps = A.eps_dev ? *A.eps_dev : A.eps;
    double vs = 1.0;
    if constexpr (MODE != MODE_PLAIN) {
        if (A.vscale) vs = *A.vscale;
    }
    const double eps_st = (MODE == MODE_FD && A.vscale) ? eps * vs : eps;
    int np = 0;
    const int c0 = (ty + 2) * kZW + (tx + 2);          // this thread's cell in a staged plane
    const int hc = tid < kZHalo ? zhalo(tid) : c0;      // the halo cell it stages
    auto gidx = [&](int z, int c) -> long {
        const int gx = wrap(x0 - 2 + c % kZW, n0), gy = wrap(y0 - 2 + c / kZW, n1);
        return ((long)wrap(z, n2) * n1 + gy) * n0 + gx;
    };
    auto load_prim = [&](int z, int c, double* q) {
        double U[5];
        load_state<MODE, 5, double>(A, G.ncell, gidx(z, c), eps_st, U, vs);
        np |= zprim(G, U, q) ? 1 : 0;
    };
    auto stage_halo = [&](int z, int s) {
        if (tid < kZHalo) {
            double q[5];
            load_prim(z, hc, q);
#pragma unroll
            for (int k = 0; k < 5; ++k) ring[s][k][hc] = q[k];
        }
    };
    int sA = 0, sB = 1, sC = 2;   // slots of planes z - 1, z, z + 1
    {
        double q[5];
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
            load_prim(zs - 1 + i, c0, q);
#pragma unroll
            for (int k = 0; k < 5; ++k) ring[i][k][c0] = q[k];
            stage_halo(zs - 1 + i, i);
        }
    }
    double Fdown[5];   // flux through the z face below this thread's cell
    {
        double qm[5], qa[5], qb[5], qp[5];
        load_prim(zs - 2, c0, qm);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            qa[k] = ring[0][k][c0];
            qb[k] = ring[1][k][c0];
            qp[k] = ring[2][k][c0];
        }
        ZRef tap[3], tam[3], tbp[3], tbm[3];
        tap[0] = {0, c0 + 1};   tam[0] = {0, c0 - 1};   tbp[0] = {1, c0 + 1};   tbm[0] = {1, c0 - 1};
        tap[1] = {0, c0 + kZW}; tam[1] = {0, c0 - kZW}; tbp[1] = {1, c0 + kZW}; tbm[1] = {1, c0 - kZW};
        tap[2] = tam[2] = tbp[2] = tbm[2] = {0, c0};
        zface<2, NSV, FLUX>(G, A.viscous_only, ring, qm, qa, qb, qp, tap, tam, tbp, tbm, Fdown);
    }
    const long gxy = (long)(y0 + ty) * n0 + (x0 + tx);
    bool nonfin = false;
    double* out = (double*)A.out;
#pragma unroll 1
    for (int z = zs; z < ze; ++z) {
        const long go = (long)z * n0 * n1 + gxy;
        double rx[5], ry[5];
        // x face on the -x side of the cell; the +x side's from the next lane of the row
        {
            const int ca = c0 - 1, cb = c0;
            double qm[5], qa[5], qb[5], qp[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                qm[k] = ring[sB][k][ca - 1];
                qa[k] = ring[sB][k][ca];
                qb[k] = ring[sB][k][cb];
                qp[k] = ring[sB][k][cb + 1];
            }
            ZRef tap[3], tam[3], tbp[3], tbm[3];
            tap[0] = tam[0] = tbp[0] = tbm[0] = {sB, ca};
            tap[1] = {sB, ca + kZW}; tam[1] = {sB, ca - kZW}; tbp[1] = {sB, cb + kZW}; tbm[1] = {sB, cb - kZW};
            tap[2] = {sC, ca};       tam[2] = {sA, ca};       tbp[2] = {sC, cb};       tbm[2] = {sA, cb};
            double F[5];
            zface<0, NSV, FLUX>(G, A.viscous_only, ring, qm, qa, qb, qp, tap, tam, tbp, tbm, F);
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const double nb = __shfl_down(F[m], 1, 16);
                rx[m] = (tx < 15) ? (F[m] - nb) * G.invdx[0] : F[m];
            }
        }
        // y face on the -y side; the +y side's from the lane 16 up, or (last row of a wave) through LDS
        {
            const int ca = c0 - kZW, cb = c0;
            double qm[5], qa[5], qb[5], qp[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                qm[k] = ring[sB][k][ca - kZW];
                qa[k] = ring[sB][k][ca];
                qb[k] = ring[sB][k][cb];
                qp[k] = ring[sB][k][cb + kZW];
            }
            ZRef tap[3], tam[3], tbp[3], tbm[3];
            tap[0] = {sB, ca + 1}; tam[0] = {sB, ca - 1}; tbp[0] = {sB, cb + 1}; tbm[0] = {sB, cb - 1};
            tap[1] = tam[1] = tbp[1] = tbm[1] = {sB, ca};
            tap[2] = {sC, ca};     tam[2] = {sA, ca};     tbp[2] = {sC, cb};     tbm[2] = {sA, cb};
            double F[5];
            zface<1, NSV, FLUX>(G, A.viscous_only, ring, qm, qa, qb, qp, tap, tam, tbp, tbm, F);
            if ((ty & 3) == 0) {
#pragma unroll
                for (int m = 0; m < 5; ++m) frow_y[ty >> 2][m][tx] = F[m];
            }
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const double nb = __shfl_down(F[m], 16, 64);
                ry[m] = ((ty & 3) != 3) ? (F[m] - nb) * G.invdx[1] : F[m];
            }
        }
        // the column's edge faces: two waves (alternating by plane), 16 lanes each
        const int we = (z & 1) * 2;
        if (wv == we && lane < 16) {
            const int cb = (lane + 2) * kZW + 18, ca = cb - 1;
            double qm[5], qa[5], qb[5], qp[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                qm[k] = ring[sB][k][ca - 1];
                qa[k] = ring[sB][k][ca];
                qb[k] = ring[sB][k][cb];
                qp[k] = ring[sB][k][cb + 1];
            }
            ZRef tap[3], tam[3], tbp[3], tbm[3];
            tap[0] = tam[0] = tbp[0] = tbm[0] = {sB, ca};
            tap[1] = {sB, ca + kZW}; tam[1] = {sB, ca - kZW}; tbp[1] = {sB, cb + kZW}; tbm[1] = {sB, cb - kZW};
            tap[2] = {sC, ca};       tam[2] = {sA, ca};       tbp[2] = {sC, cb};       tbm[2] = {sA, cb};
            double F[5];
            zface<0, NSV, FLUX>(G, A.viscous_only, ring, qm, qa, qb, qp, tap, tam, tbp, tbm, F);
#pragma unroll
            for (int m = 0; m < 5; ++m) fedge_x[m][lane] = F[m];
        } else if (wv == we + 1 && lane < 16) {
            const int cb = 18 * kZW + lane + 2, ca = cb - kZW;
            double qm[5], qa[5], qb[5], qp[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                qm[k] = ring[sB][k][ca - kZW];
                qa[k] = ring[sB][k][ca];
                qb[k] = ring[sB][k][cb];
                qp[k] = ring[sB][k][cb + kZW];
            }
            ZRef tap[3], tam[3], tbp[3], tbm[3];
            tap[0] = {sB, ca + 1}; tam[0] = {sB, ca - 1}; tbp[0] = {sB, cb + 1}; tbm[0] = {sB, cb - 1};
            tap[1] = tam[1] = tbp[1] = tbm[1] = {sB, ca};
            tap[2] = {sC, ca};     tam[2] = {sA, ca};     tbp[2] = {sC, cb};     tbm[2] = {sA, cb};
            double F[5];
            zface<1, NSV, FLUX>(G, A.viscous_only, ring, qm, qa, qb, qp, tap, tam, tbp, tbm, F);
#pragma unroll
            for (int m = 0; m < 5; ++m) frow_y[4][m][lane] = F[m];
        }
        // z face above the cell (planes z - 1 .. z + 2 of this column)
        double q2[5], Fup[5];
        {
            load_prim(z + 2, c0, q2);
            double qm[5], qa[5], qb[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                qm[k] = ring[sA][k][c0];
                qa[k] = ring[sB][k][c0];
                qb[k] = ring[sC][k][c0];
            }
            ZRef tap[3], tam[3], tbp[3], tbm[3];
            tap[0] = {sB, c0 + 1};   tam[0] = {sB, c0 - 1};   tbp[0] = {sC, c0 + 1};   tbm[0] = {sC, c0 - 1};
            tap[1] = {sB, c0 + kZW}; tam[1] = {sB, c0 - kZW}; tbp[1] = {sC, c0 + kZW}; tbm[1] = {sC, c0 - kZW};
            tap[2] = tam[2] = tbp[2] = tbm[2] = {sB, c0};
            zface<2, NSV, FLUX>(G, A.viscous_only, ring, qm, qa, qb, q2, tap, tam, tbp, tbm, Fup);
        }
        __syncthreads();   // edge faces written; plane z - 1 no longer read
        double f0v[5];
        if constexpr (MODE == MODE_FD) {
#pragma unroll
            for (int m = 0; m < 5; ++m) f0v[m] = A.f0[(long)m * G.ncell + go];
        }
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            if (tx == 15) rx[m] = (rx[m] - fedge_x[m][ty]) * G.invdx[0];
            if ((ty & 3) == 3) ry[m] = (ry[m] - frow_y[(ty + 1) >> 2][m][tx]) * G.invdx[1];
            double res = rx[m];
            res = res + ry[m];
            res = res + (Fdown[m] - Fup[m]) * G.invdx[2];
            Fdown[m] = Fup[m];
            double x;
            if constexpr (MODE == MODE_FD) x = (res - f0v[m]) / eps;
            else x = res;
            out[(long)m * G.ncell + go] = x;
            nonfin = nonfin || !(fabs(x) < __builtin_inf());
        }
        // plane z + 2 replaces plane z - 1
#pragma unroll
        for (int k = 0; k < 5; ++k) ring[sA][k][c0] = q2[k];
        stage_halo(z + 2, sA);
        __syncthreads();   // plane z + 2 staged; the edge faces read
        const int t = sA;
        sA = sB;
        sB = sC;
        sC = t;
    }
    if (A.status && (np || nonfin))
        atomicOr(A.status, (np ? (int)ROK_FLAG_NONPHYSICAL : 0) | (nonfin ? (int)ROK_FLAG_NONFINITE : 0));
}

template <int D, int RECON, bool NSV, int FLUX, int GEO, typename S, int MODE, typename OUT, int TX, int TY, int TZ>
static hipError_t launch_t(const Geom& G, const ResArgs& A, hipStream_t st) {
    int nt0 = (G.n[0] + TX - 1) / TX;
    int nt1 = (G.n[1] + TY - 1) / TY;
    int nt2 = (D == 3) ? (G.n[2] + TZ - 1) / TZ : 1;
    long nb = (long)nt0 * nt1 * nt2;
    if (nb <= 0 || nb > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_residual<D, RECON, NSV, FLUX, GEO, S, MODE, OUT, TX, TY, TZ>), dim3((unsigned)nb), dim3(kThreads), 0, st,
                       G, A, nt0, nt1);
    return hipGetLastError();
}

// Tile shape per variant: bigger tiles where the LDS footprint allows.
template <int D, int RECON, bool NSV, int FLUX, int GEO, typename S, int MODE, typename OUT>
static hipError_t launch_v(const Geom& G, const ResArgs& A, hipStream_t st) {
    constexpr bool wide = sizeof(S) <= 8;   // double or float (not a dual number)
    if constexpr (D == 2) {
        if constexpr (RECON == 1 && sizeof(S) == 8 && sizeof(typename Sc<S>::R) == 8)
            return launch_t<D, RECON, NSV, FLUX, GEO, S, MODE, OUT, 16, 16, 1>(G, A, st);   // FP64 (measured best)
        else if constexpr (RECON == 1 && wide) return launch_t<D, RECON, NSV, FLUX, GEO, S, MODE, OUT, 32, 16, 1>(G, A, st);
        else return launch_t<D, RECON, NSV, FLUX, GEO, S, MODE, OUT, 32, 8, 1>(G, A, st);
    } else {
        if constexpr (RECON == 1 && GEO == 0 && std::is_same<S, double>::value && std::is_same<OUT, double>::value &&
                      MODE != MODE_TAN) {
            if (G.n[0] % 16 == 0 && G.n[1] % 16 == 0) {
                // columns of 16 x 16 cells, each cut into nch ranges of planes: enough
                // blocks to fill the chip once, ranges of at least 8 planes
                const int nbx = G.n[0] / 16, nby = G.n[1] / 16;
                const long ncol = (long)nbx * nby;
                long nch = (kZBlocks + ncol - 1) / ncol;
                nch = std::min<long>(nch, std::max(1, G.n[2] / 8));
                const long nb = ncol * nch;
                if (nb <= 0 || nb > 0x7fffffffL) return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_res3z<NSV, FLUX, MODE>), dim3((unsigned)nb), dim3(kThreads), 0, st, G, A, nbx,
                                   nby, (int)nch);
                return hipGetLastError();
            }
        }
        return launch_t<D, RECON, NSV, FLUX, GEO, S, MODE, OUT, 16, 4, 4>(G, A, st);
    }
}

template <int D, int RECON, bool NSV, int FLUX, int GEO>
static hipError_t dispatch_prec(const Geom& G, const ResArgs& A, int kind, bool fp32, bool out_double, hipStream_t st) {
    if (!fp32) {
        if (kind == MODE_PLAIN) return launch_v<D, RECON, NSV, FLUX, GEO, double, MODE_PLAIN, double>(G, A, st);
        if (kind == MODE_FD) return launch_v<D, RECON, NSV, FLUX, GEO, double, MODE_FD, double>(G, A, st);
        return launch_v<D, RECON, NSV, FLUX, GEO, Dual<double>, MODE_TAN, double>(G, A, st);
    }
    if (kind == MODE_FD) return hipErrorNotSupported;
    if (kind == MODE_PLAIN) {
        if (out_double) return launch_v<D, RECON, NSV, FLUX, GEO, float, MODE_PLAIN, double>(G, A, st);
        return launch_v<D, RECON, NSV, FLUX, GEO, float, MODE_PLAIN, float>(G, A, st);
    }
    if (out_double) return launch_v<D, RECON, NSV, FLUX, GEO, Dual<float>, MODE_TAN, double>(G, A, st);
    return launch_v<D, RECON, NSV, FLUX, GEO, Dual<float>, MODE_TAN, float>(G, A, st);
}

// Metrics of a 2-D curvilinear periodic grid from its nodes (x, y indexed
// j * nx + i; node (i + nx, j) is node (i, j) + (Lx, 0), node (i, j + ny) is
// node (i, j) + (0, Ly)): for cell (i, j) with nodes p0 = (i, j), p1 = (i+1, j),
// p2 = (i+1, j+1), p3 = (i, j+1), the east face vector (y2 - y1, x1 - x2), the
// north face vector (y3 - y2, x2 - x3), 1 / A with
// A = ((x2 - x0)(y3 - y1) - (x3 - x1)(y2 - y0)) / 2, and the centroid
// differences across the east and north faces; nine arrays of ncell.
__global__ __launch_bounds__(256) void k_metrics(const double* xn, const double* yn, int nx, int ny, double Lx,
                                                 double Ly, double* out) {
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    const long ncell = (long)nx * ny;
    if (c >= ncell) return;
    const int i = (int)(c % nx), j = (int)(c / nx);
    const bool ei = (i + 1 == nx), ej = (j + 1 == ny);
    const int i1 = ei ? 0 : i + 1, j1 = ej ? 0 : j + 1;
    const double x0 = xn[c], y0 = yn[c];
    const double x1 = ei ? xn[(long)j * nx + i1] + Lx : xn[(long)j * nx + i1];
    const double y1 = yn[(long)j * nx + i1];
    const double x2 = ei ? xn[(long)j1 * nx + i1] + Lx : xn[(long)j1 * nx + i1];
    const double y2 = ej ? yn[(long)j1 * nx + i1] + Ly : yn[(long)j1 * nx + i1];
    const double x3 = xn[(long)j1 * nx + i];
    const double y3 = ej ? yn[(long)j1 * nx + i] + Ly : yn[(long)j1 * nx + i];
    out[c] = y2 - y1;
    out[ncell + c] = x1 - x2;
    out[2 * ncell + c] = y3 - y2;
    out[3 * ncell + c] = x2 - x3;
    const double area = 0.5 * ((x2 - x0) * (y3 - y1) - (x3 - x1) * (y2 - y0));
    out[4 * ncell + c] = 1.0 / area;
    // centroid differences across the east and north faces: nodes (i+2, j), (i+2, j+1), (i, j+2), (i+1, j+2)
    const bool e2 = (i + 2 >= nx), f2 = (j + 2 >= ny);
    const int i2 = e2 ? i + 2 - nx : i + 2, j2 = f2 ? j + 2 - ny : j + 2;
    const double x4 = e2 ? xn[(long)j * nx + i2] + Lx : xn[(long)j * nx + i2];
    const double y4 = yn[(long)j * nx + i2];
    const double x5 = e2 ? xn[(long)j1 * nx + i2] + Lx : xn[(long)j1 * nx + i2];
    const double y5 = ej ? yn[(long)j1 * nx + i2] + Ly : yn[(long)j1 * nx + i2];
    const double x6 = xn[(long)j2 * nx + i];
    const double y6 = f2 ? yn[(long)j2 * nx + i] + Ly : yn[(long)j2 * nx + i];
    const double x7 = ei ? xn[(long)j2 * nx + i1] + Lx : xn[(long)j2 * nx + i1];
    const double y7 = f2 ? yn[(long)j2 * nx + i1] + Ly : yn[(long)j2 * nx + i1];
    out[5 * ncell + c] = 0.25 * ((x4 + x5) - (x0 + x3));
    out[6 * ncell + c] = 0.25 * ((y4 + y5) - (y0 + y3));
    out[7 * ncell + c] = 0.25 * ((x6 + x7) - (x0 + x1));
    out[8 * ncell + c] = 0.25 * ((y6 + y7) - (y0 + y1));
}

// Metrics of an O-grid: nodes (x, y) indexed j * nx + i for j = 0..ny (row 0 on
// the wall, row ny on the far-field boundary), i periodic without offset; the
// same nine per-cell arrays as k_metrics (the last row's north centroid
// difference is 0: that face is the far field), then the wall face vectors
// (y(i, 0) - y(i+1, 0), x(i+1, 0) - x(i, 0)) and the vectors from each wall
// face's midpoint to the first cell's centroid, as four arrays of nx.
__global__ __launch_bounds__(256) void k_metrics_ogrid(const double* xn, const double* yn, int nx, int ny,
                                                       double* out) {
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    const long ncell = (long)nx * ny;
    if (c >= ncell) return;
    const int i = (int)(c % nx), j = (int)(c / nx);
    const int i1 = (i + 1 == nx) ? 0 : i + 1;
    const double x0 = xn[(long)j * nx + i], y0 = yn[(long)j * nx + i];
    const double x1 = xn[(long)j * nx + i1], y1 = yn[(long)j * nx + i1];
    const double x2 = xn[(long)(j + 1) * nx + i1], y2 = yn[(long)(j + 1) * nx + i1];
    const double x3 = xn[(long)(j + 1) * nx + i], y3 = yn[(long)(j + 1) * nx + i];
    out[c] = y2 - y1;
    out[ncell + c] = x1 - x2;
    out[2 * ncell + c] = y3 - y2;
    out[3 * ncell + c] = x2 - x3;
    const double area = 0.5 * ((x2 - x0) * (y3 - y1) - (x3 - x1) * (y2 - y0));
    out[4 * ncell + c] = 1.0 / area;
    const int i2 = (i + 2 >= nx) ? i + 2 - nx : i + 2;
    out[5 * ncell + c] = 0.25 * ((xn[(long)j * nx + i2] + xn[(long)(j + 1) * nx + i2]) - (x0 + x3));
    out[6 * ncell + c] = 0.25 * ((yn[(long)j * nx + i2] + yn[(long)(j + 1) * nx + i2]) - (y0 + y3));
    if (j + 2 <= ny) {
        out[7 * ncell + c] = 0.25 * ((xn[(long)(j + 2) * nx + i] + xn[(long)(j + 2) * nx + i1]) - (x0 + x1));
        out[8 * ncell + c] = 0.25 * ((yn[(long)(j + 2) * nx + i] + yn[(long)(j + 2) * nx + i1]) - (y0 + y1));
    } else {
        out[7 * ncell + c] = 0.0;   // the far-field face
        out[8 * ncell + c] = 0.0;
    }
    if (j == 0) {
        out[9 * ncell + i] = y0 - y1;
        out[9 * ncell + nx + i] = x1 - x0;
        out[9 * ncell + 2 * nx + i] = 0.25 * ((x2 + x3) - (x0 + x1));
        out[9 * ncell + 3 * nx + i] = 0.25 * ((y2 + y3) - (y0 + y1));
    }
}

hipError_t launch_metrics_ogrid(const double* xn, const double* yn, int nx, int ny, double* out, hipStream_t st) {
    const long n = (long)nx * ny;
    hipLaunchKernelGGL(k_metrics_ogrid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xn, yn, nx, ny, out);
    return hipGetLastError();
}

hipError_t launch_metrics(const double* xn, const double* yn, int nx, int ny, double Lx, double Ly, double* out,
                          hipStream_t st) {
    const long n = (long)nx * ny;
    hipLaunchKernelGGL(k_metrics, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xn, yn, nx, ny, Lx, Ly, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero(unsigned* p, long n) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_zero(void* p, long bytes, hipStream_t st) {
    const long n = bytes / 4;
    if (n <= 0) return hipSuccess;
    long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)nb), dim3(256), 0, st, (unsigned*)p, n);
    return hipGetLastError();
}

// Curvilinear grids: 2-D Euler physics in FP64 (value, FD and tangent kernels).
template <int RECON, bool NSV, int FLUX, int GEO>
static hipError_t dispatch_curv(const Geom& G, const ResArgs& A, int kind, hipStream_t st) {
    if (kind == MODE_PLAIN) return launch_v<2, RECON, NSV, FLUX, GEO, double, MODE_PLAIN, double>(G, A, st);
    if (kind == MODE_FD) return launch_v<2, RECON, NSV, FLUX, GEO, double, MODE_FD, double>(G, A, st);
    return launch_v<2, RECON, NSV, FLUX, GEO, Dual<double>, MODE_TAN, double>(G, A, st);
}

template <int D, int RECON, bool NSV>
static hipError_t dispatch_flux(const Geom& G, const ResArgs& A, int kind, bool fp32, bool out_double, hipStream_t st) {
    if (G.metric) {
        if constexpr (D == 2) {
            if (fp32) return hipErrorNotSupported;
            if (G.ogrid)
                return G.flux == 1 ? dispatch_curv<RECON, NSV, 1, 2>(G, A, kind, st)
                                   : dispatch_curv<RECON, NSV, 0, 2>(G, A, kind, st);
            return G.flux == 1 ? dispatch_curv<RECON, NSV, 1, 1>(G, A, kind, st)
                               : dispatch_curv<RECON, NSV, 0, 1>(G, A, kind, st);
        }
        return hipErrorNotSupported;
    }
    if (G.flux == 1) return dispatch_prec<D, RECON, NSV, 1, 0>(G, A, kind, fp32, out_double, st);
    return dispatch_prec<D, RECON, NSV, 0, 0>(G, A, kind, fp32, out_double, st);
}

hipError_t launch_residual(const Geom& G, int recon, bool ns, bool fp32, int kind, bool out_double,
                           const ResArgs& A, hipStream_t st) {
    if (G.D == 2) {
        if (recon == 0) return ns ? dispatch_flux<2, 0, true>(G, A, kind, fp32, out_double, st)
                                  : dispatch_flux<2, 0, false>(G, A, kind, fp32, out_double, st);
        return ns ? dispatch_flux<2, 1, true>(G, A, kind, fp32, out_double, st)
                  : dispatch_flux<2, 1, false>(G, A, kind, fp32, out_double, st);
    }
    if (recon == 0) return ns ? dispatch_flux<3, 0, true>(G, A, kind, fp32, out_double, st)
                              : dispatch_flux<3, 0, false>(G, A, kind, fp32, out_double, st);
    return ns ? dispatch_flux<3, 1, true>(G, A, kind, fp32, out_double, st)
              : dispatch_flux<3, 1, false>(G, A, kind, fp32, out_double, st);
}

}  // namespace rok
