// Adjoint (transposed) Jacobian products of the finite-volume residual:
//   ybar (+)= J(y)^T wbar                          (first-order adjoint)
//   ybar2 (+)= d/dt [J(y + t v)^T wbar] at t = 0   (second-order adjoint)
// for the right-hand side f of Sec. 3.2, eq. (11) (Euler or Navier-Stokes
// physics, first-order or MUSCL-minmod reconstruction, Rusanov or Roe flux,
// periodic Cartesian or 2-D curvilinear grid; on the latter f_c divides by
// the cell area, each inviscid face flux is the rotated one and the viscous
// one follows the chain rule through the face vector).
//
// f_c = sum_d (Fhat_{c-1/2} - Fhat_{c+1/2}) / dx_d, so the adjoint of the face
// a+1/2 (between cells a and a+1) is Fbar = (wbar_{a+1} - wbar_a) / dx_d, and
// cell c collects Fbar^T dFhat/dU_c from every face whose stencil contains c
// (first order: faces c-1/2, c+1/2; MUSCL: the four faces c-3/2 .. c+3/2).
// Each thread owns one cell and gathers its own contributions, so the result
// is deterministic without atomics; Fbar^T dFhat/dU_c comes from one reverse
// sweep of the face flux (face_flux_vjp, the transpose of the tangent of the
// residual's flux code) for Rusanov's flux, and from one forward-mode
// evaluation per variable of c for Roe's.  With a dual scalar (y + t v) the same kernel returns
// the second-order adjoint in the tangent part.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_flux.hpp"
#include "rok_kernels.hpp"

namespace rok {

// Viscous flux of the Cartesian face between cells a and b = a + e_d
// (Sec. 3.2: stress row and energy term), from the conserved states of its
// stencil: U[0] = a, U[1] = b and, for the k-th direction t != d,
// U[2 + 4k .. 5 + 4k] = a - e_t, a + e_t, b - e_t, b + e_t.  Normal
// derivatives are the difference across the face; tangential ones the mean
// of the central differences in a and b; the viscosity is constant or
// Sutherland's law at the mean temperature of a and b.
template <int D, typename S>
__device__ __forceinline__ void visc_face(const Geom& G, const S (*U)[D + 2], int d, S* Fv) {
    constexpr int NQ = 2 + 4 * (D - 1);
    const double half = 0.5;
    S vel[NQ][D], Tq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        S r, p;
        primitives<D>(G, U[q], r, vel[q], p);
        Tq[q] = p / r;
    }
    S Gr[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int bb = 0; bb < D; ++bb) {
            if (bb == d) {
                Gr[a][bb] = (vel[1][a] - vel[0][a]) * G.invdx[d];
            } else {
                const int k = (bb < d) ? bb : bb - 1;
                const S gca = (vel[3 + 4 * k][a] - vel[2 + 4 * k][a]) * G.hinv[bb];
                const S gcb = (vel[5 + 4 * k][a] - vel[4 + 4 * k][a]) * G.hinv[bb];
                Gr[a][bb] = half * (gca + gcb);
            }
        }
    }
    S div = Gr[0][0];
#pragma unroll
    for (int a = 1; a < D; ++a) div = div + Gr[a][a];
    S mu, c23mu, kappa;
    if (G.suth) {
        const S th = (half * (Tq[0] + Tq[1])) / G.t_ref;
        mu = G.mu * th * Sc<S>::sqrt_(th) * G.suth_one_s / (th + G.suth_s);
        c23mu = (2.0 / 3.0) * mu;
        kappa = mu * G.g / G.kden;
    } else {
        mu = Sc<S>::make(G.mu);
        c23mu = Sc<S>::make(G.c23mu);
        kappa = Sc<S>::make(G.kappa);
    }
    S work;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const S tau = (a == d) ? mu * (Gr[a][d] + Gr[d][a]) - c23mu * div : mu * (Gr[a][d] + Gr[d][a]);
        const S uf = half * (vel[0][a] + vel[1][a]);
        work = (a == 0) ? uf * tau : work + uf * tau;
        Fv[1 + a] = tau;
    }
    Fv[0] = Sc<S>::make(0.0);
    Fv[D + 1] = work + kappa * ((Tq[1] - Tq[0]) * G.invdx[d]);
}

// Viscous flux through a face of a 2-D curvilinear grid (Sec. 3.2), the
// stencil as in visc_face (U[0] = a, U[1] = b, U[2..5] = a - e_t, a + e_t,
// b - e_t, b + e_t with t the grid direction along the face): index-space
// differences across the face and means of the two cells' central
// differences along it, turned into Cartesian gradients by the chain rule
// through the face vector S = (sx, sy) and the centroid difference
// (dcx, dcy) across the face; the stress, work and conduction terms dotted
// with S.
// Viscous flux through a face of a 2-D curvilinear grid (Sec. 3.2) from
// index-space derivatives across the face (nu, nv, nT) and along it (tu, tv,
// tT), turned into Cartesian gradients by the chain rule through the face
// vector S = (sx, sy) and the centroid difference (dcx, dcy) across the face
// (d: 0 across i, 1 across j); the stress, work and conduction terms dotted
// with S.  uf: face velocity; Tf: face temperature (Sutherland's law).
template <typename S>
__device__ __forceinline__ void curv_visc_core(const Geom& G, int d, double sx, double sy, double dcx, double dcy,
                                               S nu, S nv, S nT, S tu, S tv, S tT, S ufx, S ufy, S Tf, S* Fv) {
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
    S mu, c23, kap;
    if (G.suth) {
        const S th = Tf / G.t_ref;
        mu = G.mu * th * Sc<S>::sqrt_(th) * G.suth_one_s / (th + G.suth_s);
        c23 = (2.0 / 3.0) * mu;
        kap = mu * G.g / G.kden;
    } else {
        mu = Sc<S>::make(G.mu);
        c23 = Sc<S>::make(G.c23mu);
        kap = Sc<S>::make(G.kappa);
    }
    const S div = ux + vy;
    const S txx = mu * (ux + ux) - c23 * div;
    const S tyy = mu * (vy + vy) - c23 * div;
    const S txy = mu * (uy + vx);
    Fv[0] = Sc<S>::make(0.0);
    Fv[1] = txx * sx + txy * sy;
    Fv[2] = txy * sx + tyy * sy;
    Fv[3] = (ufx * txx + ufy * txy + kap * Tx) * sx + (ufx * txy + ufy * tyy + kap * Ty) * sy;
}

// The same from the stencil of a periodic curvilinear face (as in visc_face:
// U[0] = a, U[1] = b, U[2..5] = a - e_t, a + e_t, b - e_t, b + e_t with t
// the grid direction along the face): differences across the face and means
// of the two cells' central differences along it.
template <typename S>
__device__ __forceinline__ void curv_visc_face(const Geom& G, const S (*U)[4], int d, double sx, double sy,
                                               double dcx, double dcy, S* Fv) {
    const double half = 0.5;
    S u[6], v[6], Tq[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        S r, vel[2], p;
        primitives<2>(G, U[q], r, vel, p);
        u[q] = vel[0];
        v[q] = vel[1];
        Tq[q] = p / r;
    }
    auto along = [&](const S* f) { return half * ((f[3] - f[2]) * half + (f[5] - f[4]) * half); };
    curv_visc_core<S>(G, d, sx, sy, dcx, dcy, u[1] - u[0], v[1] - v[0], Tq[1] - Tq[0], along(u), along(v),
                      along(Tq), half * (u[0] + u[1]), half * (v[0] + v[1]), half * (Tq[0] + Tq[1]), Fv);
}

template <int FLUX, typename S>
__device__ __forceinline__ void rotated_flux(const Geom& G, const S* UL, S rL, const S* vL, S pL, const S* UR, S rR,
                                             const S* vR, S pR, double sx, double sy, S* Fh);

// Inviscid flux through a face of a 2-D curvilinear grid with face vector
// (sx, sy): the stencil's states reconstructed in index space (first order
// U[0] = a, U[1] = b; MUSCL U[0..3] = a-1, a, b, b+1), rotated into the face
// frame n = S / |S|, the one-dimensional numerical flux there, rotated back
// and scaled by |S|.
template <int RECON, int FLUX, typename S>
__device__ __forceinline__ void curv_face_flux(const Geom& G, const S (*U)[4], double sx, double sy, S* Fh) {
    S UL[4], UR[4], vL[2], vR[2], rL, rR, pL, pR;
    if constexpr (RECON == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            UL[m] = U[0][m];
            UR[m] = U[1][m];
        }
        primitives<2>(G, UL, rL, vL, pL);
        primitives<2>(G, UR, rR, vR, pR);
    } else {
        S q[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            S rr, vv[2], pp;
            primitives<2>(G, U[k], rr, vv, pp);
            q[k][0] = rr;
            q[k][1] = vv[0];
            q[k][2] = vv[1];
            q[k][3] = pp;
        }
        S qL[4], qR[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            qL[m] = q[1][m] + 0.5 * minmod(q[1][m] - q[0][m], q[2][m] - q[1][m]);
            qR[m] = q[2][m] - 0.5 * minmod(q[2][m] - q[1][m], q[3][m] - q[2][m]);
        }
        rL = qL[0];
        rR = qR[0];
        vL[0] = qL[1];
        vL[1] = qL[2];
        vR[0] = qR[1];
        vR[1] = qR[2];
        pL = qL[3];
        pR = qR[3];
        to_conserved<2>(G, rL, vL, pL, UL);
        to_conserved<2>(G, rR, vR, pR, UR);
    }
    rotated_flux<FLUX, S>(G, UL, rL, vL, pL, UR, rR, vR, pR, sx, sy, Fh);
}

// Numerical flux through a face with vector (sx, sy) between reconstructed
// states: rotated into the face frame n = S / |S|, the one-dimensional flux,
// rotated back and scaled by |S|.
template <int FLUX, typename S>
__device__ __forceinline__ void rotated_flux(const Geom& G, const S* UL, S rL, const S* vL, S pL, const S* UR, S rR,
                                             const S* vR, S pR, double sx, double sy, S* Fh) {
    const double ln = sqrt(sx * sx + sy * sy);
    const double nx = sx / ln, ny = sy / ln;
    S vLr[2], vRr[2], ULr[4], URr[4], Fr[4];
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
    num_flux<2, FLUX>(G, 0, ULr, rL, vLr, pL, URr, rR, vRr, pR, Fr);
    Fh[0] = Fr[0] * ln;
    Fh[1] = (Fr[1] * nx - Fr[2] * ny) * ln;
    Fh[2] = (Fr[1] * ny + Fr[2] * nx) * ln;
    Fh[3] = Fr[3] * ln;
}

template <int D, int RECON, bool SECOND, int FLUX, bool NSV, int GEO>
__global__ __launch_bounds__(256) void k_vjp(Geom G, const double* y, const double* v, const double* wbar,
                                            double* ybar, double* ybar2, int accumulate, const int* gate, int col) {
    if (gate && col >= gate[0]) return;   // Krylov column beyond M_eff: nothing to add
    constexpr int NV = D + 2;
    constexpr int NS = (RECON == 0) ? 2 : 4;   // stencil cells of a face
    constexpr int NF = (RECON == 0) ? 2 : 4;   // faces per direction whose stencil contains a cell
    using T = typename std::conditional<SECOND, Dual<double>, double>::type;   // value (+ t-derivative)
    const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
    const long ncell = G.ncell;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += stride) {
        const int cx = (int)(c % n0);
        const int cy = (int)((c / n0) % n1);
        const int cz = (int)(c / ((long)n0 * n1));
        T acc[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = Sc<T>::make(0.0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double inv = G.invdx[d];
#pragma nounroll
            for (int f = 0; f < NF; ++f) {
                // face between cells a and a+1 along d; stencil starts at s0
                const int off_a = (RECON == 0) ? f - 1 : f - 2;      // a - c
                const int off_s0 = (RECON == 0) ? off_a : off_a - 1;  // first stencil cell - c
                const int kc = -off_s0;                               // position of c in the stencil
                long cell[NS];
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    int o = off_s0 + q;
                    int x = cx, yy = cy, z = cz;
                    if (d == 0) x = wrap(cx + o, n0);
                    else if (d == 1) yy = wrap(cy + o, n1);
                    else z = wrap(cz + o, n2);
                    cell[q] = ((long)z * n1 + yy) * n0 + x;
                }
                const long ca = cell[(RECON == 0) ? 0 : 1];
                const long cb = cell[(RECON == 0) ? 1 : 2];
                T fbar[NV];
                if constexpr (GEO == 0) {
#pragma unroll
                    for (int m = 0; m < NV; ++m)
                        fbar[m] = Sc<T>::make((wbar[m * ncell + cb] - wbar[m * ncell + ca]) * inv);
                } else {
                    // f_c = sum_d (Fhat_{c-1/2} - Fhat_{c+1/2}) / A_c
                    const double ia = G.metric[4 * ncell + ca], ib = G.metric[4 * ncell + cb];
#pragma unroll
                    for (int m = 0; m < NV; ++m)
                        fbar[m] = Sc<T>::make(wbar[m * ncell + cb] * ib - wbar[m * ncell + ca] * ia);
                }
                T base[NS][NV], ub[NS][NV];
#pragma unroll
                for (int q = 0; q < NS; ++q)
#pragma unroll
                    for (int m = 0; m < NV; ++m) {
                        const long i = m * ncell + cell[q];
                        if constexpr (SECOND) base[q][m] = T{y[i], v[i]};
                        else base[q][m] = y[i];
                        ub[q][m] = Sc<T>::make(0.0);
                    }
                if constexpr (GEO == 1) {
                    // rotated face flux: Fbar^T dFhat/dU_c by forward mode, one dual direction per variable of c
                    const double sx = G.metric[(long)(2 * d) * ncell + ca];
                    const double sy = G.metric[(long)(2 * d + 1) * ncell + ca];
                    using TT = Dual<T>;
#pragma unroll 1
                    for (int m = 0; m < NV; ++m) {
                        TT Ud[NS][4], Fd[4];
#pragma unroll
                        for (int q = 0; q < NS; ++q)
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                Ud[q][k] = TT{base[q][k], Sc<T>::make((q == kc && k == m) ? 1.0 : 0.0)};
                        curv_face_flux<RECON, FLUX, TT>(G, Ud, sx, sy, Fd);
                        T sum = Sc<T>::make(0.0);
#pragma unroll
                        for (int k = 0; k < 4; ++k) sum = sum + fbar[k] * Fd[k].d;
                        ub[kc][m] = sum;
                    }
                } else if constexpr (FLUX == 0) {
                    face_flux_vjp<D, RECON, T>(G, base, d, fbar, ub);
                } else {
                    // Roe: Fbar^T dFhat/dU_c by forward mode, one dual direction per variable of c
                    using TT = Dual<T>;
#pragma unroll 1
                    for (int m = 0; m < NV; ++m) {
                        TT Ud[NS][NV], Fd[NV];
#pragma unroll
                        for (int q = 0; q < NS; ++q)
#pragma unroll
                            for (int k = 0; k < NV; ++k)
                                Ud[q][k] = TT{base[q][k], Sc<T>::make((q == kc && k == m) ? 1.0 : 0.0)};
                        face_flux_cells<D, RECON, TT, 1>(G, Ud, d, Fd);
                        T sum = Sc<T>::make(0.0);
#pragma unroll
                        for (int k = 0; k < NV; ++k) sum = sum + fbar[k] * Fd[k].d;
                        ub[kc][m] = sum;
                    }
                }
#pragma unroll
                for (int q = 0; q < NS; ++q)
                    if (q == kc)
#pragma unroll
                        for (int k = 0; k < NV; ++k) acc[k] = acc[k] + ub[q][k];
            }
            if constexpr (NSV) {
                // The face flux is Fhat - Fv: cell c collects -Fbar^T dFv/dU_c
                // from every face whose viscous stencil holds it, one face per
                // stencil position (position kv of c), each by forward mode.
                constexpr int NQ = 2 + 4 * (D - 1);
                auto cell_at = [&](int od, int ot, int t) -> long {
                    int o[3] = {0, 0, 0};
                    o[d] += od;
                    if (ot) o[t] += ot;
                    const int x = wrap(cx + o[0], n0), yy = wrap(cy + o[1], n1);
                    const int z = (D == 3) ? wrap(cz + o[2], n2) : 0;
                    return ((long)z * n1 + yy) * n0 + x;
                };
#pragma nounroll
                for (int kv = 0; kv < NQ; ++kv) {
                    // offset of face cell a from c, and of each stencil cell from a
                    int ad = 0, at = 0, tdir = 0;
                    if (kv == 0) ad = 0;
                    else if (kv == 1) ad = -1;
                    else {
                        const int k = (kv - 2) / 4, r = (kv - 2) % 4;
                        tdir = (k < d) ? k : k + 1;
                        ad = (r >= 2) ? -1 : 0;          // c on the b side
                        at = (r % 2 == 0) ? 1 : -1;      // c = a - e_t (r even) or a + e_t
                    }
                    long cell[NQ];
                    cell[0] = cell_at(ad, at, tdir);
                    cell[1] = cell_at(ad + 1, at, tdir);
#pragma unroll
                    for (int k = 0; k < D - 1; ++k) {
                        const int t = (k < d) ? k : k + 1;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int od = ad + (r >= 2 ? 1 : 0);
                            int ot = (r % 2 == 0) ? -1 : 1;
                            // offsets along t add up: (a's offset from c) + (stencil cell's from a)
                            if (t == tdir) cell[2 + 4 * k + r] = cell_at(od, at + ot, t);
                            else {
                                int o3[3] = {0, 0, 0};
                                o3[d] += od;
                                o3[tdir] += at;
                                o3[t] += ot;
                                const int x = wrap(cx + o3[0], n0), yy = wrap(cy + o3[1], n1);
                                const int z = (D == 3) ? wrap(cz + o3[2], n2) : 0;
                                cell[2 + 4 * k + r] = ((long)z * n1 + yy) * n0 + x;
                            }
                        }
                    }
                    T fbar[NV];
                    if constexpr (GEO == 0) {
#pragma unroll
                        for (int m = 0; m < NV; ++m)
                            fbar[m] = Sc<T>::make((wbar[m * ncell + cell[1]] - wbar[m * ncell + cell[0]]) * inv);
                    } else {
                        const double ia = G.metric[4 * ncell + cell[0]], ib = G.metric[4 * ncell + cell[1]];
#pragma unroll
                        for (int m = 0; m < NV; ++m)
                            fbar[m] = Sc<T>::make(wbar[m * ncell + cell[1]] * ib - wbar[m * ncell + cell[0]] * ia);
                    }
                    T base[NQ][NV];
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int m = 0; m < NV; ++m) {
                            const long i = m * ncell + cell[q];
                            if constexpr (SECOND) base[q][m] = T{y[i], v[i]};
                            else base[q][m] = y[i];
                        }
                    using TT = Dual<T>;
#pragma unroll 1
                    for (int m = 0; m < NV; ++m) {
                        TT Ud[NQ][NV], Fd[NV];
#pragma unroll
                        for (int q = 0; q < NQ; ++q)
#pragma unroll
                            for (int k = 0; k < NV; ++k)
                                Ud[q][k] = TT{base[q][k], Sc<T>::make((q == kv && k == m) ? 1.0 : 0.0)};
                        if constexpr (GEO == 0) {
                            visc_face<D, TT>(G, Ud, d, Fd);
                        } else {
                            const long a0 = cell[0];
                            curv_visc_face<TT>(G, Ud, d, G.metric[(long)(2 * d) * ncell + a0],
                                               G.metric[(long)(2 * d + 1) * ncell + a0],
                                               G.metric[(long)(5 + 2 * d) * ncell + a0],
                                               G.metric[(long)(6 + 2 * d) * ncell + a0], Fd);
                        }
                        T sum = Sc<T>::make(0.0);
#pragma unroll
                        for (int k = 1; k < NV; ++k) sum = sum + fbar[k] * Fd[k].d;
                        acc[m] = acc[m] - sum;
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const long o = k * ncell + c;
            if constexpr (SECOND) {
                ybar[o] = accumulate ? ybar[o] + acc[k].v : acc[k].v;
                ybar2[o] = accumulate ? ybar2[o] + acc[k].d : acc[k].d;
            } else {
                ybar[o] = accumulate ? ybar[o] + acc[k] : acc[k];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// O-grid (2-D, periodic in i, wall at j = -1/2, far field at j = ny - 1/2).
// A face's flux Fhat - Fv is evaluated from a 4 x 3 patch of cells P[a][b]:
// i-faces (kind 0) between (i, j) and (i + 1, j): P[a][b] = (i + a - 1, j + b - 1);
// j-faces (kind 1) between (i, j) and (i, j + 1): P[a][b] = (i + b - 1, j + a - 1);
// the wall face below (i, 0) (kind 2) and the far-field face above (i, ny - 1)
// (kind 3) read P[1][1] only.  Rows outside the grid hold a copy of P[1][1]
// and are never read: MUSCL slopes and derivatives along j are one-sided
// (or zero) in the first and last rows, as in the residual.
template <int RECON, int FLUX, bool NSV, typename S>
__device__ __forceinline__ void ogrid_face(const Geom& G, int kind, int j, long fc, const S (*P)[3][4], S* F) {
    const long ncell = G.ncell;
    const int ny = G.n[1], n0 = G.n[0];
    const double half = 0.5;
    if (kind >= 2) {
        S r, vel[2], p;
        primitives<2>(G, P[1][1], r, vel, p);
        if (kind == 2) {
            const int i = (int)(fc % n0);
            const double wx = G.metric[9 * ncell + i], wy = G.metric[9 * ncell + n0 + i];
            F[0] = Sc<S>::make(0.0);
            F[1] = p * wx;
            F[2] = p * wy;
            F[3] = Sc<S>::make(0.0);
            if constexpr (NSV) {
                const S zero = Sc<S>::make(0.0);
                const S T0 = p / r;
                S Fv[4];
                curv_visc_core<S>(G, 1, wx, wy, G.metric[9 * ncell + 2 * n0 + i], G.metric[9 * ncell + 3 * n0 + i],
                                  vel[0] - 0.0, vel[1] - 0.0, T0 - G.t_wall, zero, zero, zero, zero, zero,
                                  half * (T0 + G.t_wall), Fv);
#pragma unroll
                for (int m = 1; m < 4; ++m) F[m] = F[m] - Fv[m];
            }
        } else {
            S Ub[4], Uf[4], rf, vf[2], pf;
            to_conserved<2>(G, r, vel, p, Ub);
#pragma unroll
            for (int m = 0; m < 4; ++m) Uf[m] = Sc<S>::make(G.uinf[m]);
            primitives<2>(G, Uf, rf, vf, pf);
            rotated_flux<FLUX, S>(G, Ub, r, vel, p, Uf, rf, vf, pf, G.metric[2 * ncell + fc], G.metric[3 * ncell + fc],
                                  F);
        }
        return;
    }
    const int d = kind;
    constexpr int A0 = (RECON == 0) ? 1 : 0, A1 = (RECON == 0) ? 2 : 3;   // patch slots the flux reads
    constexpr int B0 = NSV ? 0 : 1, B1 = NSV ? 2 : 1;
    S q[4][3][4];   // primitives (r, u, v, p) of the patch
#pragma unroll
    for (int a = A0; a <= A1; ++a)
#pragma unroll
        for (int b = B0; b <= B1; ++b) {
            S vel[2];
            primitives<2>(G, P[a][b], q[a][b][0], vel, q[a][b][3]);
            q[a][b][1] = vel[0];
            q[a][b][2] = vel[1];
        }
    S UL[4], UR[4], vL[2], vR[2], rL, rR, pL, pR;
    if constexpr (RECON == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            UL[m] = P[1][1][m];
            UR[m] = P[2][1][m];
        }
        rL = q[1][1][0], rR = q[2][1][0], pL = q[1][1][3], pR = q[2][1][3];
        vL[0] = q[1][1][1], vL[1] = q[1][1][2], vR[0] = q[2][1][1], vR[1] = q[2][1][2];
    } else {
        const bool flatL = d == 1 && j == 0, flatR = d == 1 && j + 1 == ny - 1;
        S qL[4], qR[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const S am1 = q[0][1][m], a0 = q[1][1][m], ap1 = q[2][1][m], ap2 = q[3][1][m];
            qL[m] = flatL ? a0 + half * Sc<S>::make(0.0) : a0 + half * minmod(a0 - am1, ap1 - a0);
            qR[m] = flatR ? ap1 - half * Sc<S>::make(0.0) : ap1 - half * minmod(ap1 - a0, ap2 - ap1);
        }
        rL = qL[0], rR = qR[0], pL = qL[3], pR = qR[3];
        vL[0] = qL[1], vL[1] = qL[2], vR[0] = qR[1], vR[1] = qR[2];
        to_conserved<2>(G, rL, vL, pL, UL);
        to_conserved<2>(G, rR, vR, pR, UR);
    }
    rotated_flux<FLUX, S>(G, UL, rL, vL, pL, UR, rR, vR, pR, G.metric[(long)(2 * d) * ncell + fc],
                          G.metric[(long)(2 * d + 1) * ncell + fc], F);
    if constexpr (NSV) {
        // derivatives along the face: central in the periodic i direction; along
        // j one-sided in the first and last rows
        auto T = [&](int a, int b) { return q[a][b][3] / q[a][b][0]; };
        S nf[3], tf[3], uf[2];
        const S Ta = T(1, 1), Tb = T(2, 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            auto val = [&](int a, int b) { return k < 2 ? q[a][b][1 + k] : T(a, b); };
            nf[k] = val(2, 1) - val(1, 1);
            S ga, gb;
            if (d == 1) {
                ga = (val(1, 2) - val(1, 0)) * half;
                gb = (val(2, 2) - val(2, 0)) * half;
            } else if (j == 0) {
                ga = val(1, 2) - val(1, 1);
                gb = val(2, 2) - val(2, 1);
            } else if (j == ny - 1) {
                ga = val(1, 1) - val(1, 0);
                gb = val(2, 1) - val(2, 0);
            } else {
                ga = (val(1, 2) - val(1, 0)) * half;
                gb = (val(2, 2) - val(2, 0)) * half;
            }
            tf[k] = half * (ga + gb);
            if (k < 2) uf[k] = half * (val(1, 1) + val(2, 1));
        }
        S Fv[4];
        curv_visc_core<S>(G, d, G.metric[(long)(2 * d) * ncell + fc], G.metric[(long)(2 * d + 1) * ncell + fc],
                          G.metric[(long)(5 + 2 * d) * ncell + fc], G.metric[(long)(6 + 2 * d) * ncell + fc], nf[0],
                          nf[1], nf[2], tf[0], tf[1], tf[2], uf[0], uf[1], half * (Ta + Tb), Fv);
#pragma unroll
        for (int m = 1; m < 4; ++m) F[m] = F[m] - Fv[m];
    }
}

// Adjoint on an O-grid: cell c gathers Fbar^T d(Fhat - Fv)/dU_c from every
// (face, patch position) pair that places c in the face's patch, each by
// forward mode; Fbar of a face is wbar_b / A_b - wbar_a / A_a (the wall face
// has only b = (i, 0), the far-field face only a = (i, ny - 1)).  One thread
// per (variable m, cell c), c fastest: it seeds the one dual direction U_c[m].
template <int RECON, bool SECOND, int FLUX, bool NSV>
__global__ __launch_bounds__(64) void k_vjp_ogrid(Geom G, const double* y, const double* v, const double* wbar,
                                                  double* ybar, double* ybar2, int accumulate, const int* gate,
                                                  int col) {
    if (gate && col >= gate[0]) return;
    using T = typename std::conditional<SECOND, Dual<double>, double>::type;
    using TT = Dual<T>;
    const int n0 = G.n[0], ny = G.n[1];
    const long ncell = G.ncell;
    const double* ia = G.metric + 4 * ncell;
    constexpr int A0 = (RECON == 0) ? 1 : 0, A1 = (RECON == 0) ? 2 : 3;   // patch rows a the flux reads
    constexpr int B0 = NSV ? 0 : 1, B1 = NSV ? 2 : 1;                     // patch columns b
    const long stride = (long)gridDim.x * blockDim.x;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < 4 * ncell; idx += stride) {
        const int m = (int)(idx / ncell);
        const long c = idx - (long)m * ncell;
        const int cx = (int)(c % n0), cy = (int)(c / n0);
        T acc = Sc<T>::make(0.0);
        auto load = [&](long cell, T* u) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const long o = m * ncell + cell;
                if constexpr (SECOND) u[m] = T{y[o], v[o]};
                else u[m] = y[o];
            }
        };
        // one (face, position) pair: fi, fj the face's cell a (or the wall /
        // far-field cell), (pa, pb) the position of c in its patch
        auto face = [&](int kind, int fi, int fj, int pa, int pb) {
            const long fc = (long)fj * n0 + fi;
            T base[4][3][4];
            if (kind >= 2) {
                load(fc, base[1][1]);
            } else {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        int ii, jj;
                        if (kind == 0) ii = wrap(fi + a - 1, n0), jj = fj + b - 1;
                        else ii = wrap(fi + b - 1, n0), jj = fj + a - 1;
                        if (a < A0 || a > A1 || b < B0 || b > B1 || jj < 0 || jj >= ny) {
                            ii = fi;
                            jj = fj;
                        }
                        load((long)jj * n0 + ii, base[a][b]);
                    }
            }
            T fbar[4];
            if (kind == 2) {
#pragma unroll
                for (int m = 0; m < 4; ++m) fbar[m] = Sc<T>::make(wbar[m * ncell + fc] * ia[fc]);
            } else if (kind == 3) {
#pragma unroll
                for (int m = 0; m < 4; ++m) fbar[m] = Sc<T>::make(-(wbar[m * ncell + fc] * ia[fc]));
            } else {
                const long fb = (kind == 0) ? (long)fj * n0 + wrap(fi + 1, n0) : fc + n0;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    fbar[m] = Sc<T>::make(wbar[m * ncell + fb] * ia[fb] - wbar[m * ncell + fc] * ia[fc]);
            }
            TT Ud[4][3][4], Fd[4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        Ud[a][b][k] = TT{base[a][b][k], Sc<T>::make((a == pa && b == pb && k == m) ? 1.0 : 0.0)};
            ogrid_face<RECON, FLUX, NSV, TT>(G, kind, fj, fc, Ud, Fd);
            T sum = Sc<T>::make(0.0);
#pragma unroll
            for (int k = 0; k < 4; ++k) sum = sum + fbar[k] * Fd[k].d;
            acc = acc + sum;
        };
#pragma nounroll
        for (int a = A0; a <= A1; ++a)
#pragma nounroll
            for (int b = B0; b <= B1; ++b) {
                // i-face with cell a = (cx - a + 1, cy - b + 1)
                const int fj0 = cy - (b - 1);
                if (fj0 >= 0 && fj0 < ny) face(0, wrap(cx - (a - 1), n0), fj0, a, b);
                // j-face with cell a = (cx - b + 1, cy - a + 1), j in [0, ny - 2]
                const int fj1 = cy - (a - 1);
                if (fj1 >= 0 && fj1 <= ny - 2) face(1, wrap(cx - (b - 1), n0), fj1, a, b);
            }
        if (cy == 0) face(2, cx, 0, 1, 1);
        if (cy == ny - 1) face(3, cx, ny - 1, 1, 1);
        if constexpr (SECOND) {
            ybar[idx] = accumulate ? ybar[idx] + acc.v : acc.v;
            ybar2[idx] = accumulate ? ybar2[idx] + acc.d : acc.d;
        } else {
            ybar[idx] = accumulate ? ybar[idx] + acc : acc;
        }
    }
}

template <int RECON, int FLUX, bool NSV>
static hipError_t launch_vjp_og(const Geom& G, const double* y, const double* v, const double* wbar, double* ybar,
                                double* ybar2, int accumulate, const int* gate, int col, hipStream_t st) {
    long g = (4 * G.ncell + 63) / 64;   // small blocks: O-grids have few cells and much work per cell
    if (g > 65536) g = 65536;
    if (v)
        hipLaunchKernelGGL((k_vjp_ogrid<RECON, true, FLUX, NSV>), dim3((unsigned)g), dim3(64), 0, st, G, y, v, wbar,
                           ybar, ybar2, accumulate, gate, col);
    else
        hipLaunchKernelGGL((k_vjp_ogrid<RECON, false, FLUX, NSV>), dim3((unsigned)g), dim3(64), 0, st, G, y, v,
                           wbar, ybar, ybar2, accumulate, gate, col);
    return hipGetLastError();
}

template <int RECON>
static hipError_t launch_vjp_ogrid(const Geom& G, const double* y, const double* v, const double* wbar, double* ybar,
                                   double* ybar2, int accumulate, const int* gate, int col, hipStream_t st) {
    const bool ns = G.mu != 0.0;
    if (G.flux == 1) {
        if (ns) return launch_vjp_og<RECON, 1, true>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
        return launch_vjp_og<RECON, 1, false>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
    }
    if (ns) return launch_vjp_og<RECON, 0, true>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
    return launch_vjp_og<RECON, 0, false>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
}

template <int D, int RECON, int FLUX, bool NSV, int GEO = 0>
static hipError_t launch_vjp_f(const Geom& G, const double* y, const double* v, const double* wbar, double* ybar,
                               double* ybar2, int accumulate, const int* gate, int col, hipStream_t st) {
    long g = (G.ncell + 255) / 256;
    if (g > 16384) g = 16384;
    if (v)
        hipLaunchKernelGGL((k_vjp<D, RECON, true, FLUX, NSV, GEO>), dim3((unsigned)g), dim3(256), 0, st, G, y, v, wbar,
                           ybar, ybar2, accumulate, gate, col);
    else
        hipLaunchKernelGGL((k_vjp<D, RECON, false, FLUX, NSV, GEO>), dim3((unsigned)g), dim3(256), 0, st, G, y, v, wbar,
                           ybar, ybar2, accumulate, gate, col);
    return hipGetLastError();
}

template <int D, int RECON, bool NSV>
static hipError_t launch_vjp_n(const Geom& G, const double* y, const double* v, const double* wbar, double* ybar,
                               double* ybar2, int accumulate, const int* gate, int col, hipStream_t st) {
    if (G.flux == 1) return launch_vjp_f<D, RECON, 1, NSV>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
    return launch_vjp_f<D, RECON, 0, NSV>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
}

template <int D, int RECON>
static hipError_t launch_vjp_t(const Geom& G, const double* y, const double* v, const double* wbar, double* ybar,
                               double* ybar2, int accumulate, const int* gate, int col, hipStream_t st) {
    if constexpr (D == 2) {
        if (G.metric && G.ogrid)
            return launch_vjp_ogrid<RECON>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
        // periodic curvilinear grid
        if (G.metric) {
            if (G.mu != 0.0) {
                if (G.flux == 1)
                    return launch_vjp_f<2, RECON, 1, true, 1>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
                return launch_vjp_f<2, RECON, 0, true, 1>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
            }
            if (G.flux == 1) return launch_vjp_f<2, RECON, 1, false, 1>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
            return launch_vjp_f<2, RECON, 0, false, 1>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
        }
    }
    if (G.mu != 0.0) return launch_vjp_n<D, RECON, true>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
    return launch_vjp_n<D, RECON, false>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
}

hipError_t launch_vjp(const Geom& G, int recon, const double* y, const double* v, const double* wbar, double* ybar,
                      double* ybar2, int accumulate, hipStream_t st, const int* gate, int col) {
    if (G.D == 2) return recon == 0 ? launch_vjp_t<2, 0>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st)
                                    : launch_vjp_t<2, 1>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
    return recon == 0 ? launch_vjp_t<3, 0>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st)
                      : launch_vjp_t<3, 1>(G, y, v, wbar, ybar, ybar2, accumulate, gate, col, st);
}

}  // namespace rok

