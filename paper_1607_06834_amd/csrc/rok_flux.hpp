// Pointwise pieces of the finite-volume right-hand side f (Sec. 3.2, eq. 11),
// templated on the scalar type (double, float, or dual numbers for exact
// derivatives): |.| and minmod with the branch rules of the reconstruction,
// the physical Euler flux, Rusanov's and Roe's fluxes, primitive <-> conserved variables
// and the flux of one face from the conserved states of its stencil cells.
// Every formula keeps one fixed, left-to-right operation order.
#pragma once

#include "rok_device.hpp"

namespace rok {

template <typename S> __device__ __forceinline__ S sabs(S x) { return Sc<S>::val(x) >= 0 ? x : -x; }

template <typename S> __device__ __forceinline__ S minmod(S a, S b) {
    using R = typename Sc<S>::R;
    if (Sc<S>::val(a) * Sc<S>::val(b) <= (R)0) return Sc<S>::make(0.0);
    return (Sc<S>::val(sabs(a)) <= Sc<S>::val(sabs(b))) ? a : b;
}

template <int D, typename S>
__device__ __forceinline__ void euler_flux(const S* U, const S* vel, S p, int d, S* F) {
    S un = vel[d];
    F[0] = U[1 + d];
#pragma unroll
    for (int e = 0; e < D; ++e) F[1 + e] = (e == d) ? U[1 + e] * un + p : U[1 + e] * un;
    F[D + 1] = (U[D + 1] + p) * un;
}

template <int D, typename S>
__device__ __forceinline__ void rusanov(const Geom& G, int d, const S* UL, S rL, const S* vL, S pL,
                                        const S* UR, S rR, const S* vR, S pR, S* Fh) {
    using R = typename Sc<S>::R;
    const R g = (R)G.g;
    const R half = (R)0.5;
    S cL = Sc<S>::sqrt_(g * pL / rL);
    S cR = Sc<S>::sqrt_(g * pR / rR);
    S sL = sabs(vL[d]) + cL;
    S sR = sabs(vR[d]) + cR;
    S a = (Sc<S>::val(sL) >= Sc<S>::val(sR)) ? sL : sR;
    S FL[D + 2], FR[D + 2];
    euler_flux<D>(UL, vL, pL, d, FL);
    euler_flux<D>(UR, vR, pR, d, FR);
    S ha = half * a;
#pragma unroll
    for (int m = 0; m < D + 2; ++m) Fh[m] = half * (FL[m] + FR[m]) - ha * (UR[m] - UL[m]);
}

// Roe's approximate Riemann flux along d (Roe 1981): the central flux minus
// half the sum over waves of |lambda_k| alpha_k r_k, with density-weighted
// averages of the two states.  Waves: u_n - c, u_n (entropy and D-1 shear
// waves), u_n + c; strengths alpha_1,3 = (dp -+ rho c du_n) / (2 c^2),
// alpha_2 = drho - dp / c^2, shear alpha_e = rho du_e; eigenvectors
// (1, u - c n, H - u_n c), (1, u, |u|^2 / 2), (0, e_e, u_e),
// (1, u + c n, H + u_n c).  Harten's entropy fix on the acoustic waves:
// |lambda| < delta -> (lambda^2 + delta^2) / (2 delta), delta = c / 8.
constexpr double kRoeFix = 0.125;

template <typename S>
__device__ __forceinline__ S roe_fixed(S lam, S delta) {
    S l = sabs(lam);
    if (Sc<S>::val(l) < Sc<S>::val(delta)) l = (l * l + delta * delta) / (delta + delta);
    return l;
}

// The dissipation vector sum_k |lambda_k| alpha_k r_k from the averaged state
// (u, H, rho, c2) and the primitive jumps (dr, du, dp) across the face.
template <int D, typename S>
__device__ __forceinline__ void roe_dissipation(const Geom& G, int d, const S* u, S H, S rho, S ke, S dr,
                                                const S* du, S dp, S* Dv) {
    using R = typename Sc<S>::R;
    const R gm1 = (R)G.gm1, half = (R)0.5;
    const S hke = half * ke;
    const S c2 = gm1 * (H - hke);
    const S c = Sc<S>::sqrt_(c2);
    const S un = u[d];
    const S rc = rho * c;
    const S cc = c2 + c2;
    const S a1 = (dp - rc * du[d]) / cc;
    const S a3 = (dp + rc * du[d]) / cc;
    const S a2 = dr - dp / c2;
    const S delta = (R)kRoeFix * c;
    const S l1 = roe_fixed(un - c, delta);
    const S l2 = sabs(un);
    const S l3 = roe_fixed(un + c, delta);
    const S w1 = l1 * a1, w2 = l2 * a2, w3 = l3 * a3;
    S wt[D];
#pragma unroll
    for (int e = 0; e < D; ++e) wt[e] = (e != d) ? l2 * (rho * du[e]) : Sc<S>::make(0.0);
    Dv[0] = w1 + w2 + w3;
#pragma unroll
    for (int e = 0; e < D; ++e) {
        if (e == d) Dv[1 + e] = w1 * (u[e] - c) + w2 * u[e] + w3 * (u[e] + c);
        else Dv[1 + e] = w1 * u[e] + w2 * u[e] + w3 * u[e] + wt[e];
    }
    const S unc = un * c;
    S en = w1 * (H - unc) + w2 * hke + w3 * (H + unc);
#pragma unroll
    for (int e = 0; e < D; ++e)
        if (e != d) en = en + wt[e] * u[e];
    Dv[D + 1] = en;
}

template <int D, typename S>
__device__ __forceinline__ void roe(const Geom& G, int d, const S* UL, S rL, const S* vL, S pL, const S* UR, S rR,
                                    const S* vR, S pR, S* Fh) {
    using R = typename Sc<S>::R;
    const R half = (R)0.5;
    S FL[D + 2], FR[D + 2];
    euler_flux<D>(UL, vL, pL, d, FL);
    euler_flux<D>(UR, vR, pR, d, FR);
    const S sL = Sc<S>::sqrt_(rL), sR = Sc<S>::sqrt_(rR);
    const S den = sL + sR;
    const S wL = sL / den, wR = sR / den;
    S u[D], du[D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        u[e] = wL * vL[e] + wR * vR[e];
        du[e] = vR[e] - vL[e];
    }
    const S HL = (UL[D + 1] + pL) / rL;
    const S HR = (UR[D + 1] + pR) / rR;
    const S H = wL * HL + wR * HR;
    const S rho = sL * sR;
    S ke = u[0] * u[0];
#pragma unroll
    for (int e = 1; e < D; ++e) ke = ke + u[e] * u[e];
    S Dv[D + 2];
    roe_dissipation<D>(G, d, u, H, rho, ke, rR - rL, du, pR - pL, Dv);
#pragma unroll
    for (int m = 0; m < D + 2; ++m) Fh[m] = half * (FL[m] + FR[m]) - half * Dv[m];
}

// The inviscid numerical flux selected at compile time (ROK_RUSANOV = 0, ROK_ROE = 1).
template <int D, int FLUX, typename S>
__device__ __forceinline__ void num_flux(const Geom& G, int d, const S* UL, S rL, const S* vL, S pL, const S* UR,
                                         S rR, const S* vR, S pR, S* Fh) {
    if constexpr (FLUX == 0) rusanov<D>(G, d, UL, rL, vL, pL, UR, rR, vR, pR, Fh);
    else roe<D>(G, d, UL, rL, vL, pL, UR, rR, vR, pR, Fh);
}

template <int D, typename S>
__device__ __forceinline__ void to_conserved(const Geom& G, S r, const S* vel, S p, S* U) {
    using R = typename Sc<S>::R;
    const R gm1 = (R)G.gm1;
    const R half = (R)0.5;
    S ke = vel[0] * vel[0];
#pragma unroll
    for (int d = 1; d < D; ++d) ke = ke + vel[d] * vel[d];
    U[0] = r;
#pragma unroll
    for (int d = 0; d < D; ++d) U[1 + d] = r * vel[d];
    U[D + 1] = p / gm1 + (half * r) * ke;
}


template <int D, typename S>
__device__ __forceinline__ void primitives(const Geom& G, const S* U, S& r, S* vel, S& p) {
    using R = typename Sc<S>::R;
    const R gm1 = (R)G.gm1;
    const R half = (R)0.5;
    r = U[0];
#pragma unroll
    for (int d = 0; d < D; ++d) vel[d] = U[1 + d] / r;
    S ke = vel[0] * vel[0];
#pragma unroll
    for (int d = 1; d < D; ++d) ke = ke + vel[d] * vel[d];
    p = gm1 * (U[D + 1] - (half * r) * ke);
}

// Inviscid flux of the face between stencil cells a and b = a + 1 along d,
// from the conserved states of the stencil: first order U[0] = a, U[1] = b;
// MUSCL U[0..3] = a-1, a, b, b+1.  FLUX: 0 Rusanov, 1 Roe.
template <int D, int RECON, typename S, int FLUX = 0>
__device__ __forceinline__ void face_flux_cells(const Geom& G, const S (*U)[D + 2], int d, S* Fh) {
    using R = typename Sc<S>::R;
    constexpr int NV = D + 2;
    S UL[NV], UR[NV], vL[D], vR[D], rL, rR, pL, pR;
    if constexpr (RECON == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            UL[m] = U[0][m];
            UR[m] = U[1][m];
        }
        primitives<D>(G, UL, rL, vL, pL);
        primitives<D>(G, UR, rR, vR, pR);
    } else {
        const R half = (R)0.5;
        S q[4][NV];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            S rr, vv[D], pp;
            primitives<D>(G, U[k], rr, vv, pp);
            q[k][0] = rr;
#pragma unroll
            for (int e = 0; e < D; ++e) q[k][1 + e] = vv[e];
            q[k][D + 1] = pp;
        }
        S qL[NV], qR[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            S am1 = q[0][m], a0 = q[1][m], ap1 = q[2][m], ap2 = q[3][m];
            qL[m] = a0 + half * minmod(a0 - am1, ap1 - a0);
            qR[m] = ap1 - half * minmod(ap1 - a0, ap2 - ap1);
        }
        rL = qL[0];
        rR = qR[0];
#pragma unroll
        for (int e = 0; e < D; ++e) {
            vL[e] = qL[1 + e];
            vR[e] = qR[1 + e];
        }
        pL = qL[D + 1];
        pR = qR[D + 1];
        to_conserved<D>(G, rL, vL, pL, UL);
        to_conserved<D>(G, rR, vR, pR, UR);
    }
    if constexpr (FLUX == 0) rusanov<D>(G, d, UL, rL, vL, pL, UR, rR, vR, pR, Fh);
    else roe<D>(G, d, UL, rL, vL, pL, UR, rR, vR, pR, Fh);
}

// ---------------------------------------------------------------------------
// Reverse mode of face_flux_cells: given Fbar = dL/dFhat at one face, adds
// Fbar^T dFhat/dU_q to Ubar[q] for every stencil cell q.  The branches
// (|.|, the wave-speed maximum, minmod) are those the forward evaluation
// takes, so this is the transpose of the tangent of face_flux_cells.  T may
// itself be a dual number, which yields the derivative of the adjoint along
// the dual direction (the second-order adjoint).
// ---------------------------------------------------------------------------
template <int D, typename T>
__device__ __forceinline__ void prim_rev(const Geom& G, const T* U, T rb, const T* vb_in, T pb, T* Ub) {
    using R = typename Sc<T>::R;
    const R gm1 = (R)G.gm1, half = (R)0.5;
    const T r = U[0];
    T vel[D], vb[D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        vel[e] = U[1 + e] / r;
        vb[e] = vb_in[e];
    }
    T ke = vel[0] * vel[0];
#pragma unroll
    for (int e = 1; e < D; ++e) ke = ke + vel[e] * vel[e];
    // p = gm1 (E - (r/2) ke)
    Ub[D + 1] = Ub[D + 1] + gm1 * pb;
    const T tb = -(gm1 * pb);                 // adjoint of t = (r/2) ke
    rb = rb + half * ke * tb;
    const T keb = half * r * tb;
#pragma unroll
    for (int e = 0; e < D; ++e) vb[e] = vb[e] + (vel[e] + vel[e]) * keb;
    // vel_e = U[1+e] / r
#pragma unroll
    for (int e = 0; e < D; ++e) {
        Ub[1 + e] = Ub[1 + e] + vb[e] / r;
        rb = rb - vb[e] * vel[e] / r;
    }
    Ub[0] = Ub[0] + rb;
}

// Reverse of to_conserved (U = (r, r vel, p/gm1 + (r/2) ke)): adds to rb, vb, pb.
template <int D, typename T>
__device__ __forceinline__ void cons_rev(const Geom& G, T r, const T* vel, const T* Ub, T& rb, T* vb, T& pb) {
    using R = typename Sc<T>::R;
    const R gm1 = (R)G.gm1, half = (R)0.5;
    T ke = vel[0] * vel[0];
#pragma unroll
    for (int e = 1; e < D; ++e) ke = ke + vel[e] * vel[e];
    rb = rb + Ub[0] + half * ke * Ub[D + 1];
    const T keb = half * r * Ub[D + 1];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        rb = rb + Ub[1 + e] * vel[e];
        vb[e] = vb[e] + Ub[1 + e] * r + (vel[e] + vel[e]) * keb;
    }
    pb = pb + Ub[D + 1] / gm1;
}

// One side of the reverse of rusanov(): the Euler flux of that side carries
// weight 1/2; when this side's wave speed is the maximum (taken), the
// adjoint ab of the maximum flows into its |u_d| + sqrt(g p / r).
template <int D, typename T>
__device__ __forceinline__ void rusanov_side_rev(const Geom& G, int d, const T* U, T r, const T* v, T p, T c, T x,
                                                 bool taken, T ab, const T* Fb, T* Ub, T& rb, T* vb, T& pb) {
    using R = typename Sc<T>::R;
    const R g = (R)G.g, half = (R)0.5;
    const T un = v[d];
    T unb = Sc<T>::make(0.0);
    Ub[1 + d] = Ub[1 + d] + half * Fb[0];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const T fb = half * Fb[1 + e];
        Ub[1 + e] = Ub[1 + e] + fb * un;
        unb = unb + fb * U[1 + e];
        if (e == d) pb = pb + fb;
    }
    const T fe = half * Fb[D + 1];
    Ub[D + 1] = Ub[D + 1] + fe * un;
    pb = pb + fe * un;
    unb = unb + fe * (U[D + 1] + p);
    if (taken) {
        unb = (Sc<T>::val(un) >= 0) ? unb + ab : unb - ab;
        const T xb = ab / (c + c);
        pb = pb + g * xb / r;
        rb = rb - xb * x / r;
    }
    vb[d] = vb[d] + unb;
}

// Reverse of rusanov(): adds to the adjoints of both side states.
template <int D, typename T>
__device__ __forceinline__ void rusanov_rev(const Geom& G, int d, const T* UL, T rL, const T* vL, T pL, const T* UR,
                                            T rR, const T* vR, T pR, const T* Fb, T* ULb, T& rLb, T* vLb, T& pLb,
                                            T* URb, T& rRb, T* vRb, T& pRb) {
    using R = typename Sc<T>::R;
    const R g = (R)G.g, half = (R)0.5;
    constexpr int NV = D + 2;
    const T xL = g * pL / rL, xR = g * pR / rR;
    const T cL = Sc<T>::sqrt_(xL), cR = Sc<T>::sqrt_(xR);
    const T sL = sabs(vL[d]) + cL, sR = sabs(vR[d]) + cR;
    const bool takeL = Sc<T>::val(sL) >= Sc<T>::val(sR);
    const T ha = half * (takeL ? sL : sR);
    // Fh = half (FL + FR) - ha (UR - UL)
    T hab = Sc<T>::make(0.0);
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        hab = hab - Fb[m] * (UR[m] - UL[m]);
        URb[m] = URb[m] - ha * Fb[m];
        ULb[m] = ULb[m] + ha * Fb[m];
    }
    const T ab = half * hab;
    rusanov_side_rev<D>(G, d, UL, rL, vL, pL, cL, xL, takeL, ab, Fb, ULb, rLb, vLb, pLb);
    rusanov_side_rev<D>(G, d, UR, rR, vR, pR, cR, xR, !takeL, ab, Fb, URb, rRb, vRb, pRb);
}

// Ubar[q] += Fbar^T dFhat/dU_q for the stencil cells of one face (conserved
// states U[q]; first order: 2 cells, MUSCL: 4).
template <int D, int RECON, typename T>
__device__ __forceinline__ void face_flux_vjp(const Geom& G, const T (*U)[D + 2], int d, const T* Fb,
                                              T (*Ub)[D + 2]) {
    using R = typename Sc<T>::R;
    constexpr int NV = D + 2;
    const T zero = Sc<T>::make(0.0);
    T ULb[NV], URb[NV], vLb[D], vRb[D], rLb = zero, rRb = zero, pLb = zero, pRb = zero;
#pragma unroll
    for (int m = 0; m < NV; ++m) ULb[m] = URb[m] = zero;
#pragma unroll
    for (int e = 0; e < D; ++e) vLb[e] = vRb[e] = zero;
    if constexpr (RECON == 0) {
        T rL, rR, pL, pR, vL[D], vR[D];
        primitives<D>(G, U[0], rL, vL, pL);
        primitives<D>(G, U[1], rR, vR, pR);
        rusanov_rev<D>(G, d, U[0], rL, vL, pL, U[1], rR, vR, pR, Fb, ULb, rLb, vLb, pLb, URb, rRb, vRb, pRb);
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            Ub[0][m] = Ub[0][m] + ULb[m];
            Ub[1][m] = Ub[1][m] + URb[m];
        }
        prim_rev<D>(G, U[0], rLb, vLb, pLb, Ub[0]);
        prim_rev<D>(G, U[1], rRb, vRb, pRb, Ub[1]);
    } else {
        const R half = (R)0.5;
        T q[4][NV];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T rr, vv[D], pp;
            primitives<D>(G, U[k], rr, vv, pp);
            q[k][0] = rr;
#pragma unroll
            for (int e = 0; e < D; ++e) q[k][1 + e] = vv[e];
            q[k][D + 1] = pp;
        }
        // reconstruction, remembering the minmod branch: 0 -> zero, 1 -> first slope, 2 -> second
        T qL[NV], qR[NV];
        int brL[NV], brR[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const T am1 = q[0][m], a0 = q[1][m], ap1 = q[2][m], ap2 = q[3][m];
            const T x1 = a0 - am1, y1 = ap1 - a0, x2 = ap1 - a0, y2 = ap2 - ap1;
            brL[m] = (Sc<T>::val(x1) * Sc<T>::val(y1) <= (R)0) ? 0
                     : ((Sc<T>::val(sabs(x1)) <= Sc<T>::val(sabs(y1))) ? 1 : 2);
            brR[m] = (Sc<T>::val(x2) * Sc<T>::val(y2) <= (R)0) ? 0
                     : ((Sc<T>::val(sabs(x2)) <= Sc<T>::val(sabs(y2))) ? 1 : 2);
            qL[m] = a0 + half * minmod(x1, y1);
            qR[m] = ap1 - half * minmod(x2, y2);
        }
        T UL[NV], UR[NV], vL[D], vR[D];
#pragma unroll
        for (int e = 0; e < D; ++e) {
            vL[e] = qL[1 + e];
            vR[e] = qR[1 + e];
        }
        to_conserved<D>(G, qL[0], vL, qL[D + 1], UL);
        to_conserved<D>(G, qR[0], vR, qR[D + 1], UR);
        rusanov_rev<D>(G, d, UL, qL[0], vL, qL[D + 1], UR, qR[0], vR, qR[D + 1], Fb, ULb, rLb, vLb, pLb, URb, rRb,
                       vRb, pRb);
        cons_rev<D>(G, qL[0], vL, ULb, rLb, vLb, pLb);
        cons_rev<D>(G, qR[0], vR, URb, rRb, vRb, pRb);
        T qLb[NV], qRb[NV];
        qLb[0] = rLb;
        qRb[0] = rRb;
#pragma unroll
        for (int e = 0; e < D; ++e) {
            qLb[1 + e] = vLb[e];
            qRb[1 + e] = vRb[e];
        }
        qLb[D + 1] = pLb;
        qRb[D + 1] = pRb;
        T qb[4][NV];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int m = 0; m < NV; ++m) qb[k][m] = zero;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            // qL = a0 + half mm(a0 - am1, ap1 - a0)
            qb[1][m] = qb[1][m] + qLb[m];
            const T mL = half * qLb[m];
            if (brL[m] == 1) {
                qb[1][m] = qb[1][m] + mL;
                qb[0][m] = qb[0][m] - mL;
            } else if (brL[m] == 2) {
                qb[2][m] = qb[2][m] + mL;
                qb[1][m] = qb[1][m] - mL;
            }
            // qR = ap1 - half mm(ap1 - a0, ap2 - ap1)
            qb[2][m] = qb[2][m] + qRb[m];
            const T mR = -(half * qRb[m]);
            if (brR[m] == 1) {
                qb[2][m] = qb[2][m] + mR;
                qb[1][m] = qb[1][m] - mR;
            } else if (brR[m] == 2) {
                qb[3][m] = qb[3][m] + mR;
                qb[2][m] = qb[2][m] - mR;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T vb[D];
#pragma unroll
            for (int e = 0; e < D; ++e) vb[e] = qb[k][1 + e];
            prim_rev<D>(G, U[k], qb[k][0], vb, qb[k][D + 1], Ub[k]);
        }
    }
}

// ---------------------------------------------------------------------------
// Reference-state form used by the FP32 kernels.  At low Mach number the
// pressure and energy are large constants plus small variations, and the
// flux differences that make up f are differences of those variations: in
// FP32 the fluxes themselves would lose most of those digits.  The FP32
// kernels therefore carry primitive perturbations q' = q - q0 (taken in FP64
// from a constant reference state q0 = (r0, u0, p0) before rounding) and
// evaluate F(q0 + q') - F(q0) from them without cancellation; the constant
// F(q0) drops out of every flux difference.
// ---------------------------------------------------------------------------
template <int D, typename R>
struct RefState {
    R r0, u0[D], p0, m0[D], H0;   // H0 = E0 + p0
};

// Rusanov flux minus F(q0) at a face, from the perturbations of the left and
// right primitive states (q = r', u'_0..u'_{D-1}, p').
template <int D, typename S>
__device__ __forceinline__ void rusanov_ref(const Geom& G, const RefState<D, typename Sc<S>::R>& Q, int d,
                                            const S* qL, const S* qR, S* Fh) {
    using R = typename Sc<S>::R;
    const R g = (R)G.g, gm1 = (R)G.gm1, half = (R)0.5;
    constexpr int NV = D + 2;
    S F[2][NV], Up[2][NV], sp[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const S* q = side ? qR : qL;
        const S rp = q[0], pp = q[D + 1];
        const S r = Q.r0 + rp, p = Q.p0 + pp;
        S u[D], mp[D];
#pragma unroll
        for (int e = 0; e < D; ++e) {
            u[e] = Q.u0[e] + q[1 + e];
            mp[e] = Q.r0 * q[1 + e] + rp * u[e];      // rho u - rho0 u0
        }
        S uu = u[0] * u[0], ku = q[1] * (u[0] + Q.u0[0]);
#pragma unroll
        for (int e = 1; e < D; ++e) {
            uu = uu + u[e] * u[e];
            ku = ku + q[1 + e] * (u[e] + Q.u0[e]);       // |u|^2 - |u0|^2
        }
        const S Ep = pp / gm1 + half * (rp * uu + Q.r0 * ku);   // E - E0
        const S Hp = Ep + pp;                                    // (E + p) - (E0 + p0)
        Up[side][0] = rp;
#pragma unroll
        for (int e = 0; e < D; ++e) Up[side][1 + e] = mp[e];
        Up[side][D + 1] = Ep;
        F[side][0] = mp[d];
#pragma unroll
        for (int e = 0; e < D; ++e)
            F[side][1 + e] = (e == d) ? mp[d] * u[e] + Q.m0[d] * q[1 + e] + pp : mp[d] * u[e] + Q.m0[d] * q[1 + e];
        F[side][D + 1] = Hp * u[d] + Q.H0 * q[1 + d];
        sp[side] = sabs(u[d]) + Sc<S>::sqrt_(g * p / r);
    }
    const S a = (Sc<S>::val(sp[0]) >= Sc<S>::val(sp[1])) ? sp[0] : sp[1];
    const S ha = half * a;
#pragma unroll
    for (int m = 0; m < NV; ++m) Fh[m] = half * (F[0][m] + F[1][m]) - ha * (Up[1][m] - Up[0][m]);
}

// Roe flux minus F(q0) at a face in the reference-state form: the central part
// from the flux perturbations (as in rusanov_ref), the dissipation from the
// full averaged state and the jumps of the primitive perturbations (which are
// the jumps of the primitives themselves).
template <int D, typename S>
__device__ __forceinline__ void roe_ref(const Geom& G, const RefState<D, typename Sc<S>::R>& Q, int d, const S* qL,
                                        const S* qR, S* Fh) {
    using R = typename Sc<S>::R;
    const R gm1 = (R)G.gm1, half = (R)0.5;
    constexpr int NV = D + 2;
    S F[2][NV], Hs[2], rs[2], sq[2], us[2][D];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const S* q = side ? qR : qL;
        const S rp = q[0], pp = q[D + 1];
        const S r = Q.r0 + rp;
        S u[D], mp[D];
#pragma unroll
        for (int e = 0; e < D; ++e) {
            u[e] = Q.u0[e] + q[1 + e];
            mp[e] = Q.r0 * q[1 + e] + rp * u[e];
        }
        S uu = u[0] * u[0], ku = q[1] * (u[0] + Q.u0[0]);
#pragma unroll
        for (int e = 1; e < D; ++e) {
            uu = uu + u[e] * u[e];
            ku = ku + q[1 + e] * (u[e] + Q.u0[e]);
        }
        const S Ep = pp / gm1 + half * (rp * uu + Q.r0 * ku);
        const S Hp = Ep + pp;
        F[side][0] = mp[d];
#pragma unroll
        for (int e = 0; e < D; ++e)
            F[side][1 + e] = (e == d) ? mp[d] * u[e] + Q.m0[d] * q[1 + e] + pp : mp[d] * u[e] + Q.m0[d] * q[1 + e];
        F[side][D + 1] = Hp * u[d] + Q.H0 * q[1 + d];
        rs[side] = r;
        sq[side] = Sc<S>::sqrt_(r);
        Hs[side] = (Q.H0 + Hp) / r;          // (E + p) / rho
#pragma unroll
        for (int e = 0; e < D; ++e) us[side][e] = u[e];
    }
    const S den = sq[0] + sq[1];
    const S wL = sq[0] / den, wR = sq[1] / den;
    S u[D], du[D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        u[e] = wL * us[0][e] + wR * us[1][e];
        du[e] = qR[1 + e] - qL[1 + e];
    }
    const S H = wL * Hs[0] + wR * Hs[1];
    const S rho = sq[0] * sq[1];
    S ke = u[0] * u[0];
#pragma unroll
    for (int e = 1; e < D; ++e) ke = ke + u[e] * u[e];
    S Dv[NV];
    roe_dissipation<D>(G, d, u, H, rho, ke, qR[0] - qL[0], du, qR[D + 1] - qL[D + 1], Dv);
    (void)rs;
#pragma unroll
    for (int m = 0; m < NV; ++m) Fh[m] = half * (F[0][m] + F[1][m]) - half * Dv[m];
}

template <int D, int FLUX, typename S>
__device__ __forceinline__ void num_flux_ref(const Geom& G, const RefState<D, typename Sc<S>::R>& Q, int d,
                                             const S* qL, const S* qR, S* Fh) {
    if constexpr (FLUX == 0) rusanov_ref<D>(G, Q, d, qL, qR, Fh);
    else roe_ref<D>(G, Q, d, qL, qR, Fh);
}

}  // namespace rok
