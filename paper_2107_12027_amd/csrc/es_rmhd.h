// Device physics of the RMHD system: state, conservative variables, flux,
// entropy variables, conservative-to-primitive recovery, the two-point EC pair
// flux with its Godunov-Powell source pair, and the ES face dissipation with a
// numeric scaled eigen-structure.
//
// Primitive slots P = (rho, u_1, u_2, u_3, p, B_1, B_2, B_3) with u = W v (all
// three components kept in 2D), conservative slots U = (D, m_1..3, E, B_1..3).
#pragma once

#include <type_traits>

#include "es_rhd.h"
#include "es_dual.h"

namespace es {

// Derived quantities of a primitive state (Section 1): W, v, beta = rho/p,
// h = 1 + G/(G-1) p/rho, v.B, b^0 = W v.B, b = B/W + W (v.B) v,
// |b|^2 = |B|^2/W^2 + (v.B)^2.
template <typename R>
struct StateRMHD {
    R rho, p, W, beta, h, vB, b0, bsq, BB;
    R u[3], v[3], B[3], b[3];
};

template <typename R>
__device__ __forceinline__ StateRMHD<R> rmhd_state(double G, const R* P) {
    StateRMHD<R> s;
    s.rho = P[0];
    s.p = P[4];
    R uu = R(0.0), BB = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.u[k] = P[1 + k];
        s.B[k] = P[5 + k];
        uu += s.u[k] * s.u[k];
        BB += s.B[k] * s.B[k];
    }
    s.W = xsqrt(R(1.0) + uu);
    const R iW = R(1.0) / s.W;
    R vB = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) { s.v[k] = s.u[k] * iW; vB += s.v[k] * s.B[k]; }
    s.vB = vB;
    s.BB = BB;
    s.beta = s.rho / s.p;
    s.h = R(1.0) + (G / (G - 1.0)) * s.p / s.rho;
    s.b0 = s.W * vB;
#pragma unroll
    for (int k = 0; k < 3; ++k) s.b[k] = s.B[k] * iW + s.W * vB * s.v[k];
    s.bsq = BB * iW * iW + vB * vB;
    return s;
}

// U(P) (eq. RMHDdiv2): D = rho W, m = (Z + |B|^2) v - (v.B) B,
// E = Z - p - |b|^2/2 + |B|^2, Z = rho h W^2.
template <typename R>
__device__ __forceinline__ void rmhd_cons(const StateRMHD<R>& s, R* U) {
    const R Z = s.rho * s.h * s.W * s.W;
    U[0] = s.rho * s.W;
#pragma unroll
    for (int k = 0; k < 3; ++k) U[1 + k] = (Z + s.BB) * s.v[k] - s.vB * s.B[k];
    U[4] = Z - s.p - R(0.5) * s.bsq + s.BB;
#pragma unroll
    for (int k = 0; k < 3; ++k) U[5 + k] = s.B[k];
}

// x_1 flux F_1(P) (eq. RMHDdiv2), p_tot = p + |b|^2/2.
template <typename R>
__device__ __forceinline__ void rmhd_flux1(const StateRMHD<R>& s, const R* U, R* F) {
    const R ptot = s.p + R(0.5) * s.bsq;
    const R iW2 = R(1.0) / (s.W * s.W);
    F[0] = U[0] * s.v[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        R val = U[1 + c] * s.v[0] - s.B[0] * (s.B[c] * iW2 + s.vB * s.v[c]);
        if (c == 0) val = val + ptot;
        F[1 + c] = val;
    }
    F[4] = U[1];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[5 + c] = s.v[0] * s.B[c] - s.B[0] * s.v[c];
}

// Entropy variables V = (G/(G-1) + ln rho + ln beta/(G-1) + beta, beta u, -beta W, beta b)
template <typename R>
__device__ __forceinline__ void rmhd_entropy_vars(double G, const StateRMHD<R>& s, R* V) {
    V[0] = (G / (G - 1.0)) + xlog(s.rho) + xlog(s.beta) * (1.0 / (G - 1.0)) + s.beta;
#pragma unroll
    for (int k = 0; k < 3; ++k) { V[1 + k] = s.beta * s.u[k]; V[5 + k] = s.beta * s.b[k]; }
    V[4] = -s.beta * s.W;
}

// Phi'(V) in U slots (eq. Phi): (0, B/W^2 + v (v.B), v.B, v)
template <typename R>
__device__ __forceinline__ void rmhd_phi_prime(const StateRMHD<R>& s, R* Pp) {
    const R iW2 = R(1.0) / (s.W * s.W);
    Pp[0] = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) { Pp[1 + k] = s.B[k] * iW2 + s.v[k] * s.vB; Pp[5 + k] = s.v[k]; }
    Pp[4] = s.vB;
}

// Conservative -> primitive (Section 1: a scalar nonlinear equation) in the
// unknown Z = rho h W^2:  v.B = (m.B)/Z,
//   |v|^2 = (Z^2 |m|^2 + (m.B)^2 (2Z + |B|^2)) / (Z^2 (Z + |B|^2)^2),
//   p = (G-1)/G (Z/W^2 - D/W),
//   f(Z) = Z - p + |B|^2 - |B|^2/(2 W^2) - (m.B)^2/(2 Z^2) - E = 0.
// Safeguarded Newton (f' by a dual number) on the bracket (0, 2(E+1) + |B|^2],
// starting from ``guess`` when it lies inside; iterates with |v| >= 1 move the
// lower end of the bracket.  Returns 0 on success, 1 for an inadmissible state
// (D <= 0 or p <= 0), 2 without convergence.
__device__ __forceinline__ int c2p_rmhd(double G, const double* U, double guess, double* P) {
    const double D = U[0], E = U[4];
    double mm2 = 0.0, BB = 0.0, mB = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mm2 += U[1 + k] * U[1 + k];
        BB += U[5 + k] * U[5 + k];
        mB += U[1 + k] * U[5 + k];
    }
    if (!(D > 0.0) || !(E > 0.0)) return 1;
    double lo = 0.0, hi = 2.0 * (E + 1.0) + BB;
    double Z = (guess > lo && guess < hi) ? guess : hi;
    const double gm1 = (G - 1.0) / G;
    int conv = 0;
    using D1 = Dual<1>;
    for (int it = 0; it < 300; ++it) {
        const D1 z = D1::seed(Z, 0);
        const D1 v2 = (z * z * mm2 + mB * mB * (2.0 * z + BB)) / (z * z * (z + BB) * (z + BB));
        if (!(v2.v < 1.0)) {
            lo = Z;
            Z = 0.5 * (lo + hi);
            if (hi - lo <= 1e-16 * hi) break;
            continue;
        }
        const D1 W2 = 1.0 / (1.0 - v2);
        const D1 W = xsqrt(W2);
        const D1 p = gm1 * (z / W2 - D / W);
        const D1 f = z - p + BB - BB / (2.0 * W2) - mB * mB / (2.0 * z * z) - E;
        if (f.v == 0.0) { conv = 1; break; }
        if (f.v < 0.0) lo = Z; else hi = Z;
        double Zn = Z - f.v / f.d[0];
        if (!(Zn > lo && Zn < hi)) Zn = 0.5 * (lo + hi);
        const double dz = fabs(Zn - Z);
        Z = Zn;
        if (dz <= 1e-15 * Z || hi - lo <= 1e-15 * hi) { conv = 1; break; }
    }
    const double vB = mB / Z;
    double v[3], v2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) { v[k] = (U[1 + k] + vB * U[5 + k]) / (Z + BB); v2 += v[k] * v[k]; }
    if (!(v2 < 1.0)) return 1;
    const double W = 1.0 / sqrt(1.0 - v2);
    const double rho = D / W;
    const double p = gm1 * (Z / (W * W) - rho);
    if (!(p > 0.0) || !(p < INFINITY)) return 1;
    P[0] = rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) { P[1 + k] = W * v[k]; P[5 + k] = U[5 + k]; }
    P[4] = p;
    return conv ? 0 : 2;
}

// Node data of the residual's line loads: primitive state, logarithms and the
// derived quantities the pair flux averages (R = double, or dual numbers for the
// adjoint's local Jacobians).
template <typename R = double>
struct NodeRMHDT {
    R rho, p, beta, W, lr, lb, b0, Wb0, Wb02, sb, b02;
    R u[3], B[3], b[3], Wbk2[3], bk2[3];
};
using NodeRMHD = NodeRMHDT<double>;

__device__ __forceinline__ double value_of(double x) { return x; }

template <typename R = double>
__device__ __forceinline__ NodeRMHDT<R> node_rmhd(double G, const R* P, R lr, R lb) {
    const StateRMHD<R> s = rmhd_state<R>(G, P);
    NodeRMHDT<R> n;
    n.rho = s.rho; n.p = s.p; n.beta = s.beta; n.W = s.W; n.lr = lr; n.lb = lb;
    n.b0 = s.b0;
    n.Wb0 = s.W * s.b0;
    n.Wb02 = s.W * s.b0 * s.b0;
    n.b02 = s.b0 * s.b0;
    R sb = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        n.u[k] = s.u[k]; n.B[k] = s.B[k]; n.b[k] = s.b[k];
        n.bk2[k] = s.b[k] * s.b[k];
        n.Wbk2[k] = s.W * n.bk2[k];
        sb += n.bk2[k];
    }
    n.sb = sb;
    return n;
}

// Two-point EC flux for RMHD (eq. ECFluxCurv, eq. UFcircle): F = a_t U~ + sum_j a_j F~_j
// with U~ the paper's closed form (Section 3.1; R_1 read with the k = 1..3 sum of
// {W (b^k)^2}/2 - {b^k} U~_{k+5}) and F~_j solving [V].F~_j = [psi_j] - {B_j}[Phi];
// {.} arithmetic means (of products where products appear), ^ln logarithmic means.
// Also the source pair B~ = 1/4 sum_j (a_j,l + a_j,r)(B_j,l + B_j,r) (eq. BFlux_O2)
// and the VCL pair value a_t (eq. MetricsFlux_O2).
//
// R = float is the mixed form: the pair algebra in FP32 except the small-jump
// branch of the logarithmic means (FP64), written as coefficients K_t = U~ and
// K_j = F~_j that are contracted with the metrics in FP64 (as the RHD mixed
// form: equal states give equal coefficients, so the metric sums cancel in FP64);
// B~ and a_t stay FP64.
// NR: the node type (double, or the dual numbers of the adjoint, then R = NR and
// F holds dual numbers too).
template <int DIM, typename R = double, typename NR = double>
__device__ __forceinline__ void pair_flux_rmhd(double G, const NodeRMHDT<NR>& l, const NodeRMHDT<NR>& r,
                                               const double* al, const double* ar,
                                               typename std::conditional<std::is_same<R, float>::value, double,
                                                                         R>::type* F,
                                               double& Jt, double& Bt) {
    constexpr bool F32 = std::is_same<R, float>::value;
    using OT = typename std::conditional<F32, double, R>::type;
    R rho_ln, beta_ln;
    if constexpr (F32) {
        rho_ln = log_mean_mixed(l.rho, r.rho, l.lr, r.lr);
        beta_ln = log_mean_mixed(l.beta, r.beta, l.lb, r.lb);
    } else {
        rho_ln = log_mean(l.rho, r.rho, l.lr, r.lr);
        beta_ln = log_mean(l.beta, r.beta, l.lb, r.lb);
    }
    auto mean = [](const NR& a, const NR& b) { return R(0.5) * (R(a) + R(b)); };
    const R rho = mean(l.rho, r.rho), beta = mean(l.beta, r.beta);
    const R W = mean(l.W, r.W), b0 = mean(l.b0, r.b0);
    const R Wb0 = mean(l.Wb0, r.Wb0), Wb02 = mean(l.Wb02, r.Wb02);
    const R sb = mean(l.sb, r.sb), b02 = mean(l.b02, r.b02);
    R u[3], b[3], B[3], Wbk2[3], bk2[3], ujsb[3], ujb02[3];
    R uu = R(0.0), sbk2 = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u[k] = mean(l.u[k], r.u[k]);
        b[k] = mean(l.b[k], r.b[k]);
        B[k] = mean(l.B[k], r.B[k]);
        Wbk2[k] = mean(l.Wbk2[k], r.Wbk2[k]);
        bk2[k] = mean(l.bk2[k], r.bk2[k]);
        ujsb[k] = R(0.5) * (R(l.u[k]) * R(l.sb) + R(r.u[k]) * R(r.sb));
        ujb02[k] = R(0.5) * (R(l.u[k]) * R(l.b02) + R(r.u[k]) * R(r.b02));
        uu += u[k] * u[k];
        sbk2 += bk2[k];
    }
    R iW, ib, a0, iden;
    if constexpr (F32) {
        iW = frcp(W);
        ib = frcp(beta);
        a0 = R(1.0) + frcp(R(G - 1.0) * beta_ln);
        iden = frcp(W * W - uu);
    } else {
        iW = 1.0 / W;
        ib = 1.0 / beta;
        a0 = 1.0 + 1.0 / ((G - 1.0) * beta_ln);
        iden = 1.0 / (W * W - uu);
    }
    // U~
    R Ut[8];
    const R U1 = rho_ln * W;
    R UB[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) UB[k] = (W * W * b[k] - Wb0 * u[k]) * iW;
    const R a1 = rho + R(0.5) * beta * sbk2 + R(0.5) * beta * Wb02 * iW;
    R R1 = -a0 * U1 - R(0.5) * Wb02;
#pragma unroll
    for (int k = 0; k < 3; ++k) R1 += R(0.5) * Wbk2[k] - b[k] * UB[k];
    R Rk[3], uR = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) { Rk[k] = (a1 * u[k] - beta * Wb0 * b[k]) * iW; uR += u[k] * Rk[k]; }
    const R Dd = beta * (W * W - uu) * iW;
    R U5;
    if constexpr (F32) U5 = (uR - beta * R1) * frcp(Dd);
    else U5 = (uR - beta * R1) / Dd;
    Ut[0] = U1;
#pragma unroll
    for (int k = 0; k < 3; ++k) { Ut[1 + k] = u[k] * U5 * iW + Rk[k] * ib; Ut[5 + k] = UB[k]; }
    Ut[4] = U5;
    const double at = 0.5 * (al[0] + ar[0]);
#pragma unroll
    for (int c = 0; c < 8; ++c) F[c] = at * OT(Ut[c]);
    double bt = 0.0;
    // F~_j for the directions of the grid
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        const double aj = 0.5 * (al[1 + j] + ar[1 + j]);
        bt += 0.25 * (al[1 + j] + ar[1 + j]) * (value_of(l.B[j]) + value_of(r.B[j]));
        const R c0 = -beta * (u[j] * b0 + B[j]);
        const R F1 = rho_ln * u[j];
        R FB[3], Pk[3], uP = R(0.0), bFB = R(0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            FB[k] = u[j] * b[k] + c0 * u[k] * ib * iW;
            Pk[k] = (c0 * iW) * (b[k] - b0 * u[k] * iW);
        }
        Pk[j] += rho + R(0.5) * beta * sb - R(0.5) * beta * b02;
#pragma unroll
        for (int k = 0; k < 3; ++k) { uP += u[k] * Pk[k]; bFB += b[k] * FB[k]; }
        const R Q = R(0.5) * ujsb[j] - R(0.5) * ujb02[j] - B[j] * b0;
        const R F5 = W * (a0 * F1 + uP * ib + bFB - Q) * iden;
        F[0] += aj * OT(F1);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            F[1 + k] += aj * OT(u[k] * F5 * iW + Pk[k] * ib);
            F[5 + k] += aj * OT(FB[k]);
        }
        F[4] += aj * OT(F5);
    }
    Jt = at;
    Bt = bt;
}

// ---------------------------------------------------------------------------
// numeric scaled eigen-structure of the (Godunov-Powell modified) x_1 flux
// Jacobian at a state in the rotated frame
// ---------------------------------------------------------------------------

// Jacobians dU/dP, dF_1/dP (+ Phi'(V) e_{B_1}^T, the Godunov-Powell term) and
// dV/dP at the primitive state P by forward-mode dual numbers.
__device__ __forceinline__ void rmhd_jacobians(double G, const double* P, double JU[8][8],
                                               double JF[8][8], double JV[8][8], double* Pp) {
    using D8 = Dual<8>;
    D8 Pd[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) Pd[i] = D8::seed(P[i], i);
    const StateRMHD<D8> s = rmhd_state<D8>(G, Pd);
    D8 U[8], F[8], V[8];
    rmhd_cons<D8>(s, U);
    rmhd_flux1<D8>(s, U, F);
    rmhd_entropy_vars<D8>(G, s, V);
    D8 Ph[8];
    rmhd_phi_prime<D8>(s, Ph);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        Pp[r] = Ph[r].v;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            JU[r][c] = U[r].d[c];
            JF[r][c] = F[r].d[c] + (c == 5 ? Ph[r].v : 0.0);
            JV[r][c] = V[r].d[c];
        }
    }
}

// Inverse of a small dense matrix by Gauss-Jordan elimination with partial pivoting.
template <int N>
__device__ __forceinline__ void invert(double A[N][N], double X[N][N]) {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) X[r][c] = r == c ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int piv = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < N; ++r)
            if (fabs(A[r][k]) > best) { best = fabs(A[r][k]); piv = r; }
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            if (r == piv) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    double t = A[k][c]; A[k][c] = A[r][c]; A[r][c] = t;
                    t = X[k][c]; X[k][c] = X[r][c]; X[r][c] = t;
                }
            }
        }
        const double ip = 1.0 / A[k][k];
#pragma unroll
        for (int c = 0; c < N; ++c) { A[k][c] *= ip; X[k][c] *= ip; }
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (r == k) continue;
            const double f = A[r][k];
#pragma unroll
            for (int c = 0; c < N; ++c) { A[r][c] -= f * A[k][c]; X[r][c] -= f * X[k][c]; }
        }
    }
}

// Cyclic Jacobi eigen-decomposition of the symmetric 8x8 matrix Q held as its
// lower triangle (36 entries: only what a symmetric rotation changes is
// updated).  lam receives the eigenvalues, the columns of Zv the orthonormal
// eigenvectors.  Rotation (p, q): t = sgn(th)/(|th| + sqrt(th^2 + 1)),
// th = (a_qq - a_pp)/(2 a_pq), c = 1/sqrt(t^2 + 1), s = t c, tau = s/(1 + c):
// a_pp -= t a_pq, a_qq += t a_pq, a_pq = 0, and for r != p, q
// a_rp -= s (a_rq + tau a_rp), a_rq += s (a_rp - tau a_rq) (the same for the
// rows of Zv).  An element below 1e-18 of its diagonal pair is set to zero
// instead of rotated; the sweeps stop when the off-diagonal part is below
// 1e-30 of the diagonal (squared) or after 12 sweeps.
__device__ __forceinline__ constexpr int tri8(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

__device__ __forceinline__ void jacobi_eigen_sym8(const double Q[8][8], double lam[8], double Zv[8][8]) {
    double a[36];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) a[tri8(i, j)] = Q[i][j];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) Zv[r][c] = r == c ? 1.0 : 0.0;
#pragma unroll 1
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            dia += a[tri8(i, i)] * a[tri8(i, i)];
#pragma unroll
            for (int j = 0; j < i; ++j) off += a[tri8(i, j)] * a[tri8(i, j)];
        }
        if (!(off > 1e-30 * dia)) break;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
#pragma unroll
            for (int q = p + 1; q < 8; ++q) {
                const double apq = a[tri8(q, p)];
                const double app = a[tri8(p, p)], aqq = a[tri8(q, q)];
                if (fabs(apq) <= 1e-18 * (fabs(app) + fabs(aqq))) {
                    a[tri8(q, p)] = 0.0;
                    continue;
                }
                // (|th| <= 5e17 here, so th^2 + 1 stays finite; the reciprocals and
                // roots are of positive normal numbers)
                const double th = fdiv(aqq - app, 2.0 * apq);
                const double t = fdiv(th >= 0.0 ? 1.0 : -1.0, fabs(th) + psqrt(th * th + 1.0));
                const double c = frsqrt(t * t + 1.0), sn = t * c, tau = fdiv(sn, 1.0 + c);
                a[tri8(p, p)] = app - t * apq;
                a[tri8(q, q)] = aqq + t * apq;
                a[tri8(q, p)] = 0.0;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    if (r == p || r == q) continue;
                    const double arp = a[tri8(r, p)], arq = a[tri8(r, q)];
                    a[tri8(r, p)] = arp - sn * (arq + tau * arp);
                    a[tri8(r, q)] = arq + sn * (arp - tau * arq);
                }
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const double zp = Zv[r][p], zq = Zv[r][q];
                    Zv[r][p] = zp - sn * (zq + tau * zp);
                    Zv[r][q] = zq + sn * (zp - tau * zq);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) lam[i] = a[tri8(i, i)];
}

// Symmetric pencil of the eigenproblem in entropy variables: A0 = dU/dV =
// JU JV^{-1} and S = dF/dV = JF JV^{-1} (both symmetric; symmetrised against
// rounding); with A0 = L L^T, Q = L^{-1} S L^{-T}; Q = Z diag(lambda) Z^T gives
// R = L Z with R R^T = A0 and (dF/dU) R = R diag(lambda) (Section 4).
__device__ __forceinline__ void rmhd_pencil(const double JU[8][8], const double JF[8][8],
                                            double JV[8][8], double Lc[8][8], double Q[8][8]) {
    double X[8][8];
    invert<8>(JV, X);
    double A0[8][8], S[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            double a = 0.0, f = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) { a += JU[r][k] * X[k][c]; f += JF[r][k] * X[k][c]; }
            A0[r][c] = a;
            S[r][c] = f;
        }
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = r + 1; c < 8; ++c) {
            const double a = 0.5 * (A0[r][c] + A0[c][r]), f = 0.5 * (S[r][c] + S[c][r]);
            A0[r][c] = A0[c][r] = a;
            S[r][c] = S[c][r] = f;
        }
    // Cholesky A0 = L L^T
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) Lc[r][c] = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double d = A0[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lc[j][k] * Lc[j][k];
        const double ljj = sqrt(d);
        Lc[j][j] = ljj;
        const double il = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
            double s = A0[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= Lc[i][k] * Lc[j][k];
            Lc[i][j] = s * il;
        }
    }
    // Y = L^{-1} S (forward substitution per column), Q = L^{-1} Y^T
    double Y[8][8];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double s = S[i][c];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= Lc[i][k] * Y[k][c];
            Y[i][c] = s / Lc[i][i];
        }
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double s = Y[c][i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= Lc[i][k] * Q[k][c];
            Q[i][c] = s / Lc[i][i];
        }
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = r + 1; c < 8; ++c) {
            const double q = 0.5 * (Q[r][c] + Q[c][r]);
            Q[r][c] = Q[c][r] = q;
        }
}

// Spectral radius of the Godunov-Powell modified x_1 flux Jacobian at the
// rotated state P (rho, u = W v, p, B), for eq. cfl.  Its eigenvalues are v_1
// (entropy and divergence waves), the Alfven pair and the magnetosonic quartet;
// the fast pair, the extreme roots of the magnetosonic dispersion relation of
// ideal RMHD,
//   Q(l) = rho h (1/c_s^2 - 1) a^4 - (rho h + |b|^2/c_s^2) a^2 g + (b^1 - l b^0)^2 g,
//   a = W (l - v_1), g = 1 - l^2, c_s^2 = Gamma p / (rho h),
// bound all the others.  The four roots are real and lie in (-1, 1), the leading
// coefficient is positive and Q(+-1) = rho h (1/c_s^2 - 1) a^4 > 0, so Newton's
// method started at l = 1 (l = -1) moves monotonically to the largest (smallest)
// root.  (Checked against the eigenvalues of the full Jacobian by the CFL parity
// tests; the dissipation keeps the numeric eigen-structure, which it needs for
// the eigenvectors.)
__device__ __forceinline__ double rmhd_max_speed(double G, const double* P) {
    const double rho = P[0], p = P[4];
    const double u1 = P[1], u2 = P[2], u3 = P[3];
    const double B1 = P[5], B2 = P[6], B3 = P[7];
    const double W = sqrt(1.0 + u1 * u1 + u2 * u2 + u3 * u3);
    const double iW = 1.0 / W;
    const double v1 = u1 * iW;
    const double b0 = u1 * B1 + u2 * B2 + u3 * B3;                 // W (v . B)
    const double b1 = B1 * iW + b0 * v1;
    const double vB = b0 * iW;
    const double bb = (B1 * B1 + B2 * B2 + B3 * B3) * iW * iW + vB * vB;
    const double rh = rho + G / (G - 1.0) * p;
    const double ics2 = rh / (G * p);
    const double A = rh * (ics2 - 1.0), C = rh + bb * ics2;
    double ext[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        double l = side == 0 ? 1.0 : -1.0;
#pragma unroll 1
        for (int it = 0; it < 200; ++it) {
            const double a = W * (l - v1), g = 1.0 - l * l, e = b1 - l * b0;
            const double a2 = a * a;
            const double q = A * a2 * a2 - C * a2 * g + e * e * g;
            const double dq = 4.0 * A * a2 * a * W - C * (2.0 * a * W * g - 2.0 * a2 * l) - 2.0 * e * b0 * g -
                              2.0 * e * e * l;
            const double step = q / dq;
            // monotone: the iterate moves towards the root until rounding stops it
            if (!(side == 0 ? step > 0.0 : step < 0.0)) break;
            l -= step;
            if (fabs(step) <= 1e-16) break;
        }
        ext[side] = l;
    }
    return fmax(fabs(ext[0]), fabs(ext[1]));
}

// Rotate the vector slots (1..3) and (5..7) of an 8-vector by T (or T^T).
template <bool TRANSPOSE>
__device__ __forceinline__ void rotate8(const double T[3][3], const double* a, double* o) {
    o[0] = a[0];
    o[4] = a[4];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double t = TRANSPOSE ? T[c][r] : T[r][c];
            s1 += t * a[1 + c];
            s2 += t * a[5 + c];
        }
        o[1 + r] = s1;
        o[5 + r] = s2;
    }
}

// Eigen-groups of the RMHD pencil: eigenvalues closer than GROUP_TOL (chained)
// form one group, and each group gets the A0^{-1}-Gram-Schmidt sequence of the
// projections of unit seeds onto its eigenspace, P_g e_s = sum_{a in g} r_a
// (r_a^T A0^{-1} e_s); the group of v_n (entropy and div B waves) takes e_D,
// e_{B_n} first, the others e_1, e_2, ...  A seed contributes when what is left of
// its projection exceeds SEED_TOL times its A0^{-1} norm.  In z-space (r = L z)
// the A0^{-1} products are Euclidean and r_a^T A0^{-1} e_s = z_a . (L^{-1} e_s).
// Writes Rc[k] = L z for the canonical vector z of position k (a member of k's
// group); Zv (the eigenvectors z_a as columns) is overwritten by R = L Z.
constexpr double GROUP_TOL = 1e-6;
constexpr double SEED_TOL = 1e-3;

__device__ __forceinline__ void canonical_columns(const double* lam, double Zv[8][8],
                                                  const double Lc[8][8], double vn, double Rc[8][8]) {
    // group labels: smallest index reachable through chains of close eigenvalues
    int lab[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) lab[k] = k;
#pragma unroll 1
    for (int it = 0; it < 7; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int l = lab[k];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (fabs(lam[k] - lam[j]) <= GROUP_TOL && lab[j] < l) l = lab[j];
            lab[k] = l;
        }
    }
    int labc = lab[0];
    {
        double e = fabs(lam[0] - vn);
#pragma unroll
        for (int k = 1; k < 8; ++k)
            if (fabs(lam[k] - vn) < e) { e = fabs(lam[k] - vn); labc = lab[k]; }
    }
    // seed coefficients C[a][s] = z_a . (L^{-1} e_s) and |L^{-1} e_s|
    double C[8][8], yn[8];
#pragma unroll
    for (int sd = 0; sd < 8; ++sd) {
        double li[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double v = i == sd ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) v -= Lc[i][k] * li[k];
            li[i] = v / Lc[i][i];
        }
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) q += li[i] * li[i];
        yn[sd] = sqrt(q);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            double c = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) c += Zv[i][a] * li[i];
            C[a][sd] = c;
        }
    }
    // R = L Z in place (row i of R needs rows 0..i of Z)
#pragma unroll
    for (int i = 7; i >= 0; --i)
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k <= i; ++k) sum += Lc[i][k] * Zv[k][a];
            Zv[i][a] = sum;
        }
    // Gram-Schmidt in the coordinates of the orthonormal z_a: at slot t every group
    // projects its seed of slot t (e_D, e_{B_n}, e_1, ... for the group of v_n; e_t
    // for the others), removes the components along its members accepted so far,
    // and gives the remainder, normalised, to its next member when it exceeds
    // SEED_TOL |L^{-1} e_s| (the groups have disjoint supports, so they proceed
    // side by side).  W[k] holds the coordinates of the basis vector of position k.
    constexpr int SC[8] = {0, 5, 1, 2, 3, 4, 6, 7};
    double W[8][8];
    bool acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        acc[k] = false;
#pragma unroll
        for (int a = 0; a < 8; ++a) W[k][a] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        double r[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) r[a] = lab[a] == labc ? C[a][SC[t]] : C[a][t];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (!acc[k]) continue;
            double ip = 0.0;
#pragma unroll
            for (int a = 0; a < 8; ++a) ip += W[k][a] * r[a];
#pragma unroll
            for (int a = 0; a < 8; ++a) r[a] -= ip * W[k][a];
        }
        bool placed[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) placed[k] = acc[k];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (acc[k]) continue;
            // k may take this slot when all earlier members of its group were placed
            // at earlier slots (one member per group and slot)
            bool next = true;
#pragma unroll
            for (int j = 0; j < k; ++j)
                if (lab[j] == lab[k] && !placed[j]) next = false;
            if (!next) continue;
            double nn = 0.0;
#pragma unroll
            for (int a = 0; a < 8; ++a) nn += lab[a] == lab[k] ? r[a] * r[a] : 0.0;
            nn = sqrt(nn);
            const double ys = lab[k] == labc ? yn[SC[t]] : yn[t];
            if (nn > SEED_TOL * ys) {
                const double inn = 1.0 / nn;
#pragma unroll
                for (int a = 0; a < 8; ++a) W[k][a] = lab[a] == lab[k] ? r[a] * inn : 0.0;
                acc[k] = true;
            }
        }
    }
    // columns of R for the canonical basis: R_c[k] = R W[k]
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double sum = 0.0;
#pragma unroll
            for (int a = 0; a < 8; ++a) sum += Zv[i][a] * W[k][a];
            Rc[k][i] = sum;
        }
}

// Face frame and eigen-structure of the RMHD dissipation at face i+1/2 (shared by
// face_diss_rmhd and its adjoint): the rotation T of the face metric normal, the
// rotated entropy variables TV2, TV3 of nodes i and i+1, lambda^ and the columns
// Rc[k] = L z_k of R (z_k the canonical basis vector of position k).
// Frame of face i+1/2: the rotation T of the mean metric normal (a_t, L n) of
// nodes i and i+1 and their rotated entropy variables TV2, TV3.
template <int DIM>
__device__ __forceinline__ void face_frame_rmhd(double G, const double* P2, const double* P3, const double* al,
                                                const double* ar, double T[3][3], double* TV2, double* TV3,
                                                double& at, double& L) {
    at = 0.5 * (al[0] + ar[0]);
    double ax[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < DIM; ++j) ax[j] = 0.5 * (al[1 + j] + ar[1 + j]);
    L = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    const double iL = 1.0 / L;
    double nrm[3] = {ax[0] * iL, ax[1] * iL, ax[2] * iL};
    rotation<3>(nrm, T);            // n_3 = 0 in 2D gives the 2D rotation
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const StateRMHD<double> s = rmhd_state<double>(G, q == 0 ? P2 : P3);
        double V[8];
        rmhd_entropy_vars<double>(G, s, V);
        rotate8<false>(T, V, q == 0 ? TV2 : TV3);
    }
}

template <int DIM>
__device__ __forceinline__ void face_eigen_rmhd(double G, const double* P2, const double* P3, const double* al,
                                                const double* ar, double T[3][3], double* TV2, double* TV3,
                                                double& lhat, double Rc[8][8]) {
    double at, L;
    face_frame_rmhd<DIM>(G, P2, P3, al, ar, T, TV2, TV3, at, L);
    // face state (rotated frame)
    double Vb[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) Vb[c] = 0.5 * (TV2[c] + TV3[c]);
    const double vu2 = Vb[1] * Vb[1] + Vb[2] * Vb[2] + Vb[3] * Vb[3];
    const double beta = sqrt(Vb[4] * Vb[4] - vu2);
    const double ib = 1.0 / beta;
    double Pf[8];
    const double W = -Vb[4] * ib;
    const double rho = exp(Vb[0] - G / (G - 1.0) - log(beta) / (G - 1.0) - beta);
    Pf[0] = rho;
    Pf[4] = rho * ib;
    double u[3], b[3], ub = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) { u[k] = Vb[1 + k] * ib; b[k] = Vb[5 + k] * ib; ub += u[k] * b[k]; }
    const double b0 = ub / W;
#pragma unroll
    for (int k = 0; k < 3; ++k) { Pf[1 + k] = u[k]; Pf[5 + k] = W * b[k] - b0 * u[k]; }
    const double vn = u[0] / W;

    double JU[8][8], JF[8][8], JV[8][8], Pp[8], Lc[8][8], Q[8][8], Zv[8][8];
    rmhd_jacobians(G, Pf, JU, JF, JV, Pp);
    rmhd_pencil(JU, JF, JV, Lc, Q);
    double lam[8];
    jacobi_eigen_sym8(Q, lam, Zv);
    lhat = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) lhat = fmax(lhat, fabs(at + L * lam[k]));
    // canonical basis in every group of (nearly) equal eigenvalues
    canonical_columns(lam, Zv, Lc, vn, Rc);
}

// ES dissipation for RMHD at one face (eq. ESFlux_HO): as face_diss_rhd with
// T = diag{1, T_0, 1, T_0}, the face state from the mean rotated entropy
// variables (explicit inverse of V: beta^2 = V_5^2 - |V_2..4|^2, u = V_2..4/beta,
// W = -V_5/beta, ln rho = V_1 - G/(G-1) - ln(beta)/(G-1) - beta, p = rho/beta,
// b = V_6..8/beta, b^0 = u.b/W, B = W b - b^0 u), and R from the symmetric pencil
// (A0, S) of the Godunov-Powell modified Jacobian, with the canonical basis in
// every group of nearly equal eigenvalues (canonical_columns; the group of v_n
// holds the entropy and div B waves and is seeded with e_D, e_{B_n}).
// nodes: the 8 primitive slots of the stencil nodes i-2..i+3.
// P: the order parameter p (stencil of 2p nodes i-p+1 .. i+p, WENO of order 2p-1).
template <int DIM, bool MIXED = false, int P = 3>
__device__ __forceinline__ void face_diss_rmhd(double G, double eps, const double Pn[2 * P][8],
                                               const double* al, const double* ar, double* d) {
    constexpr int NS = 2 * P, CI = P - 1;    // stencil size, index of node i
    double T[3][3], TV[NS][8], lhat, Rc[8][8];
    face_eigen_rmhd<DIM>(G, Pn[CI], Pn[CI + 1], al, ar, T, TV[CI], TV[CI + 1], lhat, Rc);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if (j == CI || j == CI + 1) continue;
        const StateRMHD<double> s = rmhd_state<double>(G, Pn[j]);
        double V[8];
        rmhd_entropy_vars<double>(G, s, V);
        rotate8<false>(T, V, TV[j]);
    }
    double tv2 = 0.0, tv3 = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) { tv2 = fmax(tv2, fabs(TV[CI][c])); tv3 = fmax(tv3, fabs(TV[CI + 1][c])); }
    const double tvmax = tv2 + tv3;
    // projections, WENO5, the switch and the accumulation: FP64, or FP32 in the
    // mixed form (the eigen-structure above stays FP64 there)
    using RW = typename std::conditional<MIXED, float, double>::type;
    RW TVw[NS][8];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int c = 0; c < 8; ++c) TVw[j][c] = (RW)TV[j][c];
    RW dd[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) dd[c] = RW(0.0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        RW r[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) r[i] = (RW)Rc[k][i];
        RW vt[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            RW s = RW(0.0);
#pragma unroll
            for (int c = 0; c < 8; ++c) s += r[c] * TVw[j][c];
            vt[j] = s;
        }
        RW jw;
        if (P == 4)
            jw = weno7(vt[7], vt[6], vt[5], vt[4], vt[3], vt[2], vt[1], (RW)eps) -
                 weno7(vt[0], vt[1], vt[2], vt[3], vt[4], vt[5], vt[6], (RW)eps);
        else if (P == 3)
            jw = weno5(vt[5], vt[4], vt[3], vt[2], vt[1], (RW)eps) - weno5(vt[0], vt[1], vt[2], vt[3], vt[4], (RW)eps);
        else
            jw = weno3(vt[3], vt[2], vt[1], (RW)eps) - weno3(vt[0], vt[1], vt[2], (RW)eps);
        const RW jp = vt[CI + 1] - vt[CI];
        RW r1 = RW(0.0);
#pragma unroll
        for (int c = 0; c < 8; ++c) r1 += fabs(r[c]);
        if (jw * jp > RW(0.0) && fabs(jp) > RealTraits<RW>::ytol * r1 * (RW)tvmax) {
#pragma unroll
            for (int c = 0; c < 8; ++c) dd[c] += jw * r[c];
        }
    }
    double ddd[8], o[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) ddd[c] = (double)dd[c];
    rotate8<true>(T, ddd, o);
#pragma unroll
    for (int c = 0; c < 8; ++c) d[c] = lhat * o[c];
}

}  // namespace es
