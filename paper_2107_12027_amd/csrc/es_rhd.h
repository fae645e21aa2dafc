// Device physics of the RHD system (B = 0): logarithmic mean, two-point EC
// pair flux, conservative-to-primitive recovery and the entropy-stable face
// dissipation with closed-form scaled eigenvectors.
#pragma once

#include "es_common.h"

namespace es {

constexpr double Y_TOL = 1e-10;

// Reciprocal of a finite, nonzero, normal x: the hardware estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r), each of which squares the relative
// error, so the result is within about one ulp of 1/x.  Zero, infinities and
// denormals are not handled (NaN propagates); the callers pass state quantities.
__device__ __forceinline__ double frcp(double x) {
#ifdef ES_OPCOUNT_HOST
    return 1.0 / x;
#else
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#endif
}

// Logarithmic mean [a]/[ln a] (cited in Section 3.1 to Ismail & Roe) from the
// values and their precomputed logarithms.  With f = (al - ar)/(al + ar) and
// u = f^2: for u < 1e-2 the ratio ln(al/ar)/(2f) is replaced by its series
// sum_{k=0}^{7} u^k/(2k+1) (truncation below 1e-17); otherwise [a]/[ln a].
__device__ __forceinline__ double log_mean(double al, double ar, double lnal, double lnar) {
    const double s = al + ar;
    const double dif = al - ar;
    if (dif * dif < 1e-2 * (s * s)) {
        const double f = dif * frcp(s);
        const double u = f * f;
        double F = 1.0 / 15.0;
        F = fma(F, u, 1.0 / 13.0);
        F = fma(F, u, 1.0 / 11.0);
        F = fma(F, u, 1.0 / 9.0);
        F = fma(F, u, 1.0 / 7.0);
        F = fma(F, u, 1.0 / 5.0);
        F = fma(F, u, 1.0 / 3.0);
        F = fma(F, u, 1.0);
        return 0.5 * s * frcp(F);
    }
    return dif * frcp(lnal - lnar);
}

template <int NU>
struct NodeRHD {
    double rho, p, beta, W, lr, lb;
    double u[NU];
};

// Two-point EC flux in direction k (eq. ECFluxCurv, eq. UFcircle) for RHD:
// F = a_t U~ + sum_j a_j F~_j with a = (a_l + a_r)/2 and the RHD pair
//   U~_1 = rho^ln {W},  U~_E = ({W} a0 U~_1 + {rho}/{beta} |{u}|^2) / ({W}^2 - |{u}|^2),
//   U~_m = {u} (U~_E + {rho}/{beta}) / {W},
//   F~_j = ({u_j} rho^ln, {u} C {u_j}/{W} + e_j {rho}/{beta}, C {u_j}),
//   C = {W} (a0 rho^ln + {rho}/{beta}) / ({W}^2 - |{u}|^2),  a0 = 1 + 1/((Gamma-1) beta^ln),
// the solution of [V].U~ = [phi], [V].F~_j = [psi_j] with phi = rho W, psi_j = rho u_j.
// Also returns the VCL pair value a_t (eq. MetricsFlux_O2).
template <int NU>
__device__ __forceinline__ void pair_flux_rhd(double G, const NodeRHD<NU>& l, const NodeRHD<NU>& r,
                                              const double* al, const double* ar, double* F,
                                              double& Jt) {
    const double rho_ln = log_mean(l.rho, r.rho, l.lr, r.lr);
    const double beta_ln = log_mean(l.beta, r.beta, l.lb, r.lb);
    const double rho_m = 0.5 * (l.rho + r.rho);
    const double beta_m = 0.5 * (l.beta + r.beta);
    const double W_m = 0.5 * (l.W + r.W);
    double um[NU];
    double uu = 0.0, un = 0.0;
    const double at = 0.5 * (al[0] + ar[0]);
    double ab[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        um[k] = 0.5 * (l.u[k] + r.u[k]);
        ab[k] = 0.5 * (al[1 + k] + ar[1 + k]);
        uu += um[k] * um[k];
        un += ab[k] * um[k];
    }
    const double a0 = 1.0 + frcp((G - 1.0) * beta_ln);
    const double iden = frcp(W_m * W_m - uu);
    const double pb = rho_m * frcp(beta_m);
    const double U1 = rho_ln * W_m;
    const double U5 = (a0 * U1 * W_m + pb * uu) * iden;
    const double C = W_m * (a0 * rho_ln + pb) * iden;
    F[0] = rho_ln * (at * W_m + un);
    const double s = (at * (U5 + pb) + C * un) * frcp(W_m);
#pragma unroll
    for (int k = 0; k < NU; ++k) F[1 + k] = um[k] * s + ab[k] * pb;
    F[NU + 1] = at * U5 + C * un;
    Jt = at;
}

// Conservative -> primitive for RHD (Section 1: a scalar nonlinear equation).
// Safeguarded Newton on g(p) = (G-1)[(E+p)(1-v^2) - p - D sqrt(1-v^2)] - p,
// v = |m|/(E+p), g'(p) = (G-1) v^2 (1 - D W/(E+p)) - 1 < 0; the root lies in
// (0, (G-1)E] for admissible states D > 0, E > sqrt(D^2 + |m|^2).
// The iteration starts from ``guess`` when it lies inside the bracket, else
// from the bracket midpoint.  Returns 0 on success, 1 for an inadmissible state,
// 2 without convergence.
template <int NU>
__device__ __forceinline__ int c2p_rhd(double G, double D, const double* m, double E, double guess,
                                       double& rho, double* u, double& p) {
    double mm2 = 0.0;
#pragma unroll
    for (int k = 0; k < NU; ++k) mm2 += m[k] * m[k];
    if (!(D > 0.0) || !(E > sqrt(D * D + mm2))) return 1;
    double lo = 0.0, hi = (G - 1.0) * E;
    double pk = (guess > lo && guess < hi) ? guess : 0.5 * (lo + hi);
    int conv = 0;
    for (int it = 0; it < 200; ++it) {
        const double Ep = E + pk;
        const double v2 = mm2 / (Ep * Ep);
        const double sq = sqrt(1.0 - v2);
        const double gv = (G - 1.0) * (Ep * (1.0 - v2) - pk - D * sq) - pk;
        if (gv == 0.0) { conv = 1; break; }
        if (gv > 0.0) lo = pk; else hi = pk;
        const double dg = (G - 1.0) * v2 * (1.0 - D / (sq * Ep)) - 1.0;
        double pn = pk - gv / dg;
        // Newton step while it stays in the bracket (end points included), else bisection
        if (!(pn >= lo && pn <= hi)) pn = 0.5 * (lo + hi);
        const double dp = fabs(pn - pk);
        pk = pn;
        // g is evaluated from terms of size ~(E + p): the root is fixed only to
        // ~eps (E + p), so the steps are measured against that scale
        if (dp <= 1e-15 * (E + pn) || hi - lo <= 1e-15 * (E + hi)) { conv = 1; break; }
    }
    // one more Newton correction from the converged iterate
    {
        const double Ep = E + pk;
        const double v2 = mm2 / (Ep * Ep);
        const double sq = sqrt(1.0 - v2);
        const double gv = (G - 1.0) * (Ep * (1.0 - v2) - pk - D * sq) - pk;
        const double dg = (G - 1.0) * v2 * (1.0 - D / (sq * Ep)) - 1.0;
        const double pn = pk - gv / dg;
        if (pn > 0.0) pk = pn;
    }
    p = pk;
    const double iEp = 1.0 / (E + pk);
    double v2 = 0.0;
    double v[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) { v[k] = m[k] * iEp; v2 += v[k] * v[k]; }
    const double W = 1.0 / sqrt(1.0 - v2);
    rho = D / W;
#pragma unroll
    for (int k = 0; k < NU; ++k) u[k] = W * v[k];
    return conv ? 0 : 2;
}

// WENO5-JS value at i+1/2 from point values v_{i-2..i+2} = (a, b, c, d, e).
// The weights d_k/(eps + b_k)^2 are multiplied through by prod_k (eps + b_k)^2,
// which leaves their ratios unchanged and needs a single reciprocal; with
// eps = 1e-6 the products stay far inside the FP64 range.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e, double eps) {
    const double q0 = 2.0 * a - 7.0 * b + 11.0 * c;      // 6 x candidate values
    const double q1 = -b + 5.0 * c + 2.0 * d;
    const double q2 = 2.0 * c + 5.0 * d - e;
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = b - d;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double b0 = 13.0 / 12.0 * t0 * t0 + 0.25 * s0 * s0;
    const double b1 = 13.0 / 12.0 * t1 * t1 + 0.25 * s1 * s1;
    const double b2 = 13.0 / 12.0 * t2 * t2 + 0.25 * s2 * s2;
    const double e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
    const double f0 = e0 * e0, f1 = e1 * e1, f2 = e2 * e2;
    const double w0 = 0.1 * (f1 * f2);
    const double w1 = 0.6 * (f0 * f2);
    const double w2 = 0.3 * (f0 * f1);
    return (w0 * q0 + w1 * q1 + w2 * q2) * frcp(6.0 * (w0 + w1 + w2));
}

// Face state in the rotated frame with the reciprocals the tangent map reuses.
template <int DIM>
struct FaceRHD {
    double rho, irho, p, ip, beta, W, h, v[DIM];
};

// Tangent map of the primitive state P = (rho, v, p) (rotated frame, DIM velocity
// components): dU = (dU/dP) dP and dV = (dV/dP) dP, U = (rho W, rho h W^2 v,
// rho h W^2 - p), V = (G/(G-1) + ln rho + ln beta/(G-1) + beta, beta W v, -beta W);
// c0 = G/(G-1), c1 = 1/(G-1).
template <int DIM>
__device__ __forceinline__ void tangent_rhd(double c0, double c1, const FaceRHD<DIM>& f,
                                            double drho, const double* dv, double dp, double* dU,
                                            double* dV) {
    constexpr int M = DIM + 2;
    const double W = f.W;
    double vdv = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) vdv += f.v[k] * dv[k];
    const double dW = W * W * W * vdv;
    const double dh = c0 * (dp - f.p * drho * f.irho) * f.irho;
    const double W2 = W * W;
    const double Z = f.rho * f.h * W2;
    const double dZ = (drho * f.h + f.rho * dh) * W2 + 2.0 * f.rho * f.h * W * dW;
    dU[0] = drho * W + f.rho * dW;
#pragma unroll
    for (int k = 0; k < DIM; ++k) dU[1 + k] = dZ * f.v[k] + Z * dv[k];
    dU[M - 1] = dZ - dp;
    const double dbeta = (drho - f.beta * dp) * f.ip;
    dV[0] = drho * f.irho + dbeta * (c1 * f.p * f.irho) + dbeta;
    const double dbW = dbeta * W + f.beta * dW;
#pragma unroll
    for (int k = 0; k < DIM; ++k) dV[1 + k] = dbW * f.v[k] + f.beta * W * dv[k];
    dV[M - 1] = -dbW;
}

// Rotation T_0 with first row n (Section 4), read with atan2 semantics:
// row 2 = (-n2, n1, 0)/rho_perp, row 3 = (-n3 n1/rho_perp, -n3 n2/rho_perp, rho_perp),
// rho_perp = sqrt(n1^2 + n2^2); rows (0,1,0), (-n3,0,0) when rho_perp = 0.
template <int DIM>
__device__ __forceinline__ void rotation(const double* n, double T[3][3]) {
    if (DIM == 2) {
        T[0][0] = n[0]; T[0][1] = n[1]; T[0][2] = 0.0;
        T[1][0] = -n[1]; T[1][1] = n[0]; T[1][2] = 0.0;
        T[2][0] = 0.0; T[2][1] = 0.0; T[2][2] = 1.0;
        return;
    }
    const double rp = sqrt(n[0] * n[0] + n[1] * n[1]);
    T[0][0] = n[0]; T[0][1] = n[1]; T[0][2] = n[2];
    if (rp > 0.0) {
        const double ir = frcp(rp);
        T[1][0] = -n[1] * ir; T[1][1] = n[0] * ir; T[1][2] = 0.0;
        T[2][0] = -n[2] * n[0] * ir; T[2][1] = -n[2] * n[1] * ir; T[2][2] = rp;
    } else {
        T[1][0] = 0.0; T[1][1] = 1.0; T[1][2] = 0.0;
        T[2][0] = -n[2]; T[2][1] = 0.0; T[2][2] = 0.0;
    }
}

// Entropy-stable dissipation d = lambda^ T^{-1} R Y <<V~>> at one face
// (eq. ESFlux_HO).  nd[0..5] are the stencil nodes i-2..i+3 of the face
// i+1/2; al, ar the metric vectors (a_t, a_1..a_d) of nodes i and i+1.
//  * face state: the state whose entropy variables are the mean of those of
//    nodes i and i+1 (A0 at that state turns [V] into the midpoint rule for [U]);
//    face metrics: arithmetic mean (readings of this build);
//  * lambda^ = max |a_t + L lambda_m|, lambda_+- closed form, lambda_0 = v_n;
//  * R: acoustic columns from the primitive eigenvector (scaled by lambda - v_n)
//      dp = lambda - v_n, drho = dp/(h c^2), dv_n = (1 - v_n lambda)/(rho h W^2),
//      dv_t = -v_t (dh + h W^2 v_n dv_n)/(h (1 + W^2 |v_t|^2))   [d(h W v_t) = 0],
//    normalised by sqrt(dU.dV) so that R R^T = dU/dV; the v_n cluster
//    (basis e_rho, e_vt) is replaced by its canonical A0^{-1}-orthonormal basis
//    from the cluster projector applied to the seeds e_D, e_{m_t1}(, e_{m_t2}),
//    computed in the coefficient space of the cluster basis with the Gram
//    matrix G_ab = dU_a . dV_b;
//  * WENO5-JS of V~ = R^T T V on both sides, Y_l = [<<V~_l>> [V~_l] > 0], with a
//    jump [V~_l] below Y_TOL |r_l|_1 (|T V_i|_max + |T V_i+1|_max) counted as
//    zero (sign(0) at rounding level).
template <int DIM>
__device__ __forceinline__ void face_diss_rhd(double G, double eps, const NodeRHD<DIM>* nd,
                                              const double* al, const double* ar, double* d) {
    constexpr int M = DIM + 2;
    constexpr int NC = DIM;          // cluster size (entropy + transverse shear waves)
    const double at = 0.5 * (al[0] + ar[0]);
    double ax[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < DIM; ++j) ax[j] = 0.5 * (al[1 + j] + ar[1 + j]);
    const double L = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    const double iL = frcp(L);
    double nrm[3] = {ax[0] * iL, ax[1] * iL, ax[2] * iL};
    double T[3][3];
    rotation<DIM>(nrm, T);

    // rotated entropy variables T V of the six stencil nodes
    double TV[6][M];
    const double c0 = G / (G - 1.0), c1 = 1.0 / (G - 1.0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const NodeRHD<DIM>& q = nd[j];
        TV[j][0] = c0 + q.lr + q.lb * c1 + q.beta;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) s += T[a][b] * q.u[b];
            TV[j][1 + a] = q.beta * s;
        }
        TV[j][M - 1] = -q.beta * q.W;
    }

    // face state in the rotated frame: the state whose entropy variables are the
    // mean of those of nodes i and i+1 (beta^2 = V_E^2 - |V_u|^2, u = V_u/beta,
    // W = -V_E/beta, ln rho = V_1 - G/(G-1) - ln(beta)/(G-1) - beta, p = rho/beta)
    double Vb[M];
#pragma unroll
    for (int c = 0; c < M; ++c) Vb[c] = 0.5 * (TV[2][c] + TV[3][c]);
    double vu2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) vu2 += Vb[1 + a] * Vb[1 + a];
    const double beta_f = sqrt(Vb[M - 1] * Vb[M - 1] - vu2);
    const double ib = frcp(beta_f);
    FaceRHD<DIM> fs;
    fs.beta = beta_f;
    fs.W = -Vb[M - 1] * ib;
    fs.rho = exp(Vb[0] - c0 - log(beta_f) * c1 - beta_f);
    fs.irho = frcp(fs.rho);
    fs.p = fs.rho * ib;
    fs.ip = beta_f * fs.irho;
    const double iVE = -frcp(Vb[M - 1]);      // 1/(beta W)
#pragma unroll
    for (int k = 0; k < DIM; ++k) fs.v[k] = Vb[1 + k] * iVE;
    const double rho = fs.rho, p = fs.p, W = fs.W;
    const double* v = fs.v;
    double v2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) v2 += v[k] * v[k];
    const double vn = v[0];
    // p/rho = 1/beta, so h = 1 + c0/beta and h cs^2 = G/beta
    const double h = 1.0 + c0 * ib;
    fs.h = h;
    const double cs2 = G * ib * frcp(h);
    const double cs = sqrt(cs2);
    const double disc = sqrt((1.0 - v2) * (1.0 - v2 * cs2 - vn * vn * (1.0 - cs2)));
    const double iden = frcp(1.0 - v2 * cs2);
    const double lam_m = (vn * (1.0 - cs2) - cs * disc) * iden;
    const double lam_p = (vn * (1.0 - cs2) + cs * disc) * iden;
    const double lhat = fmax(fabs(at + L * lam_m), fmax(fabs(at + L * vn), fabs(at + L * lam_p)));

    double dd[M];
#pragma unroll
    for (int c = 0; c < M; ++c) dd[c] = 0.0;
    // rounding scale of the projections r . T V at nodes i and i+1
    double tv2 = 0.0, tv3 = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) { tv2 = fmax(tv2, fabs(TV[2][c])); tv3 = fmax(tv3, fabs(TV[3][c])); }
    const double tvmax = tv2 + tv3;

    // one column r of R: project, reconstruct, switch, accumulate
    auto column = [&](const double* r) {
        double vt[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) s += r[c] * TV[j][c];
            vt[j] = s;
        }
        const double vm = weno5(vt[0], vt[1], vt[2], vt[3], vt[4], eps);
        const double vp = weno5(vt[5], vt[4], vt[3], vt[2], vt[1], eps);
        const double jw = vp - vm;
        const double jp = vt[3] - vt[2];
        // a jump within rounding of zero counts as zero (Y = 0)
        double r1 = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) r1 += fabs(r[c]);
        if (jw * jp > 0.0 && fabs(jp) > Y_TOL * r1 * tvmax) {
#pragma unroll
            for (int c = 0; c < M; ++c) dd[c] += jw * r[c];
        }
    };

    // acoustic columns
    const double hW2 = h * W * W;
    double vt2 = 0.0;
#pragma unroll
    for (int k = 1; k < DIM; ++k) vt2 += v[k] * v[k];
    const double i_rhW2 = frcp(rho * hW2);
    const double i_ht = frcp(h * (1.0 + W * W * vt2));
    const double ig = beta_f / G;                    // 1/(h cs^2)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double lam = s == 0 ? lam_m : lam_p;
        const double q = lam - vn;
        const double dp = q;
        const double drho = q * ig;
        double dv[DIM];
        dv[0] = (1.0 - vn * lam) * i_rhW2;
        const double dh = c0 * (dp - p * drho * fs.irho) * fs.irho;
        const double fac = -(dh + hW2 * vn * dv[0]) * i_ht;
#pragma unroll
        for (int k = 1; k < DIM; ++k) dv[k] = v[k] * fac;
        double dU[M], dV[M];
        tangent_rhd<DIM>(c0, c1, fs, drho, dv, dp, dU, dV);
        double nn = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) nn += dU[c] * dV[c];
        const double sc = frcp(sqrt(nn));
#pragma unroll
        for (int c = 0; c < M; ++c) dU[c] *= sc;
        column(dU);
    }

    // v_n cluster: basis e_rho, e_{v_t1}(, e_{v_t2}) in primitive variables
    double KU[NC][M], KV[NC][M];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        double dv[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) dv[k] = 0.0;
        double drho = 0.0;
        if (a == 0) drho = 1.0; else dv[a] = 1.0;
        tangent_rhd<DIM>(c0, c1, fs, drho, dv, 0.0, KU[a], KV[a]);
    }
    double Gm[NC][NC];
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            double s = 0.0, t = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) { s += KU[a][c] * KV[b][c]; t += KU[b][c] * KV[a][c]; }
            Gm[a][b] = 0.5 * (s + t);
        }
    double Gi[NC][NC];
    if (NC == 2) {
        const double det = Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0];
        const double id = frcp(det);
        Gi[0][0] = Gm[1][1] * id; Gi[1][1] = Gm[0][0] * id;
        Gi[0][1] = -Gm[0][1] * id; Gi[1][0] = -Gm[1][0] * id;
    } else {
        const double c00 = Gm[1][1] * Gm[2][2] - Gm[1][2] * Gm[2][1];
        const double c01 = Gm[1][2] * Gm[2][0] - Gm[1][0] * Gm[2][2];
        const double c02 = Gm[1][0] * Gm[2][1] - Gm[1][1] * Gm[2][0];
        const double det = Gm[0][0] * c00 + Gm[0][1] * c01 + Gm[0][2] * c02;
        const double id = frcp(det);
        Gi[0][0] = c00 * id;
        Gi[0][1] = (Gm[0][2] * Gm[2][1] - Gm[0][1] * Gm[2][2]) * id;
        Gi[0][2] = (Gm[0][1] * Gm[1][2] - Gm[0][2] * Gm[1][1]) * id;
        Gi[1][0] = c01 * id;
        Gi[1][1] = (Gm[0][0] * Gm[2][2] - Gm[0][2] * Gm[2][0]) * id;
        Gi[1][2] = (Gm[0][2] * Gm[1][0] - Gm[0][0] * Gm[1][2]) * id;
        Gi[2][0] = c02 * id;
        Gi[2][1] = (Gm[0][1] * Gm[2][0] - Gm[0][0] * Gm[2][1]) * id;
        Gi[2][2] = (Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0]) * id;
    }
    // seeds: D slot 0, transverse momentum slots 2 (and 3)
    double cf[NC][NC];     // coefficient vectors of the canonical columns
    double inq[NC];        // reciprocals of their squared A0^{-1} norms
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int seed = q == 0 ? 0 : 1 + q;
        double gs[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) gs[a] = KV[a][seed];
        double cq[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < NC; ++b) s += Gi[a][b] * gs[b];
            cq[a] = s;
        }
#pragma unroll
        for (int r = 0; r < q; ++r) {
            double ip = 0.0;
#pragma unroll
            for (int a = 0; a < NC; ++a) ip += cf[r][a] * gs[a];
            const double f = ip * inq[r];
#pragma unroll
            for (int a = 0; a < NC; ++a) cq[a] -= f * cf[r][a];
        }
        double nn = 0.0;
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) nn += cq[a] * Gm[a][b] * cq[b];
#pragma unroll
        for (int a = 0; a < NC; ++a) cf[q][a] = cq[a];
        const double rn = frcp(sqrt(nn));
        inq[q] = rn * rn;
        const double sc = rn;
        double r[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < NC; ++a) s += cq[a] * KU[a][c];
            r[c] = s * sc;
        }
        column(r);
    }

    // back to the original frame: d = lambda^ T^{-1} (R Y <<V~>>)
    d[0] = lhat * dd[0];
    d[M - 1] = lhat * dd[M - 1];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) s += T[b][a] * dd[1 + b];
        d[1 + a] = lhat * s;
    }
}

}  // namespace es
