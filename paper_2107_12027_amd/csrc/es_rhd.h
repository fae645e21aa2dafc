// Device physics of the RHD system (B = 0): logarithmic mean, two-point EC
// pair flux, conservative-to-primitive recovery and the entropy-stable face
// dissipation with closed-form scaled eigenvectors.
#pragma once

#include "es_common.h"

namespace es {

// Per-precision constants of the face dissipation: the rounding level below which
// a jump of a characteristic variable counts as zero in the sign switch Y
// (relative to |r_l|_1 (|T V_i|_max + |T V_i+1|_max)).
template <typename R>
struct RealTraits;
template <>
struct RealTraits<double> {
    static constexpr double ytol = 1e-10;
    static constexpr bool wide_range = true;     // exponent range for WENO's common denominator
};

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

// a / b as a times the reciprocal of b (frcp; the same conditions on b).  The op
// count takes it as the one division it stands for.
__device__ __forceinline__ double fdiv(double a, double b) {
#ifdef ES_OPCOUNT_HOST
    return a / b;
#else
    return a * frcp(b);
#endif
}

// Logarithmic mean [a]/[ln a] (cited in Section 3.1 to Ismail & Roe) from the
// values and their precomputed logarithms.  With f = (al - ar)/(al + ar) and
// u = f^2: for u < 1e-2 the ratio ln(al/ar)/(2f) is replaced by its series
// sum_{k=0}^{7} u^k/(2k+1) (truncation below 1e-17); otherwise [a]/[ln a].
__device__ __forceinline__ double xsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ double xexp(double x) { return exp(x); }
__device__ __forceinline__ double xlog(double x) { return log(x); }

// Reciprocal square root and square root of a positive, normal x (state and
// metric quantities that are positive by construction): the hardware estimate
// of 1/sqrt(x) refined by two Newton steps r <- r + r (1/2 - x r^2/2), each of
// which squares the relative error, and for the root s = x r with one
// correction s <- s + (x - s^2) r/2.  Unlike the general square root there is
// no rescaling for denormal or zero arguments (a zero gives NaN), which saves
// the range checks and two scalings per call.
__device__ __forceinline__ double frsqrt(double x) {
#ifdef ES_OPCOUNT_HOST
    return 1.0 / sqrt(x);
#else
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    double e = fma(-hx * r, r, 0.5);
    r = fma(r, e, r);
    e = fma(-hx * r, r, 0.5);
    return fma(r, e, r);
#endif
}
__device__ __forceinline__ double psqrt(double x) {
#ifdef ES_OPCOUNT_HOST
    return sqrt(x);
#else
    const double r = frsqrt(x);
    const double s = x * r;
    return fma(fma(-s, s, x), 0.5 * r, s);
#endif
}

#ifndef ES_OPCOUNT_HOST
// FP32 arithmetic of the mixed form: the hardware reciprocal, exp2 and log2
// (about one ulp), a correctly rounded square root.
template <>
struct RealTraits<float> {
    static constexpr float ytol = 1e-6f;
    static constexpr bool wide_range = false;
};
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float xsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ float xexp(float x) { return __expf(x); }
__device__ __forceinline__ float xlog(float x) { return __logf(x); }
__device__ __forceinline__ float frsqrt(float x) { return frcp(xsqrt(x)); }
__device__ __forceinline__ float psqrt(float x) { return xsqrt(x); }
#endif

template <typename R>
__device__ __forceinline__ R log_mean(R al, R ar, R lnal, R lnar) {
    const R s = al + ar;
    const R dif = al - ar;
    if (dif * dif < 1e-2 * (s * s)) {
        const R f = dif * frcp(s);
        const R u = f * f;
        R F = R(1.0 / 15.0);
        F = fma(F, u, R(1.0 / 13.0));
        F = fma(F, u, R(1.0 / 11.0));
        F = fma(F, u, R(1.0 / 9.0));
        F = fma(F, u, R(1.0 / 7.0));
        F = fma(F, u, R(1.0 / 5.0));
        F = fma(F, u, R(1.0 / 3.0));
        F = fma(F, u, R(1.0));
        return 0.5 * s * frcp(F);
    }
    return dif * frcp(lnal - lnar);
}

template <int NU, typename R = double>
struct NodeRHD {
    R rho, p, beta, W, lr, lb;
    R u[NU];
};

// Two-point EC flux in direction k (eq. ECFluxCurv, eq. UFcircle) for RHD:
// F = a_t U~ + sum_j a_j F~_j with a = (a_l + a_r)/2 and the RHD pair
//   U~_1 = rho^ln {W},  U~_E = ({W} a0 U~_1 + {rho}/{beta} |{u}|^2) / ({W}^2 - |{u}|^2),
//   U~_m = {u} (U~_E + {rho}/{beta}) / {W},
//   F~_j = ({u_j} rho^ln, {u} C {u_j}/{W} + e_j {rho}/{beta}, C {u_j}),
//   C = {W} (a0 rho^ln + {rho}/{beta}) / ({W}^2 - |{u}|^2),  a0 = 1 + 1/((Gamma-1) beta^ln),
// the solution of [V].U~ = [phi], [V].F~_j = [psi_j] with phi = rho W, psi_j = rho u_j.
// Also returns the VCL pair value a_t (eq. MetricsFlux_O2).
template <int NU, typename R>
__device__ __forceinline__ void pair_flux_rhd(double G, const NodeRHD<NU, R>& l, const NodeRHD<NU, R>& r,
                                              const double* al, const double* ar, R* F,
                                              double& Jt) {
    const R rho_ln = log_mean(l.rho, r.rho, l.lr, r.lr);
    const R beta_ln = log_mean(l.beta, r.beta, l.lb, r.lb);
    const R rho_m = 0.5 * (l.rho + r.rho);
    const R beta_m = 0.5 * (l.beta + r.beta);
    const R W_m = 0.5 * (l.W + r.W);
    R um[NU];
    R uu = R(0.0), un = R(0.0);
    const double at = 0.5 * (al[0] + ar[0]);
    double ab[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        um[k] = 0.5 * (l.u[k] + r.u[k]);
        ab[k] = 0.5 * (al[1 + k] + ar[1 + k]);
        uu += um[k] * um[k];
        un += ab[k] * um[k];
    }
    const R a0 = 1.0 + frcp((G - 1.0) * beta_ln);
    const R iden = frcp(W_m * W_m - uu);
    const R pb = rho_m * frcp(beta_m);
    const R U1 = rho_ln * W_m;
    const R U5 = (a0 * U1 * W_m + pb * uu) * iden;
    const R C = W_m * (a0 * rho_ln + pb) * iden;
    F[0] = rho_ln * (at * W_m + un);
    const R s = (at * (U5 + pb) + C * un) * frcp(W_m);
#pragma unroll
    for (int k = 0; k < NU; ++k) F[1 + k] = um[k] * s + ab[k] * pb;
    F[NU + 1] = at * U5 + C * un;
    Jt = at;
}

#ifndef ES_OPCOUNT_HOST
// Mixed-precision form of pair_flux_rhd: the pair algebra (means, U~, F~_j) in
// FP32 except the small-jump branch of the logarithmic means, which stays FP64;
// the contraction with the metrics and the VCL value in FP64.  The FP32 part is
// written as coefficients K_t, K_j of a_t and a_j (F = a_t K_t + sum_j a_j K_j):
// equal states give equal coefficients for every pair, so the metric sums cancel
// in FP64 and a uniform flow stays uniform to FP64 rounding on any mesh that
// satisfies the discrete SCL and VCL.
__device__ __forceinline__ float log_mean_mixed(double al, double ar, double lnal, double lnar) {
    const double s = al + ar;
    const double dif = al - ar;
    if (dif * dif < 1e-2 * (s * s)) return (float)log_mean(al, ar, lnal, lnar);
    return (float)dif * frcp((float)lnal - (float)lnar);
}

template <int NU>
__device__ __forceinline__ void pair_flux_rhd_mixed(double G, const NodeRHD<NU>& l, const NodeRHD<NU>& r,
                                                    const double* al, const double* ar, double* F,
                                                    double& Jt) {
    constexpr int M = NU + 2;
    const float rho_ln = log_mean_mixed(l.rho, r.rho, l.lr, r.lr);
    const float beta_ln = log_mean_mixed(l.beta, r.beta, l.lb, r.lb);
    const float rho_m = 0.5f * ((float)l.rho + (float)r.rho);
    const float beta_m = 0.5f * ((float)l.beta + (float)r.beta);
    const float W_m = 0.5f * ((float)l.W + (float)r.W);
    float um[NU];
    float uu = 0.0f;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        um[k] = 0.5f * ((float)l.u[k] + (float)r.u[k]);
        uu += um[k] * um[k];
    }
    const float a0 = 1.0f + frcp((float)(G - 1.0) * beta_ln);
    const float iden = frcp(W_m * W_m - uu);
    const float pb = rho_m * frcp(beta_m);
    const float U1 = rho_ln * W_m;
    const float U5 = (a0 * U1 * W_m + pb * uu) * iden;
    const float C = W_m * (a0 * rho_ln + pb) * iden;
    const float iW = frcp(W_m);
    // coefficients of a_t (Kt) and a_j (Kj) per component
    float Kt[M], Kj[M][NU];
    Kt[0] = U1;
#pragma unroll
    for (int j = 0; j < NU; ++j) Kj[0][j] = rho_ln * um[j];
    const float sU = (U5 + pb) * iW, sC = C * iW;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        Kt[1 + k] = um[k] * sU;
#pragma unroll
        for (int j = 0; j < NU; ++j) Kj[1 + k][j] = um[k] * sC * um[j] + (j == k ? pb : 0.0f);
    }
    Kt[M - 1] = U5;
#pragma unroll
    for (int j = 0; j < NU; ++j) Kj[M - 1][j] = C * um[j];
    const double at = 0.5 * (al[0] + ar[0]);
    double ab[NU];
#pragma unroll
    for (int j = 0; j < NU; ++j) ab[j] = 0.5 * (al[1 + j] + ar[1 + j]);
#pragma unroll
    for (int c = 0; c < M; ++c) {
        double f = at * (double)Kt[c];
#pragma unroll
        for (int j = 0; j < NU; ++j) f += ab[j] * (double)Kj[c][j];
        F[c] = f;
    }
    Jt = at;
}
#endif

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
// In FP64 the weights d_k/(eps + b_k)^2 are multiplied through by
// prod_k (eps + b_k)^2, which leaves their ratios unchanged and needs a single
// reciprocal; with eps = 1e-6 the products stay far inside the FP64 range.
template <typename R>
__device__ __forceinline__ R weno5(R a, R b, R c, R d, R e, R eps) {
    const R q0 = R(2.0) * a - R(7.0) * b + R(11.0) * c;      // 6 x candidate values
    const R q1 = -b + R(5.0) * c + R(2.0) * d;
    const R q2 = R(2.0) * c + R(5.0) * d - e;
    const R t0 = a - R(2.0) * b + c, s0 = a - R(4.0) * b + R(3.0) * c;
    const R t1 = b - R(2.0) * c + d, s1 = b - d;
    const R t2 = c - R(2.0) * d + e, s2 = R(3.0) * c - R(4.0) * d + e;
    const R b0 = R(13.0 / 12.0) * t0 * t0 + R(0.25) * s0 * s0;
    const R b1 = R(13.0 / 12.0) * t1 * t1 + R(0.25) * s1 * s1;
    const R b2 = R(13.0 / 12.0) * t2 * t2 + R(0.25) * s2 * s2;
    const R e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
    const R f0 = e0 * e0, f1 = e1 * e1, f2 = e2 * e2;
    R w0, w1, w2;
    if (RealTraits<R>::wide_range) {
        w0 = R(0.1) * (f1 * f2);
        w1 = R(0.6) * (f0 * f2);
        w2 = R(0.3) * (f0 * f1);
    } else {
        // FP32: products of the f_k could overflow; the hardware reciprocal is cheap
        w0 = R(0.1) * frcp(f0);
        w1 = R(0.6) * frcp(f1);
        w2 = R(0.3) * frcp(f2);
    }
    return (w0 * q0 + w1 * q1 + w2 * q2) * frcp(R(6.0) * (w0 + w1 + w2));
}

// WENO7-JS value at i+1/2 from point values v_{i-3..i+3} = (a, b, c, d, e, f, h)
// (Balsara and Shu 2000): four candidates on four-node stencils and linear weights
// (1, 12, 18, 4)/35.  The smoothness indicator of the Jiang-Shu definition,
// sum_{l=1..3} int over the cell of (p_k^(l))^2, is evaluated from the Taylor
// coefficients c_1, c_2, c_3 of the candidate cubic at the cell centre as
//   beta_k = (c_1 + c_3/4)^2 + 13/3 c_2^2 + 781/20 c_3^2,
// a sum of squares of differences of v (the expanded quadratic form cancels
// terms larger than beta by the square of the data over its variation).  With
// u = 6 (c_1 + c_3/4), t2 = 2 c_2 and t3 = 6 c_3 (integer stencils):
//   beta_k = u^2/36 + 13/12 t2^2 + 781/720 t3^2.
// FP64: the weights d_k/(eps + b_k)^2 over a common denominator (one reciprocal)
// as in weno5; FP32: reciprocal weights.
template <typename R>
__device__ __forceinline__ R weno7(R a, R b, R c, R d, R e, R f, R h, R eps) {
    const R q0 = -R(3.0) * a + R(13.0) * b - R(23.0) * c + R(25.0) * d;    // 12 x candidate values
    const R q1 = b - R(5.0) * c + R(13.0) * d + R(3.0) * e;
    const R q2 = -c + R(7.0) * d + R(7.0) * e - f;
    const R q3 = R(3.0) * d + R(13.0) * e - R(5.0) * f + h;
    const R u0 = -R(2.0) * a + R(9.0) * b - R(18.0) * c + R(11.0) * d;
    const R u1 = b - R(6.0) * c + R(3.0) * d + R(2.0) * e;
    const R u2 = -R(2.0) * c - R(3.0) * d + R(6.0) * e - f;
    const R u3 = -R(11.0) * d + R(18.0) * e - R(9.0) * f + R(2.0) * h;
    const R s0 = -a + R(4.0) * b - R(5.0) * c + R(2.0) * d;
    const R s1 = c - R(2.0) * d + e;          // candidates 1 and 2 share t2
    const R s3 = R(2.0) * d - R(5.0) * e + R(4.0) * f - h;
    const R r0 = -a + R(3.0) * b - R(3.0) * c + d;
    const R r1 = -b + R(3.0) * c - R(3.0) * d + e;
    const R r2 = -c + R(3.0) * d - R(3.0) * e + f;
    const R r3 = -d + R(3.0) * e - R(3.0) * f + h;
    const R ku = R(1.0 / 36.0), k2 = R(13.0 / 12.0), k3 = R(781.0 / 720.0);
    const R b0 = ku * u0 * u0 + k2 * s0 * s0 + k3 * r0 * r0;
    const R b1 = ku * u1 * u1 + k2 * s1 * s1 + k3 * r1 * r1;
    const R b2 = ku * u2 * u2 + k2 * s1 * s1 + k3 * r2 * r2;
    const R b3 = ku * u3 * u3 + k2 * s3 * s3 + k3 * r3 * r3;
    const R e0 = eps + b0, e1 = eps + b1, e2 = eps + b2, e3 = eps + b3;
    const R f0 = e0 * e0, f1 = e1 * e1, f2 = e2 * e2, f3 = e3 * e3;
    R w0, w1, w2, w3;
    if (RealTraits<R>::wide_range) {
        const R f01 = f0 * f1, f23 = f2 * f3;
        w0 = R(1.0) * (f1 * f23);
        w1 = R(12.0) * (f0 * f23);
        w2 = R(18.0) * (f01 * f3);
        w3 = R(4.0) * (f01 * f2);
    } else {
        w0 = R(1.0) * frcp(f0);
        w1 = R(12.0) * frcp(f1);
        w2 = R(18.0) * frcp(f2);
        w3 = R(4.0) * frcp(f3);
    }
    return (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) * frcp(R(12.0) * (w0 + w1 + w2 + w3));
}

// WENO3-JS value at i+1/2 from v_{i-1..i+1} = (a, b, c): candidates (3b - a)/2 and
// (b + c)/2, linear weights 1/3 and 2/3, smoothness indicators (b - a)^2 and
// (c - b)^2; in FP64 over a common denominator as weno5.
template <typename R>
__device__ __forceinline__ R weno3(R a, R b, R c, R eps) {
    const R q0 = R(3.0) * b - a;          // 2 x candidate values
    const R q1 = b + c;
    const R e0 = eps + (b - a) * (b - a), e1 = eps + (c - b) * (c - b);
    const R f0 = e0 * e0, f1 = e1 * e1;
    R w0, w1;
    if (RealTraits<R>::wide_range) {
        w0 = R(1.0 / 3.0) * f1;
        w1 = R(2.0 / 3.0) * f0;
    } else {
        w0 = R(1.0 / 3.0) * frcp(f0);
        w1 = R(2.0 / 3.0) * frcp(f1);
    }
    return (w0 * q0 + w1 * q1) * frcp(R(2.0) * (w0 + w1));
}

// Face state in the rotated frame with the reciprocals the tangent map reuses.
template <int DIM, typename R = double>
struct FaceRHD {
    R rho, irho, p, ip, beta, W, h, v[DIM];
};

// Tangent map of the primitive state P = (rho, v, p) (rotated frame, DIM velocity
// components): dU = (dU/dP) dP and dV = (dV/dP) dP, U = (rho W, rho h W^2 v,
// rho h W^2 - p), V = (G/(G-1) + ln rho + ln beta/(G-1) + beta, beta W v, -beta W);
// c0 = G/(G-1), c1 = 1/(G-1).
template <int DIM, typename R>
__device__ __forceinline__ void tangent_rhd(R c0, R c1, const FaceRHD<DIM, R>& f,
                                            R drho, const R* dv, R dp, R* dU,
                                            R* dV) {
    constexpr int M = DIM + 2;
    const R W = f.W;
    R vdv = R(0.0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) vdv += f.v[k] * dv[k];
    const R dW = W * W * W * vdv;
    const R dh = c0 * (dp - f.p * drho * f.irho) * f.irho;
    const R W2 = W * W;
    const R Z = f.rho * f.h * W2;
    const R dZ = (drho * f.h + f.rho * dh) * W2 + R(2.0) * f.rho * f.h * W * dW;
    dU[0] = drho * W + f.rho * dW;
#pragma unroll
    for (int k = 0; k < DIM; ++k) dU[1 + k] = dZ * f.v[k] + Z * dv[k];
    dU[M - 1] = dZ - dp;
    const R dbeta = (drho - f.beta * dp) * f.ip;
    dV[0] = drho * f.irho + dbeta * (c1 * f.p * f.irho) + dbeta;
    const R dbW = dbeta * W + f.beta * dW;
#pragma unroll
    for (int k = 0; k < DIM; ++k) dV[1 + k] = dbW * f.v[k] + f.beta * W * dv[k];
    dV[M - 1] = -dbW;
}

// Rotation T_0 with first row n (Section 4), read with atan2 semantics:
// row 2 = (-n2, n1, 0)/rho_perp, row 3 = (-n3 n1/rho_perp, -n3 n2/rho_perp, rho_perp),
// rho_perp = sqrt(n1^2 + n2^2); rows (0,1,0), (-n3,0,0) when rho_perp = 0.
template <int DIM, typename R>
__device__ __forceinline__ void rotation(const R* n, R T[3][3]) {
    if (DIM == 2) {
        T[0][0] = n[0]; T[0][1] = n[1]; T[0][2] = R(0.0);
        T[1][0] = -n[1]; T[1][1] = n[0]; T[1][2] = R(0.0);
        T[2][0] = R(0.0); T[2][1] = R(0.0); T[2][2] = R(1.0);
        return;
    }
    const R rp = xsqrt(n[0] * n[0] + n[1] * n[1]);
    T[0][0] = n[0]; T[0][1] = n[1]; T[0][2] = n[2];
    if (rp > R(0.0)) {
        const R ir = frcp(rp);
        T[1][0] = -n[1] * ir; T[1][1] = n[0] * ir; T[1][2] = R(0.0);
        T[2][0] = -n[2] * n[0] * ir; T[2][1] = -n[2] * n[1] * ir; T[2][2] = rp;
    } else {
        T[1][0] = R(0.0); T[1][1] = R(1.0); T[1][2] = R(0.0);
        T[2][0] = -n[2]; T[2][1] = R(0.0); T[2][2] = R(0.0);
    }
}

// Face state and scaled eigenvectors at one face (rotated frame): from the
// rotated entropy variables V2, V3 of nodes i and i+1 and the face metrics
// (a_t, L = |a_x|) returns lambda^ and calls col(r, q) for each column r of R,
// q = 0: acoustic lambda_-, q = 1: acoustic lambda_+, q = 2..: the v_n cluster.
template <int DIM, typename R, typename Col>
__device__ __forceinline__ R face_eigen_columns(R G, const R* V2, const R* V3, R at, R L, Col&& col) {
    constexpr int M = DIM + 2;
    constexpr int NC = DIM;          // cluster size (entropy + transverse shear waves)
    const R c0 = G / (G - R(1.0)), c1 = R(1.0) / (G - R(1.0));
    // face state in the rotated frame: the state whose entropy variables are the
    // mean of those of nodes i and i+1 (beta^2 = V_E^2 - |V_u|^2, u = V_u/beta,
    // W = -V_E/beta, ln rho = V_1 - G/(G-1) - ln(beta)/(G-1) - beta, p = rho/beta)
    R Vb[M];
#pragma unroll
    for (int c = 0; c < M; ++c) Vb[c] = R(0.5) * (V2[c] + V3[c]);
    R vu2 = R(0.0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) vu2 += Vb[1 + a] * Vb[1 + a];
    const R beta_f = psqrt(Vb[M - 1] * Vb[M - 1] - vu2);
    const R ib = frcp(beta_f);
    FaceRHD<DIM, R> fs;
    fs.beta = beta_f;
    fs.W = -Vb[M - 1] * ib;
    fs.rho = xexp(Vb[0] - c0 - xlog(beta_f) * c1 - beta_f);
    fs.irho = frcp(fs.rho);
    fs.p = fs.rho * ib;
    fs.ip = beta_f * fs.irho;
    const R iVE = -frcp(Vb[M - 1]);      // 1/(beta W)
#pragma unroll
    for (int k = 0; k < DIM; ++k) fs.v[k] = Vb[1 + k] * iVE;
    const R rho = fs.rho, p = fs.p, W = fs.W;
    const R* v = fs.v;
    R v2 = R(0.0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) v2 += v[k] * v[k];
    const R vn = v[0];
    // p/rho = 1/beta, so h = 1 + c0/beta and h cs^2 = G/beta
    const R h = R(1.0) + c0 * ib;
    fs.h = h;
    const R cs2 = G * ib * frcp(h);
    const R cs = psqrt(cs2);
    const R disc = psqrt((R(1.0) - v2) * (R(1.0) - v2 * cs2 - vn * vn * (R(1.0) - cs2)));
    const R iden = frcp(R(1.0) - v2 * cs2);
    const R lam_m = (vn * (R(1.0) - cs2) - cs * disc) * iden;
    const R lam_p = (vn * (R(1.0) - cs2) + cs * disc) * iden;
    const R lhat = fmax(fabs(at + L * lam_m), fmax(fabs(at + L * vn), fabs(at + L * lam_p)));


    // acoustic columns
    const R hW2 = h * W * W;
    R vt2 = R(0.0);
#pragma unroll
    for (int k = 1; k < DIM; ++k) vt2 += v[k] * v[k];
    const R i_rhW2 = frcp(rho * hW2);
    const R i_ht = frcp(h * (R(1.0) + W * W * vt2));
    const R ig = beta_f / G;                    // 1/(h cs^2)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const R lam = s == 0 ? lam_m : lam_p;
        const R q = lam - vn;
        const R dp = q;
        const R drho = q * ig;
        R dv[DIM];
        dv[0] = (R(1.0) - vn * lam) * i_rhW2;
        const R dh = c0 * (dp - p * drho * fs.irho) * fs.irho;
        const R fac = -(dh + hW2 * vn * dv[0]) * i_ht;
#pragma unroll
        for (int k = 1; k < DIM; ++k) dv[k] = v[k] * fac;
        R dU[M], dV[M];
        tangent_rhd<DIM>(c0, c1, fs, drho, dv, dp, dU, dV);
        R nn = R(0.0);
#pragma unroll
        for (int c = 0; c < M; ++c) nn += dU[c] * dV[c];
        const R sc = frsqrt(nn);
#pragma unroll
        for (int c = 0; c < M; ++c) dU[c] *= sc;
        col(dU, s);
    }

    // v_n cluster: basis e_rho, e_{v_t1}(, e_{v_t2}) in primitive variables
    R KU[NC][M], KV[NC][M];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        R dv[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) dv[k] = R(0.0);
        R drho = R(0.0);
        if (a == 0) drho = R(1.0); else dv[a] = R(1.0);
        tangent_rhd<DIM>(c0, c1, fs, drho, dv, R(0.0), KU[a], KV[a]);
    }
    R Gm[NC][NC];
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            R s = R(0.0), t = R(0.0);
#pragma unroll
            for (int c = 0; c < M; ++c) { s += KU[a][c] * KV[b][c]; t += KU[b][c] * KV[a][c]; }
            Gm[a][b] = R(0.5) * (s + t);
        }
    R Gi[NC][NC];
    if (NC == 2) {
        const R det = Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0];
        const R id = frcp(det);
        Gi[0][0] = Gm[1][1] * id; Gi[1][1] = Gm[0][0] * id;
        Gi[0][1] = -Gm[0][1] * id; Gi[1][0] = -Gm[1][0] * id;
    } else {
        const R c00 = Gm[1][1] * Gm[2][2] - Gm[1][2] * Gm[2][1];
        const R c01 = Gm[1][2] * Gm[2][0] - Gm[1][0] * Gm[2][2];
        const R c02 = Gm[1][0] * Gm[2][1] - Gm[1][1] * Gm[2][0];
        const R det = Gm[0][0] * c00 + Gm[0][1] * c01 + Gm[0][2] * c02;
        const R id = frcp(det);
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
    R cf[NC][NC];     // coefficient vectors of the canonical columns
    R inq[NC];        // reciprocals of their squared A0^{-1} norms
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int seed = q == 0 ? 0 : 1 + q;
        R gs[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) gs[a] = KV[a][seed];
        R cq[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            R s = R(0.0);
#pragma unroll
            for (int b = 0; b < NC; ++b) s += Gi[a][b] * gs[b];
            cq[a] = s;
        }
#pragma unroll
        for (int r = 0; r < q; ++r) {
            R ip = R(0.0);
#pragma unroll
            for (int a = 0; a < NC; ++a) ip += cf[r][a] * gs[a];
            const R f = ip * inq[r];
#pragma unroll
            for (int a = 0; a < NC; ++a) cq[a] -= f * cf[r][a];
        }
        R nn = R(0.0);
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) nn += cq[a] * Gm[a][b] * cq[b];
#pragma unroll
        for (int a = 0; a < NC; ++a) cf[q][a] = cq[a];
        const R rn = frsqrt(nn);
        inq[q] = rn * rn;
        const R sc = rn;
        R r[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            R s = R(0.0);
#pragma unroll
            for (int a = 0; a < NC; ++a) s += cq[a] * KU[a][c];
            r[c] = s * sc;
        }
        col(r, 2 + q);
    }

    return lhat;
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
//
// The stencil states come from node(j), j = 0..2P-1 (nodes i-P+1..i+P; WENO of
// order w = 2P - 1: WENO7 for P = 4, WENO5 for P = 3, WENO3 for P = 2).  The face eigen-structure
// is formed first from nodes i and i+1 alone; the rotated entropy vectors of the
// stencil are formed afterwards and projected onto the columns at once, so that
// they are not held while the eigen-structure is built (register use).
template <int DIM, typename R, int P = 3, typename NodeFn>
__device__ __forceinline__ void face_diss_rhd_fn(R G, R eps, NodeFn&& node, const R* al, const R* ar, R* d) {
    constexpr int M = DIM + 2;
    constexpr int NS = 2 * P, CI = P - 1;    // stencil size, index of node i
    const R at = R(0.5) * (al[0] + ar[0]);
    R ax[3] = {R(0.0), R(0.0), R(0.0)};
#pragma unroll
    for (int j = 0; j < DIM; ++j) ax[j] = R(0.5) * (al[1 + j] + ar[1 + j]);
    const R L = psqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    const R iL = frcp(L);
    R nrm[3] = {ax[0] * iL, ax[1] * iL, ax[2] * iL};
    R T[3][3];
    rotation<DIM>(nrm, T);

    // rotated entropy variables T V of stencil node j
    const R c0 = G / (G - R(1.0)), c1 = R(1.0) / (G - R(1.0));
    auto tv = [&](int j, R* out) {
        const NodeRHD<DIM, R> q = node(j);
        out[0] = c0 + q.lr + q.lb * c1 + q.beta;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            R s = R(0.0);
#pragma unroll
            for (int b = 0; b < DIM; ++b) s += T[a][b] * q.u[b];
            out[1 + a] = q.beta * s;
        }
        out[M - 1] = -q.beta * q.W;
    };
    R TV2[M], TV3[M];      // nodes i and i+1
    tv(CI, TV2);
    tv(CI + 1, TV3);
    // rounding scale of the projections r . T V at nodes i and i+1
    R tv2 = R(0.0), tv3 = R(0.0);
#pragma unroll
    for (int c = 0; c < M; ++c) { tv2 = fmax(tv2, fabs(TV2[c])); tv3 = fmax(tv3, fabs(TV3[c])); }
    const R tvmax = tv2 + tv3;

    R Rm[M][M];
    const R lhat = face_eigen_columns<DIM>(G, TV2, TV3, at, L, [&](const R* r, int q) {
#pragma unroll
        for (int c = 0; c < M; ++c) Rm[q][c] = r[c];
    });

    // projections of the six stencil states onto the columns (the fence keeps
    // the reads of the other four states after the eigen-structure)
#ifndef ES_OPCOUNT_HOST
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#endif
    R vt[M][NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        R TVj[M];
        if (j == CI) {
#pragma unroll
            for (int c = 0; c < M; ++c) TVj[c] = TV2[c];
        } else if (j == CI + 1) {
#pragma unroll
            for (int c = 0; c < M; ++c) TVj[c] = TV3[c];
        } else {
            tv(j, TVj);
        }
#pragma unroll
        for (int q = 0; q < M; ++q) {
            R s = R(0.0);
#pragma unroll
            for (int c = 0; c < M; ++c) s += Rm[q][c] * TVj[c];
            vt[q][j] = s;
        }
#ifndef ES_OPCOUNT_HOST
        __builtin_amdgcn_sched_barrier(0);   // one stencil state at a time
#endif
    }

    // per column: reconstruct, switch, accumulate (in column order)
    R dd[M];
#pragma unroll
    for (int c = 0; c < M; ++c) dd[c] = R(0.0);
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const R* r = Rm[q];
        R vm, vp;
        if (P == 4) {
            vm = weno7(vt[q][0], vt[q][1], vt[q][2], vt[q][3], vt[q][4], vt[q][5], vt[q][6], eps);
            vp = weno7(vt[q][7], vt[q][6], vt[q][5], vt[q][4], vt[q][3], vt[q][2], vt[q][1], eps);
        } else if (P == 3) {
            vm = weno5(vt[q][0], vt[q][1], vt[q][2], vt[q][3], vt[q][4], eps);
            vp = weno5(vt[q][5], vt[q][4], vt[q][3], vt[q][2], vt[q][1], eps);
        } else {
            vm = weno3(vt[q][0], vt[q][1], vt[q][2], eps);
            vp = weno3(vt[q][3], vt[q][2], vt[q][1], eps);
        }
        const R jw = vp - vm;
        const R jp = vt[q][CI + 1] - vt[q][CI];
        // a jump within rounding of zero counts as zero (Y = 0)
        R r1 = R(0.0);
#pragma unroll
        for (int c = 0; c < M; ++c) r1 += fabs(r[c]);
        if (jw * jp > R(0.0) && fabs(jp) > RealTraits<R>::ytol * r1 * tvmax) {
#pragma unroll
            for (int c = 0; c < M; ++c) dd[c] += jw * r[c];
        }
#ifndef ES_OPCOUNT_HOST
        // one column at a time (interleaving the columns' WENO raises register use)
        __builtin_amdgcn_sched_barrier(0);
#endif
    }

    // back to the original frame: d = lambda^ T^{-1} (R Y <<V~>>)
    d[0] = lhat * dd[0];
    d[M - 1] = lhat * dd[M - 1];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        R s = R(0.0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) s += T[b][a] * dd[1 + b];
        d[1 + a] = lhat * s;
    }
}

template <int DIM, typename R>
__device__ __forceinline__ void face_diss_rhd(R G, R eps, const NodeRHD<DIM, R>* nd,
                                              const R* al, const R* ar, R* d) {
    face_diss_rhd_fn<DIM, R>(G, eps, [&](int j) { return nd[j]; }, al, ar, d);
}

}  // namespace es
