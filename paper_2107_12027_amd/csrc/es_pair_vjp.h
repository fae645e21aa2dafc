// Reverse accumulation through the RHD two-point EC flux (eq. ECFluxCurv with
// the pair U~, F~_j of pair_flux_rhd): given the cotangent w of the flux F of
// the pair (l, r), the cotangents of both nodes' primitive states P = (rho,
// u_1..u_NU, p) in one backward sweep.  The metric contraction (a_t, a_j) is a
// constant of the map; the logarithmic means are differentiated in the branch
// their values take (the series branch for small jumps).
#pragma once

#include "es_rhd.h"

namespace es {

// The logarithmic mean L(a_l, a_r) = [a]/[ln a] of log_mean with its partial
// derivatives (the logarithms as functions of the values).  Difference branch:
// dL/da_l = (1 - L/a_l)/D, dL/da_r = (L/a_r - 1)/D with D = ln a_l - ln a_r.
// Series branch: L = s/(2 F(u)), s = a_l + a_r, f = (a_l - a_r)/s, u = f^2,
// F(u) = sum_{k<=7} u^k/(2k+1); with df/da_l = 2 a_r/s^2, df/da_r = -2 a_l/s^2,
// dL/da = 1/(2F) + q (a_r or -a_l), q = -2 f F'(u)/(F^2 s).
__device__ __forceinline__ double log_mean_d(double al, double ar, double lnal, double lnar,
                                             double& dl, double& dr) {
    const double s = al + ar;
    const double dif = al - ar;
    if (dif * dif < 1e-2 * (s * s)) {
        const double is = 1.0 / s;
        const double f = dif * is;
        const double u = f * f;
        double F = 1.0 / 15.0, dF = 0.0;
        const double c[7] = {1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0, 1.0};
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            dF = fma(dF, u, F);
            F = fma(F, u, c[k]);
        }
        const double iF = 1.0 / F;
        const double q = -2.0 * f * dF * iF * iF * is;
        dl = 0.5 * iF + q * ar;
        dr = 0.5 * iF - q * al;
        return 0.5 * s * iF;
    }
    const double iD = 1.0 / (lnal - lnar);
    const double L = dif * iD;
    dl = (1.0 - L / al) * iD;
    dr = (L / ar - 1.0) * iD;
    return L;
}

// gl = (dF/dP_l)^T w, gr = (dF/dP_r)^T w for the pair flux of pair_flux_rhd.
template <int NU>
__device__ __forceinline__ void pair_vjp_rhd(double G, const double* Pl, const double* Pr, const double* al,
                                             const double* ar, const double* w, double* gl, double* gr) {
    constexpr int M = NU + 2;
    const double* Pq[2] = {Pl, Pr};
    double rho[2], p[2], u[2][NU], W[2], beta[2], lr[2], lb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        rho[t] = Pq[t][0];
        p[t] = Pq[t][M - 1];
        double uu = 0.0;
#pragma unroll
        for (int k = 0; k < NU; ++k) { u[t][k] = Pq[t][1 + k]; uu += u[t][k] * u[t][k]; }
        W[t] = sqrt(1.0 + uu);
        beta[t] = rho[t] / p[t];
        lr[t] = log(rho[t]);
        lb[t] = log(beta[t]);
    }
    // forward values
    double drl[2], dbl[2];
    const double rho_ln = log_mean_d(rho[0], rho[1], lr[0], lr[1], drl[0], drl[1]);
    const double beta_ln = log_mean_d(beta[0], beta[1], lb[0], lb[1], dbl[0], dbl[1]);
    const double rho_m = 0.5 * (rho[0] + rho[1]);
    const double beta_m = 0.5 * (beta[0] + beta[1]);
    const double W_m = 0.5 * (W[0] + W[1]);
    const double at = 0.5 * (al[0] + ar[0]);
    double um[NU], ab[NU];
    double uu = 0.0, un = 0.0;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        um[k] = 0.5 * (u[0][k] + u[1][k]);
        ab[k] = 0.5 * (al[1 + k] + ar[1 + k]);
        uu += um[k] * um[k];
        un += ab[k] * um[k];
    }
    const double ibg = 1.0 / ((G - 1.0) * beta_ln);
    const double a0 = 1.0 + ibg;
    const double iden = 1.0 / (W_m * W_m - uu);
    const double ibm = 1.0 / beta_m;
    const double pb = rho_m * ibm;
    const double U1 = rho_ln * W_m;
    const double B = a0 * U1 * W_m + pb * uu;
    const double U5 = B * iden;
    const double A = a0 * rho_ln + pb;
    const double C = W_m * A * iden;
    const double iW = 1.0 / W_m;
    const double s = (at * (U5 + pb) + C * un) * iW;
    // backward sweep
    double g_s = 0.0, g_pb = 0.0, g_um[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        g_s += w[1 + k] * um[k];
        g_um[k] = w[1 + k] * s;
        g_pb += w[1 + k] * ab[k];
    }
    double g_U5 = w[M - 1] * at, g_C = w[M - 1] * un, g_un = w[M - 1] * C;
    const double g_X = g_s * iW;
    double g_Wm = -g_s * s * iW;
    g_U5 += g_X * at;
    g_pb += g_X * at;
    g_C += g_X * un;
    g_un += g_X * C;
    double g_rln = w[0] * (at * W_m + un);
    g_Wm += w[0] * rho_ln * at;
    g_un += w[0] * rho_ln;
    g_Wm += g_C * A * iden;
    const double g_A = g_C * W_m * iden;
    double g_iden = g_C * W_m * A;
    double g_a0 = g_A * rho_ln;
    g_rln += g_A * a0;
    g_pb += g_A;
    const double g_B = g_U5 * iden;
    g_iden += g_U5 * B;
    g_a0 += g_B * U1 * W_m;
    const double g_U1 = g_B * a0 * W_m;
    g_Wm += g_B * a0 * U1;
    g_pb += g_B * uu;
    double g_uu = g_B * pb;
    g_rln += g_U1 * W_m;
    g_Wm += g_U1 * rho_ln;
    const double g_rm = g_pb * ibm;
    const double g_bm = -g_pb * pb * ibm;
    g_Wm += -2.0 * W_m * iden * iden * g_iden;
    g_uu += iden * iden * g_iden;
    const double g_bln = -g_a0 * ibg / beta_ln;
#pragma unroll
    for (int k = 0; k < NU; ++k) g_um[k] += 2.0 * um[k] * g_uu + ab[k] * g_un;
    double* gq[2] = {gl, gr};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const double g_beta = 0.5 * g_bm + g_bln * dbl[t];
        const double g_W = 0.5 * g_Wm;
        const double iWt = 1.0 / W[t];
        gq[t][0] = 0.5 * g_rm + g_rln * drl[t] + g_beta / p[t];
#pragma unroll
        for (int k = 0; k < NU; ++k) gq[t][1 + k] = 0.5 * g_um[k] + g_W * u[t][k] * iWt;
        gq[t][M - 1] = -g_beta * beta[t] / p[t];
    }
}

}  // namespace es
