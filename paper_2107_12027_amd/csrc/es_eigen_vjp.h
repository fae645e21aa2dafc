// Reverse accumulation through the RHD face eigen-structure of
// face_eigen_columns (es_rhd.h): given the cotangents of the scaled eigenvector
// columns R (column q, entry c) and of lambda^, the cotangent of the face
// entropy variables Vb in one backward sweep, in place of one forward tangent
// pass per component of Vb.  The branch of the maximum in lambda^ is held (the
// derivative of the branch the value takes), as the sign switch Y is.
#pragma once

#include "es_rhd.h"

namespace es {

// Cotangents of the face-state quantities of FaceRHD, accumulated over the columns.
template <int DIM>
struct FaceBar {
    double rho, irho, p, ip, beta, W, h, v[DIM];
    __device__ __forceinline__ FaceBar() : rho(0.0), irho(0.0), p(0.0), ip(0.0), beta(0.0), W(0.0), h(0.0) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) v[k] = 0.0;
    }
};

// Backward sweep of tangent_rhd (es_rhd.h) at the face state f for the
// primitive perturbation (drho, dv, dp): given gdU, gdV, accumulates the
// cotangents of f into fb and returns those of (drho, dv, dp).
template <int DIM>
__device__ __forceinline__ void tangent_rhd_vjp(double c0, double c1, const FaceRHD<DIM, double>& f, double drho,
                                                const double* dv, double dp, const double* gdU,
                                                const double* gdV, FaceBar<DIM>& fb, double& g_drho,
                                                double* g_dv, double& g_dp) {
    constexpr int M = DIM + 2;
    const double W = f.W;
    double vdv = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) vdv += f.v[k] * dv[k];
    const double W2 = W * W;
    const double dW = W2 * W * vdv;
    const double X = dp - f.p * drho * f.irho;
    const double dh = c0 * X * f.irho;
    const double Z = f.rho * f.h * W2;
    const double dZ = (drho * f.h + f.rho * dh) * W2 + 2.0 * f.rho * f.h * W * dW;
    const double dbeta = (drho - f.beta * dp) * f.ip;
    const double dbW = dbeta * W + f.beta * dW;
    g_drho = 0.0;
    g_dp = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) g_dv[k] = 0.0;
    double g_dW = 0.0, g_dZ = 0.0, g_Z = 0.0, g_dbeta = 0.0, g_dh = 0.0;
    // dV_{M-1} = -dbW, dV_{1+k} = dbW v_k + beta W dv_k
    double g_dbW = -gdV[M - 1];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        g_dbW += gdV[1 + k] * f.v[k];
        fb.v[k] += gdV[1 + k] * dbW;
        fb.beta += gdV[1 + k] * W * dv[k];
        fb.W += gdV[1 + k] * f.beta * dv[k];
        g_dv[k] += gdV[1 + k] * f.beta * W;
    }
    // dbW = dbeta W + beta dW
    g_dbeta += g_dbW * W;
    fb.W += g_dbW * dbeta;
    fb.beta += g_dbW * dW;
    g_dW += g_dbW * f.beta;
    // dV_0 = drho irho + dbeta (c1 p irho + 1)
    g_drho += gdV[0] * f.irho;
    fb.irho += gdV[0] * (drho + dbeta * c1 * f.p);
    g_dbeta += gdV[0] * (c1 * f.p * f.irho + 1.0);
    fb.p += gdV[0] * dbeta * c1 * f.irho;
    // dbeta = (drho - beta dp) ip
    g_drho += g_dbeta * f.ip;
    fb.beta -= g_dbeta * dp * f.ip;
    g_dp -= g_dbeta * f.beta * f.ip;
    fb.ip += g_dbeta * (drho - f.beta * dp);
    // dU_0 = drho W + rho dW; dU_{1+k} = dZ v_k + Z dv_k; dU_{M-1} = dZ - dp
    g_drho += gdU[0] * W;
    fb.W += gdU[0] * drho;
    fb.rho += gdU[0] * dW;
    g_dW += gdU[0] * f.rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        g_dZ += gdU[1 + k] * f.v[k];
        fb.v[k] += gdU[1 + k] * dZ;
        g_Z += gdU[1 + k] * dv[k];
        g_dv[k] += gdU[1 + k] * Z;
    }
    g_dZ += gdU[M - 1];
    g_dp -= gdU[M - 1];
    // Z = rho h W^2
    fb.rho += g_Z * f.h * W2;
    fb.h += g_Z * f.rho * W2;
    fb.W += g_Z * 2.0 * f.rho * f.h * W;
    // dZ = (drho h + rho dh) W^2 + 2 rho h W dW
    g_drho += g_dZ * f.h * W2;
    fb.h += g_dZ * (drho * W2 + 2.0 * f.rho * W * dW);
    fb.rho += g_dZ * (dh * W2 + 2.0 * f.h * W * dW);
    g_dh += g_dZ * f.rho * W2;
    fb.W += g_dZ * ((drho * f.h + f.rho * dh) * 2.0 * W + 2.0 * f.rho * f.h * dW);
    g_dW += g_dZ * 2.0 * f.rho * f.h * W;
    // dh = c0 X irho, X = dp - p drho irho
    const double g_X = g_dh * c0 * f.irho;
    fb.irho += g_dh * c0 * X;
    g_dp += g_X;
    fb.p -= g_X * drho * f.irho;
    g_drho -= g_X * f.p * f.irho;
    fb.irho -= g_X * f.p * drho;
    // dW = W^3 vdv
    fb.W += g_dW * 3.0 * W2 * vdv;
    const double g_vdv = g_dW * W2 * W;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        fb.v[k] += g_vdv * dv[k];
        g_dv[k] += g_vdv * f.v[k];
    }
}

// gVb = d(sum_{q,c} gR(q, c) R[q][c] + glhat lambda^)/dVb for the face eigen-structure
// that face_eigen_columns<DIM> forms from the face entropy variables Vb (the mean
// of the two nodes').  gR(q, c) returns the cotangent of entry c of column q.
template <int DIM, typename GR>
__device__ __forceinline__ void face_eigen_vjp(double G, const double* Vb, double at, double L, GR&& gR,
                                               double glhat, double* gVb) {
    constexpr int M = DIM + 2;
    constexpr int NC = DIM;
    const double c0 = G / (G - 1.0), c1 = 1.0 / (G - 1.0);
    // ---- forward values (as face_eigen_columns forms them)
    double vu2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) vu2 += Vb[1 + a] * Vb[1 + a];
    const double VE = Vb[M - 1];
    const double bb = VE * VE - vu2;
    const double beta = sqrt(bb);
    const double ib = 1.0 / beta;
    FaceRHD<DIM, double> f;
    f.beta = beta;
    f.W = -VE * ib;
    const double lnb = log(beta);
    f.rho = exp(Vb[0] - c0 - lnb * c1 - beta);
    f.irho = 1.0 / f.rho;
    f.p = f.rho * ib;
    f.ip = beta * f.irho;
    const double iVE = -1.0 / VE;
#pragma unroll
    for (int k = 0; k < DIM; ++k) f.v[k] = Vb[1 + k] * iVE;
    double v2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) v2 += f.v[k] * f.v[k];
    const double vn = f.v[0];
    f.h = 1.0 + c0 * ib;
    const double ih = 1.0 / f.h;
    const double cs2 = G * ib * ih;
    const double cs = sqrt(cs2);
    const double E1 = 1.0 - v2;
    const double E2 = 1.0 - v2 * cs2 - vn * vn * (1.0 - cs2);
    const double disc = sqrt(E1 * E2);
    const double iden = 1.0 / (1.0 - v2 * cs2);
    const double Nmp[2] = {vn * (1.0 - cs2) - cs * disc, vn * (1.0 - cs2) + cs * disc};
    const double lam[2] = {Nmp[0] * iden, Nmp[1] * iden};
    const double W = f.W, W2 = W * W;
    const double hW2 = f.h * W2;
    double vt2 = 0.0;
#pragma unroll
    for (int k = 1; k < DIM; ++k) vt2 += f.v[k] * f.v[k];
    const double At = 1.0 + W2 * vt2;
    const double i_rhW2 = 1.0 / (f.rho * hW2);
    const double i_ht = 1.0 / (f.h * At);
    const double ig = beta / G;

    FaceBar<DIM> fb;
    double g_lam[2] = {0.0, 0.0}, g_vn = 0.0;
    double g_i_rhW2 = 0.0, g_i_ht = 0.0, g_hW2 = 0.0, g_ig = 0.0;

    // ---- lambda^ (the branch of the maximum held)
    {
        const double am = at + L * lam[0], a0 = at + L * vn, ap = at + L * lam[1];
        const double sm = am < 0.0 ? -1.0 : 1.0, s0 = a0 < 0.0 ? -1.0 : 1.0, sp = ap < 0.0 ? -1.0 : 1.0;
        const bool inner0 = fabs(a0) >= fabs(ap);
        const double inner = inner0 ? fabs(a0) : fabs(ap);
        if (fabs(am) >= inner) g_lam[0] += glhat * sm * L;
        else if (inner0) g_vn += glhat * s0 * L;
        else g_lam[1] += glhat * sp * L;
    }

    // ---- acoustic columns (q = 0: lambda_-, q = 1: lambda_+)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double lm = lam[s];
        const double q = lm - vn;
        const double dp = q, drho = q * ig;
        double dv[DIM];
        dv[0] = (1.0 - vn * lm) * i_rhW2;
        const double Xs = dp - f.p * drho * f.irho;
        const double dhs = c0 * Xs * f.irho;
        const double fac = -(dhs + hW2 * vn * dv[0]) * i_ht;
#pragma unroll
        for (int k = 1; k < DIM; ++k) dv[k] = f.v[k] * fac;
        double dU[M], dV[M];
        tangent_rhd<DIM>(c0, c1, f, drho, dv, dp, dU, dV);
        double nn = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) nn += dU[c] * dV[c];
        const double sc = 1.0 / sqrt(nn);
        // col = dU sc, sc = nn^(-1/2), nn = dU . dV
        double gdU[M], gdV[M], g_sc = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double g = gR(s, c);
            gdU[c] = g * sc;
            g_sc += g * dU[c];
        }
        const double g_nn = -0.5 * sc * sc * sc * g_sc;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            gdU[c] += g_nn * dV[c];
            gdV[c] = g_nn * dU[c];
        }
        double g_drho, g_dp, g_dv[DIM];
        tangent_rhd_vjp<DIM>(c0, c1, f, drho, dv, dp, gdU, gdV, fb, g_drho, g_dv, g_dp);
        // dv_k = v_k fac (k >= 1)
        double g_fac = 0.0;
#pragma unroll
        for (int k = 1; k < DIM; ++k) {
            g_fac += g_dv[k] * f.v[k];
            fb.v[k] += g_dv[k] * fac;
        }
        // fac = -(dhs + hW2 vn dv0) i_ht
        const double g_dhs = -g_fac * i_ht;
        g_hW2 -= g_fac * vn * dv[0] * i_ht;
        g_vn -= g_fac * hW2 * dv[0] * i_ht;
        const double g_dv0 = g_dv[0] - g_fac * hW2 * vn * i_ht;
        g_i_ht -= g_fac * (dhs + hW2 * vn * dv[0]);
        // dhs = c0 Xs irho, Xs = dp - p drho irho
        const double g_Xs = g_dhs * c0 * f.irho;
        fb.irho += g_dhs * c0 * Xs;
        g_dp += g_Xs;
        fb.p -= g_Xs * drho * f.irho;
        g_drho -= g_Xs * f.p * f.irho;
        fb.irho -= g_Xs * f.p * drho;
        // dv0 = (1 - vn lambda) i_rhW2
        g_vn -= g_dv0 * lm * i_rhW2;
        g_lam[s] -= g_dv0 * vn * i_rhW2;
        g_i_rhW2 += g_dv0 * (1.0 - vn * lm);
        // drho = q ig, dp = q, q = lambda - vn
        const double g_q = g_drho * ig + g_dp;
        g_ig += g_drho * q;
        g_lam[s] += g_q;
        g_vn -= g_q;
    }

    // ---- v_n cluster: canonical columns from the seeds (see face_eigen_columns)
    {
        double KU[NC][M], KV[NC][M];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            double dv[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) dv[k] = 0.0;
            double drho = 0.0;
            if (a == 0) drho = 1.0; else dv[a] = 1.0;
            tangent_rhd<DIM>(c0, c1, f, drho, dv, 0.0, KU[a], KV[a]);
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
            const double id = 1.0 / (Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0]);
            Gi[0][0] = Gm[1][1] * id; Gi[1][1] = Gm[0][0] * id;
            Gi[0][1] = -Gm[0][1] * id; Gi[1][0] = -Gm[1][0] * id;
        } else {
            const double c00 = Gm[1][1] * Gm[2][2] - Gm[1][2] * Gm[2][1];
            const double c01 = Gm[1][2] * Gm[2][0] - Gm[1][0] * Gm[2][2];
            const double c02 = Gm[1][0] * Gm[2][1] - Gm[1][1] * Gm[2][0];
            const double id = 1.0 / (Gm[0][0] * c00 + Gm[0][1] * c01 + Gm[0][2] * c02);
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
        // forward Gram-Schmidt in the coefficient space, keeping what the sweep needs
        double gs[NC][NC], cf[NC][NC], inq[NC], rn[NC], ipf[NC][NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int seed = q == 0 ? 0 : 1 + q;
#pragma unroll
            for (int a = 0; a < NC; ++a) gs[q][a] = KV[a][seed];
            double cq[NC];
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < NC; ++b) s += Gi[a][b] * gs[q][b];
                cq[a] = s;
            }
#pragma unroll
            for (int r = 0; r < NC; ++r) {
                if (r >= q) break;
                double ip = 0.0;
#pragma unroll
                for (int a = 0; a < NC; ++a) ip += cf[r][a] * gs[q][a];
                ipf[q][r] = ip;
                const double fr = ip * inq[r];
#pragma unroll
                for (int a = 0; a < NC; ++a) cq[a] -= fr * cf[r][a];
            }
            double nn = 0.0;
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) nn += cq[a] * Gm[a][b] * cq[b];
#pragma unroll
            for (int a = 0; a < NC; ++a) cf[q][a] = cq[a];
            rn[q] = 1.0 / sqrt(nn);
            inq[q] = rn[q] * rn[q];
        }
        // backward sweep, q from last to first (later columns feed cf and inq back)
        double g_cf[NC][NC], g_inq[NC], g_gs[NC][NC], g_Gm[NC][NC], g_Gi[NC][NC], g_KU[NC][M], g_KV[NC][M];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            g_inq[a] = 0.0;
#pragma unroll
            for (int b = 0; b < NC; ++b) { g_cf[a][b] = 0.0; g_gs[a][b] = 0.0; g_Gm[a][b] = 0.0; g_Gi[a][b] = 0.0; }
#pragma unroll
            for (int c = 0; c < M; ++c) { g_KU[a][c] = 0.0; g_KV[a][c] = 0.0; }
        }
#pragma unroll
        for (int q = NC - 1; q >= 0; --q) {
            // col = rn y, y_c = sum_a cq_a KU_a,c
            double y[M], gy[M], g_rn = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < NC; ++a) s += cf[q][a] * KU[a][c];
                y[c] = s;
                const double g = gR(2 + q, c);
                gy[c] = g * rn[q];
                g_rn += g * y[c];
            }
            double g_cq[NC];
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                double s = g_cf[q][a];
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    s += gy[c] * KU[a][c];
                    g_KU[a][c] += gy[c] * cf[q][a];
                }
                g_cq[a] = s;
            }
            // inq = rn^2, rn = nn^(-1/2)
            g_rn += g_inq[q] * 2.0 * rn[q];
            const double g_nn = -0.5 * rn[q] * rn[q] * rn[q] * g_rn;
            // nn = cq^T Gm cq
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < NC; ++b) {
                    s += (Gm[a][b] + Gm[b][a]) * cf[q][b];
                    g_Gm[a][b] += g_nn * cf[q][a] * cf[q][b];
                }
                g_cq[a] += g_nn * s;
            }
            // cq = Gi gs - sum_{r<q} (cf_r . gs) inq_r cf_r
#pragma unroll
            for (int r = 0; r < NC; ++r) {
                if (r >= q) break;
                const double fr = ipf[q][r] * inq[r];
                double g_fr = 0.0;
#pragma unroll
                for (int a = 0; a < NC; ++a) {
                    g_fr -= g_cq[a] * cf[r][a];
                    g_cf[r][a] -= g_cq[a] * fr;
                }
                const double g_ip = g_fr * inq[r];
                g_inq[r] += g_fr * ipf[q][r];
#pragma unroll
                for (int a = 0; a < NC; ++a) {
                    g_cf[r][a] += g_ip * gs[q][a];
                    g_gs[q][a] += g_ip * cf[r][a];
                }
            }
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) {
                    g_Gi[a][b] += g_cq[a] * gs[q][b];
                    g_gs[q][b] += g_cq[a] * Gi[a][b];
                }
            const int seed = q == 0 ? 0 : 1 + q;
#pragma unroll
            for (int a = 0; a < NC; ++a) g_KV[a][seed] += g_gs[q][a];
        }
        // Gi = Gm^{-1}: dGm = -Gi^T dGi Gi^T
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int d = 0; d < NC; ++d) s += Gi[c][a] * g_Gi[c][d] * Gi[b][d];
                g_Gm[a][b] -= s;
            }
        // Gm_ab = (KU_a . KV_b + KU_b . KV_a)/2
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const double sab = 0.5 * (g_Gm[a][b] + g_Gm[b][a]);
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    g_KU[a][c] += sab * KV[b][c];
                    g_KV[b][c] += sab * KU[a][c];
                }
            }
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            double dv[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) dv[k] = 0.0;
            double drho = 0.0;
            if (a == 0) drho = 1.0; else dv[a] = 1.0;
            double g_drho, g_dp, g_dv[DIM];
            tangent_rhd_vjp<DIM>(c0, c1, f, drho, dv, 0.0, g_KU[a], g_KV[a], fb, g_drho, g_dv, g_dp);
        }
    }

    // ---- acoustic eigenvalues: lambda = N iden, N = vn (1 - cs2) -+ cs disc
    double g_iden = 0.0, g_cs2 = 0.0, g_cs = 0.0, g_disc = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double sg = s == 0 ? -1.0 : 1.0;
        const double g_N = g_lam[s] * iden;
        g_iden += g_lam[s] * Nmp[s];
        g_vn += g_N * (1.0 - cs2);
        g_cs2 -= g_N * vn;
        g_cs += sg * g_N * disc;
        g_disc += sg * g_N * cs;
    }
    // iden = 1/(1 - v2 cs2)
    const double g_den = -g_iden * iden * iden;
    double g_v2 = -g_den * cs2;
    g_cs2 -= g_den * v2;
    // disc = sqrt(E1 E2)
    const double g_E = g_disc * 0.5 / disc;
    const double g_E1 = g_E * E2, g_E2 = g_E * E1;
    g_v2 -= g_E1;
    g_v2 -= g_E2 * cs2;
    g_cs2 += g_E2 * (vn * vn - v2);
    g_vn -= g_E2 * 2.0 * vn * (1.0 - cs2);
    // cs = sqrt(cs2), cs2 = G ib ih, ih = 1/h, h = 1 + c0 ib
    g_cs2 += g_cs * 0.5 / cs;
    double g_ib = g_cs2 * G * ih;
    const double g_ih = g_cs2 * G * ib;
    // i_rhW2 = 1/(rho hW2), i_ht = 1/(h At), At = 1 + W^2 vt2, hW2 = h W^2, ig = beta/G
    {
        const double t = -g_i_rhW2 * i_rhW2 * i_rhW2;
        fb.rho += t * hW2;
        g_hW2 += t * f.rho;
        const double u = -g_i_ht * i_ht * i_ht;
        fb.h += u * At;
        const double g_At = u * f.h;
        double g_W2 = g_At * vt2;
#pragma unroll
        for (int k = 1; k < DIM; ++k) fb.v[k] += 2.0 * f.v[k] * g_At * W2;
        fb.h += g_hW2 * W2;
        g_W2 += g_hW2 * f.h;
        fb.W += 2.0 * W * g_W2;
        fb.beta += g_ig / G;
    }
    fb.h -= g_ih * ih * ih;
    g_ib += fb.h * c0;
    // v2 = |v|^2, vn = v_0
#pragma unroll
    for (int k = 0; k < DIM; ++k) fb.v[k] += 2.0 * f.v[k] * g_v2;
    fb.v[0] += g_vn;
    // v_k = Vb_{1+k} iVE, iVE = -1/VE
    double g_iVE = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        gVb[1 + k] = fb.v[k] * iVE;
        g_iVE += fb.v[k] * Vb[1 + k];
    }
    double g_VE = g_iVE / (VE * VE);
    // ip = beta irho, p = rho ib, irho = 1/rho
    fb.beta += fb.ip * f.irho;
    fb.irho += fb.ip * beta;
    fb.rho += fb.p * ib;
    g_ib += fb.p * f.rho;
    fb.rho -= fb.irho * f.irho * f.irho;
    // rho = exp(Vb_0 - c0 - ln(beta) c1 - beta)
    const double g_lnr = fb.rho * f.rho;
    gVb[0] = g_lnr;
    fb.beta -= g_lnr * c1 / beta;
    fb.beta -= g_lnr;
    // W = -VE ib
    g_VE -= fb.W * ib;
    g_ib -= fb.W * VE;
    // ib = 1/beta, beta = sqrt(bb), bb = VE^2 - |Vu|^2
    fb.beta -= g_ib * ib * ib;
    const double g_bb = fb.beta * 0.5 / beta;
    g_VE += g_bb * 2.0 * VE;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gVb[1 + a] -= g_bb * 2.0 * Vb[1 + a];
    gVb[M - 1] = g_VE;
}

}  // namespace es
