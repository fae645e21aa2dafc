// Host check of the adjoint's hand-written backward sweeps (compiled for the CPU
// from the device headers, as the op count is): the RHD pair-flux VJP
// (es_pair_vjp.h) and the face eigen-structure VJP (es_eigen_vjp.h) against
// forward-mode dual-number derivatives of the same device functions, on random
// pairs (also small jumps, the series branch of the logarithmic mean) and random
// face states (near rest to fast flow), 2D and 3D.  Exit status 0 when every
// relative difference is below 1e-11 (pairs) and 1e-10 (eigen-structure).
#include "es_common.h"
#include <cmath>
#include <cstdio>
#include <random>
#undef __device__
#define __device__
#undef __forceinline__
#define __forceinline__ inline
#define ES_OPCOUNT_HOST 1
#include "es_rhd.h"
#include "es_dual.h"
#include "es_pair_vjp.h"
#include "es_eigen_vjp.h"
using namespace es;


template <int NU, typename R>
NodeRHD<NU, R> node_from_prim(const R& rho, const R* u, const R& p) {
    NodeRHD<NU, R> n; n.rho = rho; n.p = p; R uu = R(0.0);
    for (int k = 0; k < NU; ++k) { n.u[k] = u[k]; uu += u[k] * u[k]; }
    n.W = xsqrt(R(1.0) + uu); n.beta = rho / p; n.lr = xlog(rho); n.lb = xlog(n.beta); return n;
}
template <int NU, int SIDE>
void side_dual(double G, const double* Pl, const double* Pr, const double* al, const double* ar, const double* w, double* g) {
    constexpr int M = NU + 2; using D = Dual<M>;
    D rl = SIDE == 0 ? D::seed(Pl[0], 0) : D(Pl[0]);
    D pl = SIDE == 0 ? D::seed(Pl[M - 1], M - 1) : D(Pl[M - 1]);
    D rr = SIDE == 1 ? D::seed(Pr[0], 0) : D(Pr[0]);
    D pr = SIDE == 1 ? D::seed(Pr[M - 1], M - 1) : D(Pr[M - 1]);
    D ul[NU], ur[NU];
    for (int k = 0; k < NU; ++k) { ul[k] = SIDE == 0 ? D::seed(Pl[1 + k], 1 + k) : D(Pl[1 + k]); ur[k] = SIDE == 1 ? D::seed(Pr[1 + k], 1 + k) : D(Pr[1 + k]); }
    const NodeRHD<NU, D> l = node_from_prim<NU>(rl, ul, pl);
    const NodeRHD<NU, D> r = node_from_prim<NU>(rr, ur, pr);
    D F[M]; double Jt;
    pair_flux_rhd<NU>(G, l, r, al, ar, F, Jt);
    for (int i = 0; i < M; ++i) { double s = 0.0; for (int c = 0; c < M; ++c) s += w[c] * F[c].d[i]; g[i] = s; }
}
template <int NU>
int run_pair(std::mt19937_64& rng, bool small) {
    constexpr int M = NU + 2;
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double worst = 0.0;
    for (int t = 0; t < 20000; ++t) {
        double Pl[M], Pr[M], al[NU + 1], ar[NU + 1], w[M];
        Pl[0] = 0.05 + U(rng); Pl[M - 1] = 0.05 + U(rng);
        for (int k = 0; k < NU; ++k) Pl[1 + k] = 3.0 * (U(rng) - 0.5);
        double eps = small ? 1e-3 * U(rng) : 1.0;
        for (int c = 0; c < M; ++c) Pr[c] = small ? Pl[c] * (1.0 + eps * (U(rng) - 0.5)) : (c == 0 || c == M - 1 ? 0.05 + U(rng) : 3.0 * (U(rng) - 0.5));
        for (int c = 0; c <= NU; ++c) { al[c] = U(rng) - 0.5 + (c == 1); ar[c] = U(rng) - 0.5 + (c == 1); }
        for (int c = 0; c < M; ++c) w[c] = U(rng) - 0.5;
        double gl[M], gr[M], dl[M], dr[M];
        pair_vjp_rhd<NU>(5.0 / 3.0, Pl, Pr, al, ar, w, gl, gr);
        side_dual<NU, 0>(5.0 / 3.0, Pl, Pr, al, ar, w, dl);
        side_dual<NU, 1>(5.0 / 3.0, Pl, Pr, al, ar, w, dr);
        double sc = 0.0, e = 0.0;
        for (int c = 0; c < M; ++c) { sc = std::fmax(sc, std::fmax(std::fabs(dl[c]), std::fabs(dr[c]))); }
        for (int c = 0; c < M; ++c) e = std::fmax(e, std::fmax(std::fabs(gl[c] - dl[c]), std::fabs(gr[c] - dr[c])));
        worst = std::fmax(worst, e / sc);
    }
    printf("NU=%d %s: worst relative difference reverse vs dual %.3e\n", NU, small ? "small jumps" : "random pairs", worst);
    return worst < 1e-11 ? 0 : 1;
}


template <int DIM>
int run_eigen(std::mt19937_64& rng, int trials) {
    constexpr int M = DIM + 2;
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const double G = 5.0 / 3.0, c0 = G / (G - 1.0), c1 = 1.0 / (G - 1.0);
    double worst = 0.0;
    for (int t = 0; t < trials; ++t) {
        // a random admissible face state -> its entropy variables
        const double rho = 0.05 + 2.0 * U(rng), p = 0.02 + 2.0 * U(rng);
        double u[DIM], uu = 0.0;
        const double scale = t % 3 == 0 ? 1e-3 : (t % 3 == 1 ? 0.5 : 3.0);
        for (int k = 0; k < DIM; ++k) { u[k] = scale * (U(rng) - 0.5); uu += u[k] * u[k]; }
        const double W = std::sqrt(1.0 + uu), beta = rho / p;
        double Vb[M];
        Vb[0] = c0 + std::log(rho) + std::log(beta) * c1 + beta;    // G/(G-1) + ln rho + ln beta/(G-1) + beta
        // V = (.., beta W v, -beta W): u = W v
        for (int k = 0; k < DIM; ++k) Vb[1 + k] = beta * u[k];
        Vb[M - 1] = -beta * W;
        const double at = 2.0 * (U(rng) - 0.5), L = 0.5 + U(rng);
        double gR[M][M], glhat = U(rng) - 0.5;
        for (int q = 0; q < M; ++q) for (int c = 0; c < M; ++c) gR[q][c] = U(rng) - 0.5;
        double gV[M];
        face_eigen_vjp<DIM>(G, Vb, at, L, [&](int q, int c) { return gR[q][c]; }, glhat, gV);
        using D1 = Dual<1>;
        double gD[M], sc = 0.0, e = 0.0;
        for (int k = 0; k < M; ++k) {
            D1 Vd[M];
            for (int c = 0; c < M; ++c) Vd[c] = c == k ? D1::seed(Vb[c], 0) : D1(Vb[c]);
            double dir = 0.0;
            const D1 lh = face_eigen_columns<DIM>(D1(G), Vd, Vd, D1(at), D1(L), [&](const D1* r, int q) {
                for (int c = 0; c < M; ++c) dir += gR[q][c] * r[c].d[0];
            });
            gD[k] = dir + glhat * lh.d[0];
            sc = std::fmax(sc, std::fabs(gD[k]));
        }
        for (int k = 0; k < M; ++k) e = std::fmax(e, std::fabs(gV[k] - gD[k]));
        if (e / sc > worst) {
            worst = e / sc;
            if (worst > 1e-9) {
                printf("trial %d: ", t);
                for (int k = 0; k < M; ++k) printf("(%.6e %.6e) ", gV[k], gD[k]);
                printf("\n");
            }
        }
    }
    printf("DIM=%d: worst relative difference reverse vs dual %.3e over %d states\n", DIM, worst, trials);
    return worst < 1e-10 ? 0 : 1;
}
int main() {
    std::mt19937_64 rng(3);
    int bad = run_pair<2>(rng, false) + run_pair<2>(rng, true) + run_pair<3>(rng, false) + run_pair<3>(rng, true);
    std::mt19937_64 rng2(7);
    bad += run_eigen<2>(rng2, 3000) + run_eigen<3>(rng2, 3000);
    return bad;
}
