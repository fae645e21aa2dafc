// Algorithmic FP64 operation count of the residual (2D/3D RHD, p = 3).
//
// The device arithmetic of es_rhd.h (two-point EC flux and face dissipation)
// is compiled for the host with an op-counting scalar in place of double and
// executed on representative node states; each + - * /, sqrt, log, exp, fabs,
// fmax/fmin counts one operation and fma counts two.  Per node and direction
// the residual evaluates one state preparation, three two-point fluxes, one
// face dissipation and the flux-difference accumulation; these are summed
// into the per-node figure used as the algorithmic work of es_residual.
//
// Build and run (host only):  python -m paper_2107_12027_amd.build --opcount
#include "es_common.h"

#include <cmath>
#include <cstdio>
#include <random>

namespace cnt {

struct Cnt {
    double v;
    static long long ops;
    constexpr Cnt(double x = 0.0) : v(x) {}
};
long long Cnt::ops = 0;

inline Cnt operator+(Cnt a, Cnt b) { ++Cnt::ops; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++Cnt::ops; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++Cnt::ops; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++Cnt::ops; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator==(Cnt a, Cnt b) { return a.v == b.v; }
inline Cnt fma(Cnt a, Cnt b, Cnt c) { Cnt::ops += 2; return Cnt(std::fma(a.v, b.v, c.v)); }
inline Cnt sqrt(Cnt a) { ++Cnt::ops; return Cnt(std::sqrt(a.v)); }
inline Cnt log(Cnt a) { ++Cnt::ops; return Cnt(std::log(a.v)); }
inline Cnt exp(Cnt a) { ++Cnt::ops; return Cnt(std::exp(a.v)); }
inline Cnt fabs(Cnt a) { ++Cnt::ops; return Cnt(std::fabs(a.v)); }
inline Cnt fmax(Cnt a, Cnt b) { ++Cnt::ops; return Cnt(std::fmax(a.v, b.v)); }
inline Cnt fmin(Cnt a, Cnt b) { ++Cnt::ops; return Cnt(std::fmin(a.v, b.v)); }

}  // namespace cnt

using cnt::Cnt;
using cnt::fma;
using cnt::sqrt;
using cnt::log;
using cnt::exp;
using cnt::fabs;
using cnt::fmax;
using cnt::fmin;

#define ES_OPCOUNT_HOST 1
#undef __device__
#define __device__
#undef __forceinline__
#define __forceinline__ inline
#define double Cnt
#include "es_rhd.h"
#undef double

template <int DIM>
static void count(double G, std::mt19937_64& rng, int samples) {
    constexpr int NU = DIM, M = DIM + 2, NA = DIM + 1;
    std::uniform_real_distribution<double> U01(0.0, 1.0);
    auto node = [&](double base) {
        es::NodeRHD<NU> n;
        const double rho = base * (1.0 + 0.3 * U01(rng)), p = 0.5 + 0.3 * U01(rng);
        n.rho = rho; n.p = p; n.beta = rho / p;
        double uu = 0.0;
        for (int k = 0; k < NU; ++k) { n.u[k] = 0.6 * (U01(rng) - 0.5); uu += n.u[k].v * n.u[k].v; }
        n.W = std::sqrt(1.0 + uu);
        n.lr = std::log(rho); n.lb = std::log(rho / p);
        return n;
    };
    long long pair_ops = 0, face_ops = 0;
    for (int s = 0; s < samples; ++s) {
        es::NodeRHD<NU> st[6];
        for (int q = 0; q < 6; ++q) st[q] = node(1.0 + 0.05 * q);
        Cnt al[NA], ar[NA];
        for (int c = 0; c < NA; ++c) { al[c] = 0.1 * U01(rng) + (c == 1); ar[c] = 0.1 * U01(rng) + (c == 1); }
        Cnt F[M], Jt, d[M];
        Cnt::ops = 0;
        es::pair_flux_rhd<NU>(Cnt(G), st[2], st[3], al, ar, F, Jt);
        pair_ops += Cnt::ops;
        Cnt::ops = 0;
        es::face_diss_rhd<DIM>(Cnt(G), Cnt(1e-6), st, al, ar, d);
        face_ops += Cnt::ops;
    }
    const double pair = (double)pair_ops / samples, face = (double)face_ops / samples;
    // state preparation per node: |u|^2 (NU mul + NU-1 add), 1 + |u|^2, sqrt, rho/p
    const double prep = 2.0 * NU - 1 + 1 + 1 + 1;
    // flux differences: per component (M + 1 incl. J) three (sub, mul, add), one scale;
    // dissipation difference: per component sub, two mul, add
    const double accum = (M + 1) * (3 * 3 + 1) + M * 4;
    const double per_dir = prep + 3 * pair + face + accum;
    std::printf("dim %d RHD: pair %.1f face %.1f prep %.0f accum %.0f -> per node per direction %.1f, "
                "per node (all %d directions) %.1f FP64 ops\n",
                DIM, pair, face, prep, accum, per_dir, DIM, DIM * per_dir);
}

int main() {
    std::mt19937_64 rng(12345);
    count<2>(5.0 / 3.0, rng, 2000);
    count<3>(5.0 / 3.0, rng, 2000);
    return 0;
}
