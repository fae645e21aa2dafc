// Hand-written adjoint of the RMHD residual (FP64, p = 3): the vector-Jacobian
// product of L(U, J) = residual(con2prim(U / J), metrics) for the RMHD system,
// the counterpart of the RHD kernels in es_adjoint.hip (same segment layout,
// gathers and Runge-Kutta reverse sweep).
//
// Per direction the cotangent lambda of the residual is pulled back to the
// primitive states:
//   * two-point fluxes: F(a, a+n) receives w = alpha_n / dxi (lambda_{a+n} -
//     lambda_a), times dF/dP of either node (forward-mode dual numbers over the 8
//     primitive variables of one node at a time);
//   * Godunov-Powell source -Phi'(V_s) dB~_s/dxi (eq. RMHDSemiU_O2p_ES): the pair
//     value B~(a, a+n) = 1/4 sum_j (a_j,a + a_j,a+n)(B_j,a + B_j,a+n) receives
//     alpha_n / dxi (lambda_{a+n}.Phi'_{a+n} - lambda_a.Phi'_a) (linear in the
//     B of both nodes), and node s receives -dB~_s (dPhi'/dP_s)^T lambda_s;
//   * face dissipation d = lambda^ T^T sum_k r_k Y_k <<V~_k>> (eq. ESFlux_HO)
//     with the face eigen-structure (T, the columns r_k, lambda^) and the switch
//     Y held at their forward values: the reverse of the accumulation, of the
//     two WENO5 reconstructions (the gradient written out, as for RHD), of the
//     projections V~ = r_k . T V_j, and of the rotation, then (dV/dP)^T per node.
// The face eigen-structure is a numeric eigen-decomposition of the symmetric
// pencil; its derivative along the face entropy variables is not carried (it
// multiplies the WENO jumps, which vanish at the order of the scheme on smooth
// solutions), so the ES part is the frozen-eigen-structure derivative.
#include <math.h>

#include "es_internal.h"
#include "es_launch.h"
#include "es_rmhd.h"
#include "es_dual.h"

namespace es {

namespace {

constexpr int QSEG = 54;                  // output positions per segment
constexpr int QHALO = 5;                  // state halo each side
constexpr int QLOAD = QSEG + 2 * QHALO;   // 64 loaded slots
constexpr int QLINES = 2;                 // segments per block

template <int DIM>
struct AdjLDSM {
    static constexpr int NA = DIM + 1, NF = 8 + 2 + NA + 8;   // prims, logs, metrics, Phi'
    double sd[QLINES][NF][QLOAD];
    double lam[QLINES][8][QLOAD];
    double buf[QLINES][6][8][64];
};

struct AdjPlanM {
    int nseg[3];
    int nblk[3];
    long long nlines[3];
};

// Face eigen-structure of the ES dissipation held by the adjoint: for direction d,
// interior transverse line l and face f = p + 1 (face p+1/2 between positions p
// and p + 1 along the line, p = -1 .. n_d - 1), the 64 entries Rc[k][i] (k*8 + i)
// and lambda^ (entry 64) at eig[base[d] + (e * nlines[d] + l) * nface[d] + f].
constexpr int NEIG = 65;
struct FaceEigPlan {
    long long base[3];
    long long nlines[3];
    int nface[3];
    long long nthreads[3];   // faces of each direction
};

template <int DIM>
__global__ void __launch_bounds__(64) k_face_eigen_rmhd(GridDev g, double G, const double* __restrict__ prim,
                                                        const double* __restrict__ met, double* __restrict__ eig,
                                                        FaceEigPlan fp) {
    constexpr int NA = DIM + 1;
    long long t = (long long)blockIdx.x * 64 + threadIdx.x;
    int d = 0;
    while (d < DIM - 1 && t >= fp.nthreads[d]) { t -= fp.nthreads[d]; ++d; }
    if (t >= fp.nthreads[d]) return;
    const long long l = t / fp.nface[d];
    const int f = (int)(t % fp.nface[d]);
    const int p = f - 1;
    int ci = 0, cj = 0, ck = 0;
    if (d == 0) { cj = (int)(l % g.n[1]); ck = (int)(l / g.n[1]); }
    else if (d == 1) { ci = (int)(l % g.n[0]); ck = (int)(l / g.n[0]); }
    else { ci = (int)(l % g.n[0]); cj = (int)(l / g.n[0]); }
    const long long P = g.pnodes;
    const long long pstride = d == 0 ? 1 : (d == 1 ? (long long)g.P[0] : (long long)g.P[0] * g.P[1]);
    const long long i2 = pidx(g, ci, cj, ck) + (long long)p * pstride;
    const long long i3 = i2 + pstride;
    double P2[8], P3[8], al[NA], ar[NA];
#pragma unroll
    for (int c = 0; c < 8; ++c) { P2[c] = prim[c * P + i2]; P3[c] = prim[c * P + i3]; }
#pragma unroll
    for (int c = 0; c < NA; ++c) { al[c] = met[(d * NA + c) * P + i2]; ar[c] = met[(d * NA + c) * P + i3]; }
    double T[3][3], TV2[8], TV3[8], lhat, Rc[8][8];
    face_eigen_rmhd<DIM>(G, P2, P3, al, ar, T, TV2, TV3, lhat, Rc);
    double* o = eig + fp.base[d] + l * fp.nface[d] + f;
    const long long es = fp.nlines[d] * fp.nface[d];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int i = 0; i < 8; ++i) o[(k * 8 + i) * es] = Rc[k][i];
    o[64 * es] = lhat;
}

// Gradient of the WENO5-JS value weno5(a, b, c, d, e) with respect to its five
// inputs: with w_k = d_k / (eps + beta_k)^2, S = sum_k w_k, v = sum_k w_k q_k / (6 S),
// dv = [sum_k w_k dq_k + sum_k (q_k - 6 v) dw_k] / (6 S), dw_k = -2 w_k dbeta_k / (eps + beta_k).
__device__ __forceinline__ void weno5_grad_m(double a, double b, double c, double d, double e, double eps,
                                             double* gr) {
    const double q0 = 2.0 * a - 7.0 * b + 11.0 * c;
    const double q1 = -b + 5.0 * c + 2.0 * d;
    const double q2 = 2.0 * c + 5.0 * d - e;
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = b - d;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double e0 = eps + (13.0 / 12.0) * t0 * t0 + 0.25 * s0 * s0;
    const double e1 = eps + (13.0 / 12.0) * t1 * t1 + 0.25 * s1 * s1;
    const double e2 = eps + (13.0 / 12.0) * t2 * t2 + 0.25 * s2 * s2;
    const double ie0 = 1.0 / e0, ie1 = 1.0 / e1, ie2 = 1.0 / e2;
    const double w0 = 0.1 * ie0 * ie0, w1 = 0.6 * ie1 * ie1, w2 = 0.3 * ie2 * ie2;
    const double S = w0 + w1 + w2;
    const double iS6 = 1.0 / (6.0 * S);
    const double v6 = (w0 * q0 + w1 * q1 + w2 * q2) / S;
    const double c0 = -2.0 * w0 * (q0 - v6) * ie0, c1 = -2.0 * w1 * (q1 - v6) * ie1, c2 = -2.0 * w2 * (q2 - v6) * ie2;
    const double u0 = c0 * (13.0 / 6.0) * t0, v0 = c0 * 0.5 * s0;
    const double u1 = c1 * (13.0 / 6.0) * t1, v1 = c1 * 0.5 * s1;
    const double u2 = c2 * (13.0 / 6.0) * t2, v2 = c2 * 0.5 * s2;
    gr[0] = (2.0 * w0 + u0 + v0) * iS6;
    gr[1] = (-7.0 * w0 - w1 - 2.0 * u0 - 4.0 * v0 + u1 + v1) * iS6;
    gr[2] = (11.0 * w0 + 5.0 * w1 + 2.0 * w2 + u0 + 3.0 * v0 - 2.0 * u1 + u2 + 3.0 * v2) * iS6;
    gr[3] = (2.0 * w1 + 5.0 * w2 + u1 - v1 - 2.0 * u2 - 4.0 * v2) * iS6;
    gr[4] = (-w2 + u2 + v2) * iS6;
}

// Gradient of the WENO3-JS value weno3(a, b, c) = (w0 q0 + w1 q1) / (2 S), q0 = 3b - a,
// q1 = b + c, w_k = d_k / e_k^2 (d = 1/3, 2/3), e0 = eps + (b - a)^2, e1 = eps + (c - b)^2:
// dv = [sum_k w_k dq_k + sum_k (q_k - 2 v) dw_k] / (2 S), dw_k = -2 w_k de_k / e_k.
__device__ __forceinline__ void weno3_grad_m(double a, double b, double c, double eps, double* gr) {
    const double q0 = 3.0 * b - a, q1 = b + c;
    const double e0 = eps + (b - a) * (b - a), e1 = eps + (c - b) * (c - b);
    const double w0 = (1.0 / 3.0) * (e1 * e1), w1 = (2.0 / 3.0) * (e0 * e0);   // both times e0^2 e1^2
    const double S = w0 + w1;
    const double v2 = (w0 * q0 + w1 * q1) / S;
    const double c0 = -4.0 * w0 * (q0 - v2) * (b - a) / e0;
    const double c1 = -4.0 * w1 * (q1 - v2) * (c - b) / e1;
    const double i2S = 1.0 / (2.0 * S);
    gr[0] = (-w0 - c0) * i2S;
    gr[1] = (3.0 * w0 + w1 + c0 - c1) * i2S;
    gr[2] = (w1 + c1) * i2S;
}

// (dF/dP_l)^T w and (dF/dP_r)^T w for the RMHD two-point flux F(l, r).
template <int DIM, int SIDE>
__device__ __forceinline__ void pair_vjp_rmhd_side(double G, const double* Pl, const double* Pr, const double* al,
                                                   const double* ar, const double* w, double* g) {
    using D = Dual<8>;
    D Pdl[8], Pdr[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        Pdl[c] = SIDE == 0 ? D::seed(Pl[c], c) : D(Pl[c]);
        Pdr[c] = SIDE == 1 ? D::seed(Pr[c], c) : D(Pr[c]);
    }
    const NodeRMHDT<D> l = node_rmhd<D>(G, Pdl, xlog(Pdl[0]), xlog(Pdl[0] / Pdl[4]));
    const NodeRMHDT<D> r = node_rmhd<D>(G, Pdr, xlog(Pdr[0]), xlog(Pdr[0] / Pdr[4]));
    D F[8];
    double Jt, Bt;
    pair_flux_rmhd<DIM, D, D>(G, l, r, al, ar, F, Jt, Bt);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += w[c] * F[c].d[k];
        g[k] = s;
    }
}

// (the side is a template parameter so that the unseeded node's zero tangents
// fold away)
template <int DIM>
__device__ void pair_vjp_rmhd(double G, const double* Pl, const double* Pr, const double* al, const double* ar,
                              const double* w, double* gl, double* gr) {
    pair_vjp_rmhd_side<DIM, 0>(G, Pl, Pr, al, ar, w, gl);
    pair_vjp_rmhd_side<DIM, 1>(G, Pl, Pr, al, ar, w, gr);
}

// PO: the order parameter p (pairs n = 1..p, face stencils of 2p nodes).
template <int DIM, int DIR, bool ES, int PO>
__device__ __forceinline__ void residual_vjp_segment_rmhd(const GridDev& g, double G, double eps,
                                                          const double* __restrict__ prim,
                                                          const double* __restrict__ met,
                                                          const double* __restrict__ lam,
                                                          double* __restrict__ gout, int blk, int nseg,
                                                          long long nlines, AdjLDSM<DIM>& lds,
                                                          const double* __restrict__ eig, long long enf) {
    constexpr int NA = DIM + 1;
    constexpr int F_LR = 8, F_LB = 9, F_A = 10, F_PP = 10 + NA;
    auto& sd = lds.sd;
    auto& sl = lds.lam;
    auto& buf = lds.buf;
    const int lane = threadIdx.x & 63;
    const int line = threadIdx.x >> 6;
    const int seg = blk % nseg;
    const long long lid = (long long)(blk / nseg) * QLINES + line;
    const bool active = lid < nlines;
    const int n = g.n[DIR];
    const int s0 = -NG + seg * QSEG;                 // first output (padded coordinate)
    const int s_end = min(s0 + QSEG, n + NG);
    int ci = 0, cj = 0, ck = 0;
    if (active) {
        if (DIR == 0) { cj = (int)(lid % g.n[1]); ck = (int)(lid / g.n[1]); }
        else if (DIR == 1) { ci = (int)(lid % g.n[0]); ck = (int)(lid / g.n[0]); }
        else { ci = (int)(lid % g.n[0]); cj = (int)(lid / g.n[0]); }
    }
    const long long pstride = DIR == 0 ? 1 : (DIR == 1 ? (long long)g.P[0] : (long long)g.P[0] * g.P[1]);
    const long long istride = DIR == 0 ? 1 : (DIR == 1 ? (long long)g.n[0] : (long long)g.n[0] * g.n[1]);
    const long long pbase = pidx(g, ci, cj, ck);
    const long long ibase = iidx(g, ci, cj, ck);
    const long long P = g.pnodes, N = g.nodes;
    const double idxi = 1.0 / g.dxi[DIR];

    // ---- states (positions s0 - 5 .. s0 + 58), Phi'(V), residual cotangents
    {
        const int s = s0 - QHALO + lane;
        double v[10], a[NA];
#pragma unroll
        for (int c = 0; c < 10; ++c) v[c] = 0.0;
        v[0] = 1.0;
        v[4] = 1.0;
#pragma unroll
        for (int c = 0; c < NA; ++c) a[c] = c == 1 ? 1.0 : 0.0;
        if (active && s >= -NG && s < n + NG) {
            const long long idx = pbase + (long long)s * pstride;
#pragma unroll
            for (int c = 0; c < 10; ++c) v[c] = prim[c * P + idx];
#pragma unroll
            for (int c = 0; c < NA; ++c) a[c] = met[(DIR * NA + c) * P + idx];
        }
        const StateRMHD<double> st = rmhd_state<double>(G, v);
        double Pp[8];
        rmhd_phi_prime<double>(st, Pp);
#pragma unroll
        for (int c = 0; c < 10; ++c) sd[line][c][lane] = v[c];
#pragma unroll
        for (int c = 0; c < NA; ++c) sd[line][F_A + c][lane] = a[c];
#pragma unroll
        for (int c = 0; c < 8; ++c) sd[line][F_PP + c][lane] = Pp[c];
        const bool in = active && s >= 0 && s < n;
#pragma unroll
        for (int c = 0; c < 8; ++c) sl[line][c][lane] = in ? lam[c * N + ibase + (long long)s * istride] : 0.0;
    }
    __syncthreads();

    auto prim_at = [&](int q, double* Pq) {
#pragma unroll
        for (int c = 0; c < 8; ++c) Pq[c] = sd[line][c][q];
    };
    auto lamPp = [&](int q) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += sl[line][c][q] * sd[line][F_PP + c][q];
        return s;
    };
    // B~ pair value of slots (qa, qb)
    auto bpair = [&](int qa, int qb) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j)
            s += 0.25 * (sd[line][F_A + 1 + j][qa] + sd[line][F_A + 1 + j][qb]) * (sd[line][5 + j][qa] + sd[line][5 + j][qb]);
        return s;
    };

    // ---- pairs (s', s'+n), s' = s0 - 3 + lane, slot of s' = lane + 2
    const int o = lane;                            // output lane: position s0 + o, slot o + 5
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    {
        const int ql = lane + 2;
        double Pl[8], al[NA];
        if (lane < QSEG + 3) {
            prim_at(ql, Pl);
#pragma unroll
            for (int c = 0; c < NA; ++c) al[c] = sd[line][F_A + c][ql];
        }
#pragma unroll 1
        for (int nn = 1; nn <= PO; ++nn) {
            double gl[8], gr[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) { gl[c] = 0.0; gr[c] = 0.0; }
            if (active && lane < QSEG + 3) {
                const int qr = ql + nn;
                double w[8];
                bool any = false;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    w[c] = alpha_pn(PO, nn) * idxi * (sl[line][c][qr] - sl[line][c][ql]);
                    any |= w[c] != 0.0;
                }
                double ar[NA];
#pragma unroll
                for (int c = 0; c < NA; ++c) ar[c] = sd[line][F_A + c][qr];
                if (any) {
                    double Pr[8];
                    prim_at(qr, Pr);
                    pair_vjp_rmhd<DIM>(G, Pl, Pr, al, ar, w, gl, gr);
                }
                // source pair B~: linear in B_j of both nodes
                const double wB = alpha_pn(PO, nn) * idxi * (lamPp(qr) - lamPp(ql));
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    const double cb = 0.25 * wB * (al[1 + j] + ar[1 + j]);
                    gl[5 + j] += cb;
                    gr[5 + j] += cb;
                }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                buf[line][nn - 1][c][lane] = gl[c];
                buf[line][3 + nn - 1][c][lane] = gr[c];
            }
        }
    }
    __syncthreads();
    if (o < QSEG) {
#pragma unroll
        for (int nn = 1; nn <= PO; ++nn)
#pragma unroll
            for (int c = 0; c < 8; ++c)
                acc[c] += buf[line][nn - 1][c][o + 3] + buf[line][3 + nn - 1][c][o + 3 - nn];
    }

    // ---- entropy-variable cotangents of the stencil states from the faces
    double gV[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) gV[c] = 0.0;
    if (ES) {
        __syncthreads();
        // faces f = s0 - 3 + lane (stencil slots lane + 3 - PO .. lane + 2 + PO, nodes i, i+1 at
        // lane + 2, lane + 3); stencil node j at slot lane + 3 - PO + j, CI = PO - 1 the node i
        constexpr int NS = 2 * PO, CI = PO - 1, J0 = 3 - PO;
        double gw[NS][8];
#pragma unroll
        for (int j = 0; j < NS; ++j)
#pragma unroll
            for (int c = 0; c < 8; ++c) gw[j][c] = 0.0;
        if (active && lane < QSEG + 5) {
            double z[8];
            bool any = false;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                z[c] = 0.5 * idxi * (sl[line][c][lane + 2] - sl[line][c][lane + 3]);
                any |= z[c] != 0.0;
            }
            if (any) {
                double P2[8], P3[8], al[NA], ar[NA];
                prim_at(lane + 2, P2);
                prim_at(lane + 3, P3);
#pragma unroll
                for (int c = 0; c < NA; ++c) { al[c] = sd[line][F_A + c][lane + 2]; ar[c] = sd[line][F_A + c][lane + 3]; }
                // the eigen-structure of this face (held at its forward value) from
                // k_face_eigen_rmhd: face f = p + 1 of line lid, p = s0 - 3 + lane
                double T[3][3], TV[NS][8], at, L, Rc[8][8];
                face_frame_rmhd<DIM>(G, P2, P3, al, ar, T, TV[CI], TV[CI + 1], at, L);
                const double* ef = eig + lid * (n + 1) + (s0 - 2 + lane);
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int i = 0; i < 8; ++i) Rc[k][i] = ef[(k * 8 + i) * enf];
                const double lhat = ef[64 * enf];
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    if (j == CI || j == CI + 1) continue;
                    double Pj[8], V[8];
                    prim_at(lane + J0 + j, Pj);
                    const StateRMHD<double> st = rmhd_state<double>(G, Pj);
                    rmhd_entropy_vars<double>(G, st, V);
                    rotate8<false>(T, V, TV[j]);
                }
                double tv2 = 0.0, tv3 = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) { tv2 = fmax(tv2, fabs(TV[CI][c])); tv3 = fmax(tv3, fabs(TV[CI + 1][c])); }
                const double tvmax = tv2 + tv3;
                // d = lhat T^T dd: cotangent of dd
                double gdd[8];
                rotate8<false>(T, z, gdd);
#pragma unroll
                for (int c = 0; c < 8; ++c) gdd[c] *= lhat;
                double gTV[NS][8];
#pragma unroll
                for (int j = 0; j < NS; ++j)
#pragma unroll
                    for (int c = 0; c < 8; ++c) gTV[j][c] = 0.0;
#pragma unroll 1
                for (int k = 0; k < 8; ++k) {
                    const double* r = Rc[k];
                    double vt[NS];
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        double s = 0.0;
#pragma unroll
                        for (int c = 0; c < 8; ++c) s += r[c] * TV[j][c];
                        vt[j] = s;
                    }
                    double jw;
                    if (PO == 3)
                        jw = weno5(vt[5], vt[4], vt[3], vt[2], vt[1], eps) -
                             weno5(vt[0], vt[1], vt[2], vt[3], vt[4], eps);
                    else
                        jw = weno3(vt[3], vt[2], vt[1], eps) - weno3(vt[0], vt[1], vt[2], eps);
                    const double jp = vt[CI + 1] - vt[CI];
                    double r1 = 0.0;
#pragma unroll
                    for (int c = 0; c < 8; ++c) r1 += fabs(r[c]);
                    if (jw * jp > 0.0 && fabs(jp) > RealTraits<double>::ytol * r1 * tvmax) {
                        double gjw = 0.0;
#pragma unroll
                        for (int c = 0; c < 8; ++c) gjw += gdd[c] * r[c];
                        double djw[NS];
                        if (PO == 3) {
                            double gp[5], gm[5];
                            weno5_grad_m(vt[5], vt[4], vt[3], vt[2], vt[1], eps, gp);
                            weno5_grad_m(vt[0], vt[1], vt[2], vt[3], vt[4], eps, gm);
                            djw[0] = -gm[0];
                            djw[1] = gp[4] - gm[1];
                            djw[2] = gp[3] - gm[2];
                            djw[3] = gp[2] - gm[3];
                            djw[4] = gp[1] - gm[4];
                            djw[NS - 1] = gp[0];
                        } else {
                            double gp[3], gm[3];
                            weno3_grad_m(vt[3], vt[2], vt[1], eps, gp);
                            weno3_grad_m(vt[0], vt[1], vt[2], eps, gm);
                            djw[0] = -gm[0];
                            djw[1] = gp[2] - gm[1];
                            djw[2] = gp[1] - gm[2];
                            djw[NS - 1] = gp[0];
                        }
#pragma unroll
                        for (int j = 0; j < NS; ++j) {
                            const double gv = gjw * djw[j];
#pragma unroll
                            for (int c = 0; c < 8; ++c) gTV[j][c] += gv * r[c];
                        }
                    }
                }
                // TV_j = T V_j: cotangent of V_j
#pragma unroll
                for (int j = 0; j < NS; ++j) rotate8<true>(T, gTV[j], gw[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < NS; ++j)
#pragma unroll
            for (int c = 0; c < 8; ++c) buf[line][j][c][lane] = gw[j][c];
        __syncthreads();
        if (o < QSEG) {
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int c = 0; c < 8; ++c) gV[c] += buf[line][j][c][o + 5 - J0 - j];
        }
    }

    // ---- node terms: the Godunov-Powell source (Phi'(P_s) against the B~
    // differences) and the entropy-variable chain, one dual pass over P_s
    const int s = s0 + o;
    if (active && o < QSEG && s < s_end) {
        const int q = o + 5;
        double dB = 0.0;
#pragma unroll
        for (int nn = 1; nn <= PO; ++nn) dB += alpha_pn(PO, nn) * (bpair(q, q + nn) - bpair(q - nn, q));
        dB *= idxi;
        double lq[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) lq[c] = sl[line][c][q];
        using D = Dual<8>;
        D Pd[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) Pd[c] = D::seed(sd[line][c][q], c);
        const StateRMHD<D> st = rmhd_state<D>(G, Pd);
        D Pp[8], V[8];
        rmhd_phi_prime<D>(st, Pp);
        if (ES) rmhd_entropy_vars<D>(G, st, V);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) t -= dB * lq[c] * Pp[c].d[k];
            if (ES) {
#pragma unroll
                for (int c = 0; c < 8; ++c) t += gV[c] * V[c].d[k];
            }
            acc[k] += t;
        }
        const long long idx = pbase + (long long)s * pstride;
#pragma unroll
        for (int c = 0; c < 8; ++c) gout[c * P + idx] = acc[c];
    }
}

template <int DIM, bool ES, int PO>
__global__ void __launch_bounds__(128) k_residual_vjp_rmhd(GridDev g, double G, double eps,
                                                           const double* __restrict__ prim,
                                                           const double* __restrict__ met,
                                                           const double* __restrict__ lam,
                                                           double* __restrict__ gdir, AdjPlanM pl,
                                                           const double* __restrict__ eig, FaceEigPlan fp) {
    __shared__ AdjLDSM<DIM> lds;
    const long long slab = 8LL * g.pnodes;
    int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    if (b < pl.nblk[0]) {
        residual_vjp_segment_rmhd<DIM, 0, ES, PO>(g, G, eps, prim, met, lam, gdir, b, pl.nseg[0], pl.nlines[0], lds,
                                              eig + fp.base[0], fp.nlines[0] * fp.nface[0]);
        return;
    }
    b -= pl.nblk[0];
    if (DIM == 2 || b < pl.nblk[1]) {
        residual_vjp_segment_rmhd<DIM, 1, ES, PO>(g, G, eps, prim, met, lam, gdir + slab, b, pl.nseg[1], pl.nlines[1],
                                              lds, eig + fp.base[1], fp.nlines[1] * fp.nface[1]);
        return;
    }
    b -= pl.nblk[1];
    if (DIM == 3)
        residual_vjp_segment_rmhd<DIM, 2, ES, PO>(g, G, eps, prim, met, lam, gdir + 2 * slab, b, pl.nseg[2],
                                              pl.nlines[2], lds, eig + fp.base[2], fp.nlines[2] * fp.nface[2]);
}

// Solve A^T y = b (8 x 8) by Gaussian elimination with partial pivoting on A^T.
__device__ __forceinline__ void solve_transposed8(const double A[8][8], const double* b, double* y) {
    double Mx[8][9];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
        for (int c = 0; c < 8; ++c) Mx[r][c] = A[c][r];
        Mx[r][8] = b[r];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int piv = k;
        double best = fabs(Mx[k][k]);
#pragma unroll
        for (int r = k + 1; r < 8; ++r)
            if (fabs(Mx[r][k]) > best) { best = fabs(Mx[r][k]); piv = r; }
#pragma unroll
        for (int r = k + 1; r < 8; ++r) {
            if (r == piv) {
#pragma unroll
                for (int c = 0; c <= 8; ++c) { const double t = Mx[k][c]; Mx[k][c] = Mx[r][c]; Mx[r][c] = t; }
            }
        }
        const double ik = 1.0 / Mx[k][k];
#pragma unroll
        for (int r = k + 1; r < 8; ++r) {
            const double f = Mx[r][k] * ik;
#pragma unroll
            for (int c = k; c <= 8; ++c) Mx[r][c] -= f * Mx[k][c];
        }
    }
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        double s = Mx[k][8];
#pragma unroll
        for (int c = k + 1; c < 8; ++c) s -= Mx[k][c] * y[c];
        y[k] = s / Mx[k][k];
    }
}

// Pull a primitive cotangent back through con2prim by the implicit-function rule,
// (dUbar/dP)^T y = g_P with dUbar/dP by dual numbers (U(P) of eq. RMHDdiv2), then
// g_Ucurv = y / J, g_J = -(y . Ucurv) / J^2.  FOLD: g_P is the residual VJP's padded
// cotangent by direction, ghost cotangents folded onto the interior nodes they
// copy; otherwise an interior field of 8 components.
template <int DIM, bool FOLD>
__global__ void __launch_bounds__(256) k_fold_con2prim_vjp_rmhd(GridDev g, double G,
                                                                const double* __restrict__ prim,
                                                                const double* __restrict__ U,
                                                                const double* __restrict__ J,
                                                                const double* __restrict__ gsrc,
                                                                double* __restrict__ gU,
                                                                double* __restrict__ gJ) {
    int i, j, k;
    if (!box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) return;
    const long long P = g.pnodes, N = g.nodes;
    const long long slab = 8LL * P;
    const long long pi0 = pidx(g, i, j, k);
    const long long t = iidx(g, i, j, k);
    double gP[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) gP[c] = FOLD ? 0.0 : gsrc[c * N + t];
    const int ijk[3] = {i, j, k};
    const double* gdir = gsrc;
#pragma unroll
    for (int d = 0; d < (FOLD ? DIM : 0); ++d) {
        const double* gd = gdir + d * slab;
        const long long str = d == 0 ? 1 : (d == 1 ? (long long)g.P[0] : (long long)g.P[0] * g.P[1]);
        const int n = g.n[d], me = ijk[d];
#pragma unroll
        for (int c = 0; c < 8; ++c) gP[c] += gd[c * P + pi0];
#pragma unroll
        for (int q = 0; q < 2 * NG; ++q) {
            const int gpos = q < NG ? q - NG : n + (q - NG);
            if (map_sol(gpos, n, g.bc[d]) == me) {
                const long long gi = pi0 + (long long)(gpos - me) * str;
#pragma unroll
                for (int c = 0; c < 8; ++c) gP[c] += gd[c * P + gi];
            }
        }
    }
    using D = Dual<8>;
    D Pd[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) Pd[c] = D::seed(prim[c * P + pi0], c);
    const StateRMHD<D> st = rmhd_state<D>(G, Pd);
    D Ud[8];
    rmhd_cons<D>(st, Ud);
    double A[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) A[r][c] = Ud[r].d[c];
    double y[8];
    solve_transposed8(A, gP, y);
    const double iJ = 1.0 / J[t];
    double gj = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        gU[c * N + t] = y[c] * iJ;
        gj -= y[c] * U[c * N + t];
    }
    gJ[t] = gj * iJ * iJ;
}

// VJP of Ucurv = J U(P) at the interior nodes: g_P = J (dU/dP)^T g_Ucurv with dU/dP
// by dual numbers, g_J = U(P) . g_Ucurv (gJ may be null).  prim: interior, 8 comps.
__global__ void __launch_bounds__(256) k_prim2con_vjp_rmhd(GridDev g, double G,
                                                           const double* __restrict__ prim,
                                                           const double* __restrict__ J,
                                                           const double* __restrict__ gUc,
                                                           double* __restrict__ gP,
                                                           double* __restrict__ gJ) {
    const long long t = gtid();
    if (t >= g.nodes) return;
    const long long N = g.nodes;
    using D = Dual<8>;
    D Pd[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) Pd[c] = D::seed(prim[c * N + t], c);
    const StateRMHD<D> st = rmhd_state<D>(G, Pd);
    D Ud[8];
    rmhd_cons<D>(st, Ud);
    double gu[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) gu[r] = gUc[r * N + t];
    const double Jv = J[t];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) acc += Ud[r].d[c] * gu[r];
        gP[c * N + t] = Jv * acc;
    }
    if (gJ != nullptr) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) acc += Ud[r].v * gu[r];
        gJ[t] = acc;
    }
}

FaceEigPlan face_eig_plan(const GridDev& g) {
    FaceEigPlan fp{};
    long long base = 0;
    for (int d = 0; d < g.dim; ++d) {
        long long nl = 1;
        for (int a = 0; a < g.dim; ++a)
            if (a != d) nl *= g.n[a];
        fp.base[d] = base;
        fp.nlines[d] = nl;
        fp.nface[d] = g.n[d] + 1;
        fp.nthreads[d] = nl * fp.nface[d];
        base += (long long)NEIG * fp.nthreads[d];
    }
    return fp;
}

template <int DIM>
static void residual_vjp_all_rmhd(const es_ctx* c, const double* prim, const double* met, const double* lam,
                                  double* gdir, hipStream_t s) {
    const GridDev& g = c->g;
    AdjPlanM pl{};
    long long nb = 0;
    for (int d = 0; d < DIM; ++d) {
        pl.nseg[d] = (g.n[d] + 2 * NG + QSEG - 1) / QSEG;
        long long nl = 1;
        for (int a = 0; a < DIM; ++a)
            if (a != d) nl *= g.n[a];
        pl.nlines[d] = nl;
        pl.nblk[d] = (int)(((nl + QLINES - 1) / QLINES) * pl.nseg[d]);
        nb += pl.nblk[d];
    }
    const double G = c->scheme.gamma, eps = c->scheme.weno_eps;
    const unsigned thr = 64 * QLINES;
    const FaceEigPlan fp = face_eig_plan(g);
    if (c->scheme.dissipation != 0) {
        long long nt = 0;
        for (int d = 0; d < DIM; ++d) nt += fp.nthreads[d];
        k_face_eigen_rmhd<DIM><<<(unsigned)((nt + 63) / 64), 64, 0, s>>>(g, G, prim, met, c->adj_eig, fp);
        if (c->scheme.order_p == 2)
            k_residual_vjp_rmhd<DIM, true, 2><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl,
                                                                            c->adj_eig, fp);
        else
            k_residual_vjp_rmhd<DIM, true, 3><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl,
                                                                            c->adj_eig, fp);
    } else if (c->scheme.order_p == 2) {
        k_residual_vjp_rmhd<DIM, false, 2><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl,
                                                                         nullptr, fp);
    } else {
        k_residual_vjp_rmhd<DIM, false, 3><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl,
                                                                         nullptr, fp);
    }
}

}  // namespace

size_t face_eig_doubles_rmhd(const es_ctx* c) {
    const FaceEigPlan fp = face_eig_plan(c->g);
    size_t n = 0;
    for (int d = 0; d < c->g.dim; ++d) n += (size_t)NEIG * (size_t)fp.nthreads[d];
    return n;
}

hipError_t launch_residual_fold_vjp_rmhd(const es_ctx* c, const double* U, const double* J, const double* met,
                                         const double* lam, double* gU, double* gJ, hipStream_t s) {
    const GridDev& g = c->g;
    if (g.dim == 2) residual_vjp_all_rmhd<2>(c, c->prim, met, lam, c->gdir, s);
    else residual_vjp_all_rmhd<3>(c, c->prim, met, lam, c->gdir, s);
    const dim3 gr = box_grid(g.n[0], g.n[1], g.n[2]);
    if (g.dim == 2)
        k_fold_con2prim_vjp_rmhd<2, true><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, c->gdir, gU, gJ);
    else
        k_fold_con2prim_vjp_rmhd<3, true><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, c->gdir, gU, gJ);
    return hipGetLastError();
}

hipError_t launch_con2prim_vjp_rmhd(const es_ctx* c, const double* U, const double* J, const double* gprim,
                                    double* gU, double* gJ, hipStream_t s) {
    const GridDev& g = c->g;
    const dim3 gr = box_grid(g.n[0], g.n[1], g.n[2]);
    if (g.dim == 2)
        k_fold_con2prim_vjp_rmhd<2, false><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, gprim, gU, gJ);
    else
        k_fold_con2prim_vjp_rmhd<3, false><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, gprim, gU, gJ);
    return hipGetLastError();
}

hipError_t launch_prim2con_vjp_rmhd(const es_ctx* c, const double* prim, const double* J, const double* gUc,
                                    double* gprim, double* gJ, hipStream_t s) {
    const GridDev& g = c->g;
    k_prim2con_vjp_rmhd<<<grid_for(g.nodes), TPB, 0, s>>>(g, c->scheme.gamma, prim, J, gUc, gprim, gJ);
    return hipGetLastError();
}

}  // namespace es
