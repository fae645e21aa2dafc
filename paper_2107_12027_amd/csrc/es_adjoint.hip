// Hand-written adjoint (vector-Jacobian products) of the residual and of one
// SSP-RK3 step, FP64.
//
// The step is reversed stage by stage from checkpoints of the stage states.
// Within a stage the cotangent lambda of the residual L(U, J) = residual(
// con2prim(U / J), metrics) is pulled back in three parts:
//   * residual: per direction, the transposed stencil of eq. ECFlux_O2p and of
//     the dissipation differences -- each two-point flux F(s, s+n) receives
//     w = alpha_n / dxi (lambda_{s+n} - lambda_s), each face dissipation d_{f+1/2}
//     receives z = (lambda_f - lambda_{f+1}) / (2 dxi) -- times the local
//     Jacobians, gathered per node (no atomics, deterministic);
//   * ghost folding: cotangents of ghost nodes go to the interior nodes they copy;
//   * con2prim by the implicit-function rule: dP/dU = (dU/dP)^{-1}, so the state
//     cotangent solves (dU/dP)^T y = g_P at every node.
// Local Jacobians: the two-point flux by a hand-written backward sweep
// (es_pair_vjp.h, both nodes at once); the face dissipation by reverse accumulation
// through the projections, WENO (its gradient written out) and the final
// combination, and a backward sweep through the face eigen-structure
// (es_eigen_vjp.h) to the face entropy variables.  The sign switch Y, the branch
// of lambda^, the time step, the mesh and its velocity are held fixed.
#include <math.h>

#include "es_internal.h"
#include "es_launch.h"
#include "es_rhd.h"
#include "es_dual.h"
#include "es_pair_vjp.h"
#include "es_eigen_vjp.h"

namespace es {

namespace {

// Cotangents g[j] (j = 0..5, primitive slots) of the stencil states of one face
// dissipation d (face_diss_rhd) for the cotangent z of d.
// Gradient of the WENO5-JS value weno5(a, b, c, d, e) with respect to its five
// inputs, from the weights w_k = d_k / (eps + beta_k)^2 written out: with
// S = sum_k w_k and v = sum_k w_k q_k / (6 S) (q_k the six-fold candidate values),
// dv = [sum_k w_k dq_k + sum_k (q_k - 6 v) dw_k] / (6 S) and
// dw_k = -2 w_k dbeta_k / (eps + beta_k).
__device__ __forceinline__ void weno5_grad(double a, double b, double c, double d, double e, double eps,
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
    const double v6 = (w0 * q0 + w1 * q1 + w2 * q2) / S;      // 6 v
    // c_k dbeta_k with c_k = -2 w_k (q_k - 6 v) / (eps + beta_k), split over t_k and s_k
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

// Gradient of the WENO3 value weno3(a, b, c) = (w0 q0 + w1 q1) / (2 S) with
// q0 = 3b - a, q1 = b + c, w_k = d_k / e_k^2 (d = 1/3, 2/3), e0 = eps + (b - a)^2,
// e1 = eps + (c - b)^2, S = w0 + w1 (any common factor of the w_k cancels):
// dv = [w0 dq0 + w1 dq1 + (q0 - 2v) dw0 + (q1 - 2v) dw1] / (2 S), dw_k = -2 w_k de_k / e_k.
__device__ __forceinline__ void weno3_grad(double a, double b, double c, double eps, double* gr) {
    const double q0 = 3.0 * b - a, q1 = b + c;
    const double e0 = eps + (b - a) * (b - a), e1 = eps + (c - b) * (c - b);
    const double w0 = (1.0 / 3.0) * (e1 * e1), w1 = (2.0 / 3.0) * (e0 * e0);   // both times e0^2 e1^2
    const double S = w0 + w1;
    const double v2 = (w0 * q0 + w1 * q1) / S;                                   // 2 v
    const double c0 = -4.0 * w0 * (q0 - v2) * (b - a) / e0;                     // times (db - da)
    const double c1 = -4.0 * w1 * (q1 - v2) * (c - b) / e1;                     // times (dc - db)
    const double i2S = 1.0 / (2.0 * S);
    gr[0] = (-w0 - c0) * i2S;
    gr[1] = (3.0 * w0 + w1 + c0 - c1) * i2S;
    gr[2] = (w1 + c1) * i2S;
}

// P: the order parameter p (stencil of 2p nodes, WENO of order 2p - 1).
// gtv(j, c): the accumulator of the cotangent of the rotated entropy variable c of
// stencil node j (a slot of the caller's LDS, the same slot that out(j, c, .)
// later receives the primitive cotangent in); keeping these 2p x M sums out of
// the registers is what lets the 3D kernel hold its column loop without spills.
// gra(q, c): the cotangent of entry c of eigenvector column q, likewise an LDS
// slot of the caller (it lives from the column loop through the eigen-structure
// tangents, whose dual-number arithmetic needs the registers).
template <int DIM, int P, typename NodeFn, typename Sync, typename GT, typename GRA, typename Out>
__device__ void face_vjp_rhd(double G, double eps, NodeFn&& node, Sync&& sync, const double* al,
                             const double* ar, const double* z, GT&& gtv, GRA&& gra, Out&& out) {
    constexpr int M = DIM + 2;
    constexpr int NS = 2 * P, CI = P - 1;
    const double at = 0.5 * (al[0] + ar[0]);
    double ax[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < DIM; ++j) ax[j] = 0.5 * (al[1 + j] + ar[1 + j]);
    const double L = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    const double iL = frcp(L);
    double nrm[3] = {ax[0] * iL, ax[1] * iL, ax[2] * iL};
    double T[3][3];
    rotation<DIM>(nrm, T);
    const double c0 = G / (G - 1.0), c1 = 1.0 / (G - 1.0);

    // (the stencil states are read through node(j) here and again at the end, so
    // that they need not stay in registers in between)
    double TV[NS][M];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const NodeRHD<DIM> q = node(j);
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

    // forward: the eigen-structure as a matrix (column q in Rm[q])
    double Rm[M][M];
    const double lhat = face_eigen_columns<DIM>(G, TV[CI], TV[CI + 1], at, L, [&](const double* r, int q) {
#pragma unroll
        for (int c = 0; c < M; ++c) Rm[q][c] = r[c];
    });
    double tv2 = 0.0, tv3 = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) { tv2 = fmax(tv2, fabs(TV[CI][c])); tv3 = fmax(tv3, fabs(TV[CI + 1][c])); }
    const double tvmax = tv2 + tv3;

    // z in the rotated frame: d = lhat T^T dd, so d(z.d)/d(dd) = lhat T z
    double zr[M];
    zr[0] = z[0];
    zr[M - 1] = z[M - 1];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) s += T[a][b] * z[1 + b];
        zr[1 + a] = s;
    }

    double dd[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        dd[c] = 0.0;
#pragma unroll
        for (int j = 0; j < NS; ++j) gtv(j, c) = 0.0;
    }
#pragma unroll 1
    for (int q = 0; q < M; ++q) {
        // column q and its cotangent row through selects (no dynamic register indexing)
        double r[M], gRq[M];
#pragma unroll
        for (int c = 0; c < M; ++c) { r[c] = 0.0; gRq[c] = 0.0; }
#pragma unroll
        for (int qq = 0; qq < M; ++qq)
#pragma unroll
            for (int c = 0; c < M; ++c) r[c] = qq == q ? Rm[qq][c] : r[c];
        double vt[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) s += r[c] * TV[j][c];
            vt[j] = s;
        }
        // the jump and its switch exactly as in the forward dissipation
        double jwv;
        if (P == 3)
            jwv = weno5(vt[5], vt[4], vt[3], vt[2], vt[1], eps) - weno5(vt[0], vt[1], vt[2], vt[3], vt[4], eps);
        else
            jwv = weno3(vt[3], vt[2], vt[1], eps) - weno3(vt[0], vt[1], vt[2], eps);
        const double jp = vt[CI + 1] - vt[CI];
        double r1 = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) r1 += fabs(r[c]);
        if (jwv * jp > 0.0 && fabs(jp) > RealTraits<double>::ytol * r1 * tvmax) {
            // d(jw)/d(vt_j): the upwind-from-the-right value minus the one from the left
            double djw[NS];
            if (P == 3) {
                double gp[5], gm[5];
                weno5_grad(vt[5], vt[4], vt[3], vt[2], vt[1], eps, gp);
                weno5_grad(vt[0], vt[1], vt[2], vt[3], vt[4], eps, gm);
                djw[0] = -gm[0];
                djw[1] = gp[4] - gm[1];
                djw[2] = gp[3] - gm[2];
                djw[3] = gp[2] - gm[3];
                djw[4] = gp[1] - gm[4];
                djw[NS - 1] = gp[0];
            } else {
                double gp[3], gm[3];
                weno3_grad(vt[3], vt[2], vt[1], eps, gp);
                weno3_grad(vt[0], vt[1], vt[2], eps, gm);
                djw[0] = -gm[0];
                djw[1] = gp[2] - gm[1];
                djw[2] = gp[1] - gm[2];
                djw[NS - 1] = gp[0];
            }
            double rz = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) { dd[c] += jwv * r[c]; rz += r[c] * zr[c]; }
            const double gjw = lhat * rz;
#pragma unroll
            for (int c = 0; c < M; ++c) gRq[c] += lhat * jwv * zr[c];
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const double gv = gjw * djw[j];
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    gtv(j, c) += gv * r[c];
                    gRq[c] += gv * TV[j][c];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < M; ++c) gra(q, c) = gRq[c];
    }
    double glhat = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) glhat += zr[c] * dd[c];

    // rotated entropy variables -> primitive (rho, u, p) of stencil node j, handed
    // to out(j, c, value)
    auto to_prim = [&](int j) {
        const NodeRHD<DIM> q = node(j);
        double gt[M];              // read all of node j's sums before out() reuses the slots
#pragma unroll
        for (int c = 0; c < M; ++c) gt[c] = gtv(j, c);
        const double ip = 1.0 / q.p, irho = 1.0 / q.rho;
        double su = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double tu = 0.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) tu += T[a][b] * q.u[b];
            su += gt[1 + a] * tu;
        }
        const double sbu = q.beta * su;
        double res[M];
        res[0] = gt[0] * ((1.0 + c1) * irho + ip) + su * ip - gt[M - 1] * q.W * ip;
        res[M - 1] = -gt[0] * (c1 + q.beta) * ip - sbu * ip + gt[M - 1] * q.beta * q.W * ip;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) s += T[a][b] * gt[1 + a];
            res[1 + b] = q.beta * s - gt[M - 1] * q.beta * q.u[b] / q.W;
        }
#pragma unroll
        for (int c = 0; c < M; ++c) out(j, c, res[c]);
    };
    // the outer stencil nodes are complete before the eigen-structure tangents
    sync();
#pragma unroll
    for (int j = 0; j < NS; ++j)
        if (j != CI && j != CI + 1) to_prim(j);

    // face eigen-structure: one backward sweep from the column and lambda^
    // cotangents to the face entropy variables, which reach nodes i and i+1
    // through the face mean
    double Vb[M], gVb[M];
#pragma unroll
    for (int c = 0; c < M; ++c) Vb[c] = 0.5 * (TV[CI][c] + TV[CI + 1][c]);
    face_eigen_vjp<DIM>(G, Vb, at, L, gra, glhat, gVb);
#pragma unroll
    for (int c = 0; c < M; ++c) {
        gtv(CI, c) += 0.5 * gVb[c];
        gtv(CI + 1, c) += 0.5 * gVb[c];
    }
    sync();
    to_prim(CI);
    to_prim(CI + 1);
}

// ---------------------------------------------------------------------------
// residual VJP: one wavefront per segment of padded positions along a line
// ---------------------------------------------------------------------------
constexpr int ASEG = 54;                  // output positions per segment
constexpr int AHALO = 5;                  // state halo each side
constexpr int ALOAD = ASEG + 2 * AHALO;   // 64 loaded slots
constexpr int ALINES = 2;                 // segments per block

template <int DIM>
struct AdjLDS {
    static constexpr int NU = DIM, M = DIM + 2, NA = DIM + 1, NF = 6 + NU + NA;
    double sd[ALINES][NF][ALOAD];
    double lam[ALINES][M][ALOAD];
    double buf[ALINES][6][M][64];
    double gr[ALINES][M][M][64];     // cotangents of the face eigenvector columns
};

struct AdjPlan {
    int flat[3];          // flat (1) or aligned (0) segment layout
    int nsl[3];           // segments per line of the aligned layout
    int nseg[3];
    int nblk[3];
    long long nlines[3];
};

template <int DIM, int DIR, bool ES, int PO>
__device__ __forceinline__ void residual_vjp_segment(const GridDev& g, double G, double eps,
                                                     const double* __restrict__ prim,
                                                     const double* __restrict__ met,
                                                     const double* __restrict__ lam,
                                                     double* __restrict__ gout, int blk, int nseg,
                                                     long long nlines, bool flat, int nsl, AdjLDS<DIM>& lds) {
    constexpr int NU = DIM, M = DIM + 2, NA = DIM + 1;
    constexpr int F_RHO = 0, F_P = 1, F_BETA = 2, F_W = 3, F_LR = 4, F_LB = 5, F_U = 6, F_A = 6 + NU;
    auto& sd = lds.sd;
    auto& sl = lds.lam;
    auto& buf = lds.buf;
    const int lane = threadIdx.x & 63;
    const int line = threadIdx.x >> 6;
    // segment w of sequence `line` (the lines dealt to ALINES sequences, es_seq.h)
    // outputs ASEG consecutive positions.  Flat layout: the padded node sequences
    // (n + 2 NG nodes per line) laid end to end, a pair or face across two lines
    // joining ghost nodes of both, whose residual cotangents are zero, so that it
    // contributes nothing; aligned: ceil((n + 2 NG) / ASEG) segments per line.  A
    // segment past the sweep's last one runs with no active lane (the block
    // synchronises).
    const long long w = blk;
    const int n = g.n[DIR];
    const int PL = n + 2 * NG;
    const long long pstride = DIR == 0 ? 1 : (DIR == 1 ? (long long)g.P[0] : (long long)g.P[0] * g.P[1]);
    const long long istride = DIR == 0 ? 1 : (DIR == 1 ? (long long)g.n[0] : (long long)g.n[0] * g.n[1]);
    const long long P = g.pnodes, N = g.nodes;
    const double idxi = 1.0 / g.dxi[DIR];
    // line (nlines if none) and padded coordinate s of sequence position
    // w ASEG - AHALO + q, and the padded / interior index of the line's node 0
    const int nf = DIR == 0 ? g.n[1] : g.n[0];
    const SeqBase sb = flat ? seq_base(w * ASEG - AHALO, PL, NG, nf, ALINES, line)
                            : seq_base_aligned(w, nsl, ASEG, AHALO, NG, nf, ALINES, line);
    auto locate = [&](int q, long long& lid, int& s, long long& pbase, long long& ibase) {
        int fa, fb;
        seq_at(sb, q, flat, PL, NG, nf, ALINES, line, lid, s, fa, fb);
        if (w >= nseg || lid < 0 || s < -NG || s >= n + NG) lid = nlines;
        const int ci = DIR == 0 ? 0 : fa, cj = DIR == 0 ? fa : (DIR == 1 ? 0 : fb), ck = DIR == 2 ? 0 : fb;
        pbase = pidx(g, ci, cj, ck);
        ibase = iidx(g, ci, cj, ck);
    };
    const bool active = w < nseg;

    // ---- states (positions w ASEG - 5 .. w ASEG + 58) and residual cotangents
    {
        long long lid, pbase, ibase;
        int s;
        locate(lane, lid, s, pbase, ibase);
        double rho = 1.0, p = 1.0, lr = 0.0, lb = 0.0, u[NU], a[NA];
#pragma unroll
        for (int c = 0; c < NU; ++c) u[c] = 0.0;
#pragma unroll
        for (int c = 0; c < NA; ++c) a[c] = c == 1 ? 1.0 : 0.0;
        if (lid < nlines) {
            const long long idx = pbase + (long long)s * pstride;
            rho = prim[idx];
#pragma unroll
            for (int c = 0; c < NU; ++c) u[c] = prim[(1 + c) * P + idx];
            p = prim[(M - 1) * P + idx];
            lr = prim[M * P + idx];
            lb = prim[(M + 1) * P + idx];
#pragma unroll
            for (int c = 0; c < NA; ++c) a[c] = met[(DIR * NA + c) * P + idx];
        }
        double uu = 0.0;
#pragma unroll
        for (int c = 0; c < NU; ++c) uu += u[c] * u[c];
        sd[line][F_RHO][lane] = rho;
        sd[line][F_P][lane] = p;
        sd[line][F_BETA][lane] = rho / p;
        sd[line][F_W][lane] = sqrt(1.0 + uu);
        sd[line][F_LR][lane] = lr;
        sd[line][F_LB][lane] = lb;
#pragma unroll
        for (int c = 0; c < NU; ++c) sd[line][F_U + c][lane] = u[c];
#pragma unroll
        for (int c = 0; c < NA; ++c) sd[line][F_A + c][lane] = a[c];
        const bool in = lid < nlines && s >= 0 && s < n;
#pragma unroll
        for (int c = 0; c < M; ++c) sl[line][c][lane] = in ? lam[c * N + ibase + (long long)s * istride] : 0.0;
    }
    __syncthreads();

    auto prim_at = [&](int q, double* Pq) {
        Pq[0] = sd[line][F_RHO][q];
#pragma unroll
        for (int c = 0; c < NU; ++c) Pq[1 + c] = sd[line][F_U + c][q];
        Pq[M - 1] = sd[line][F_P][q];
    };
    auto node_at = [&](int q) {
        NodeRHD<NU> nd;
        nd.rho = sd[line][F_RHO][q];
        nd.p = sd[line][F_P][q];
        nd.beta = sd[line][F_BETA][q];
        nd.W = sd[line][F_W][q];
        nd.lr = sd[line][F_LR][q];
        nd.lb = sd[line][F_LB][q];
#pragma unroll
        for (int c = 0; c < NU; ++c) nd.u[c] = sd[line][F_U + c][q];
        return nd;
    };

    // ---- pairs (s', s'+n), s' = w ASEG - 3 + lane, slot of s' = lane + 2
    const int o = lane;                            // output lane: position w ASEG + o
    double acc[M];
#pragma unroll
    for (int c = 0; c < M; ++c) acc[c] = 0.0;
    {
        const int ql = lane + 2;
        double Pl[M], al[NA];
        if (lane < ASEG + 3) {
            prim_at(ql, Pl);
#pragma unroll
            for (int c = 0; c < NA; ++c) al[c] = sd[line][F_A + c][ql];
        }
#pragma unroll 1
        for (int nn = 1; nn <= PO; ++nn) {
            double gl[M], gr[M];
#pragma unroll
            for (int c = 0; c < M; ++c) { gl[c] = 0.0; gr[c] = 0.0; }
            if (active && lane < ASEG + 3) {
                const int qr = ql + nn;
                double w[M];
                bool any = false;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    w[c] = alpha_pn(PO, nn) * idxi * (sl[line][c][qr] - sl[line][c][ql]);
                    any |= w[c] != 0.0;
                }
                if (any) {
                    double Pr[M], ar[NA];
                    prim_at(qr, Pr);
#pragma unroll
                    for (int c = 0; c < NA; ++c) ar[c] = sd[line][F_A + c][qr];
                    pair_vjp_rhd<NU>(G, Pl, Pr, al, ar, w, gl, gr);
                }
            }
#pragma unroll
            for (int c = 0; c < M; ++c) {
                buf[line][nn - 1][c][lane] = gl[c];
                buf[line][3 + nn - 1][c][lane] = gr[c];
            }
        }
    }
    __syncthreads();
    if (o < ASEG) {
#pragma unroll
        for (int nn = 1; nn <= PO; ++nn)
#pragma unroll
            for (int c = 0; c < M; ++c)
                acc[c] += buf[line][nn - 1][c][o + 3] + buf[line][3 + nn - 1][c][o + 3 - nn];
    }

    if (ES) {
        __syncthreads();
        // ---- faces f = w ASEG - 3 + lane (stencil slots lane + 3 - PO .. lane + 2 + PO); the
        // cotangents of the 2 PO stencil states go to buf[j][.][lane]
        bool any = false;
        double z[M];
        if (active && lane < ASEG + 5) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                z[c] = 0.5 * idxi * (sl[line][c][lane + 2] - sl[line][c][lane + 3]);
                any |= z[c] != 0.0;
            }
        }
        if (any) {
            double al[NA], ar[NA];
#pragma unroll
            for (int c = 0; c < NA; ++c) { al[c] = sd[line][F_A + c][lane + 2]; ar[c] = sd[line][F_A + c][lane + 3]; }
            // the fence makes the later stages reread the stencil from LDS
            face_vjp_rhd<DIM, PO>(G, eps, [&](int j) { return node_at(lane + 3 - PO + j); },
                              [] { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); }, al, ar, z,
                              [&](int j, int c) -> double& { return buf[line][j][c][lane]; },
                              [&](int q, int c) -> double& { return lds.gr[line][q][c][lane]; },
                              [&](int j, int c, double v) { buf[line][j][c][lane] = v; });
        } else {
#pragma unroll
            for (int j = 0; j < 2 * PO; ++j)
#pragma unroll
                for (int c = 0; c < M; ++c) buf[line][j][c][lane] = 0.0;
        }
        __syncthreads();
        if (o < ASEG) {
#pragma unroll
            for (int j = 0; j < 2 * PO; ++j)
#pragma unroll
                for (int c = 0; c < M; ++c) acc[c] += buf[line][j][c][o + 2 + PO - j];
        }
    }

    long long lid_out, pbase_out, ibase_out;
    int s_out;
    locate(AHALO + o, lid_out, s_out, pbase_out, ibase_out);
    (void)ibase_out;
    if (o < ASEG && lid_out < nlines) {
        const long long idx = pbase_out + (long long)s_out * pstride;
#pragma unroll
        for (int c = 0; c < M; ++c) gout[c * P + idx] = acc[c];
    }
}

// Cotangents of the padded primitive states, one slab (M comps, padded layout)
// per direction; only positions along lines through interior transverse
// coordinates are written.
template <int DIM, bool ES, int PO>
__global__ void __launch_bounds__(128) k_residual_vjp(GridDev g, double G, double eps,
                                                      const double* __restrict__ prim,
                                                      const double* __restrict__ met,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ gdir, AdjPlan pl) {
    constexpr int M = DIM + 2;
    __shared__ AdjLDS<DIM> lds;
    const long long slab = (long long)M * g.pnodes;
    int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    if (b < pl.nblk[0]) {
        residual_vjp_segment<DIM, 0, ES, PO>(g, G, eps, prim, met, lam, gdir, b, pl.nseg[0], pl.nlines[0], pl.flat[0], pl.nsl[0], lds);
        return;
    }
    b -= pl.nblk[0];
    if (DIM == 2 || b < pl.nblk[1]) {
        residual_vjp_segment<DIM, 1, ES, PO>(g, G, eps, prim, met, lam, gdir + slab, b, pl.nseg[1], pl.nlines[1], pl.flat[1], pl.nsl[1], lds);
        return;
    }
    b -= pl.nblk[1];
    if (DIM == 3)
        residual_vjp_segment<DIM, 2, ES, PO>(g, G, eps, prim, met, lam, gdir + 2 * slab, b, pl.nseg[2], pl.nlines[2], pl.flat[2], pl.nsl[2], lds);
}

// Solve A^T y = b for a small dense A (n x n, row-major) by Gaussian elimination
// with partial pivoting on A^T.
template <int n>
__device__ __forceinline__ void solve_transposed(double A[n][n], const double* b, double* y) {
    double Mx[n][n + 1];
#pragma unroll
    for (int r = 0; r < n; ++r) {
#pragma unroll
        for (int c = 0; c < n; ++c) Mx[r][c] = A[c][r];
        Mx[r][n] = b[r];
    }
#pragma unroll
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(Mx[k][k]);
#pragma unroll
        for (int r = k + 1; r < n; ++r)
            if (fabs(Mx[r][k]) > best) { best = fabs(Mx[r][k]); piv = r; }
        if (piv != k) {
#pragma unroll
            for (int r = k + 1; r < n; ++r) {
                if (r == piv) {
#pragma unroll
                    for (int c = 0; c <= n; ++c) { const double t = Mx[k][c]; Mx[k][c] = Mx[r][c]; Mx[r][c] = t; }
                }
            }
        }
        const double ik = 1.0 / Mx[k][k];
#pragma unroll
        for (int r = k + 1; r < n; ++r) {
            const double f = Mx[r][k] * ik;
#pragma unroll
            for (int c = k; c <= n; ++c) Mx[r][c] -= f * Mx[k][c];
        }
    }
#pragma unroll
    for (int k = n - 1; k >= 0; --k) {
        double s = Mx[k][n];
#pragma unroll
        for (int c = k + 1; c < n; ++c) s -= Mx[k][c] * y[c];
        y[k] = s / Mx[k][k];
    }
}

// dUbar/dP of the RHD map at one node, P = (rho, u, p): D = rho W,
// m = (rho + c0 p) W u, E = (rho + c0 p) W^2 - p, c0 = Gamma/(Gamma-1), W^2 = 1 + |u|^2.
template <int DIM>
__device__ __forceinline__ void rhd_dU_dP(double G, double rho, const double* u, double p,
                                          double A[DIM + 2][DIM + 2]) {
    constexpr int NU = DIM, M = DIM + 2;
    double uu = 0.0;
#pragma unroll
    for (int c = 0; c < NU; ++c) uu += u[c] * u[c];
    const double W = sqrt(1.0 + uu), iW = 1.0 / W;
    const double c0 = G / (G - 1.0);
    const double rh = rho + c0 * p;
    A[0][0] = W;
#pragma unroll
    for (int l = 0; l < NU; ++l) A[0][1 + l] = rho * u[l] * iW;
    A[0][M - 1] = 0.0;
#pragma unroll
    for (int kk = 0; kk < NU; ++kk) {
        A[1 + kk][0] = W * u[kk];
#pragma unroll
        for (int l = 0; l < NU; ++l) A[1 + kk][1 + l] = rh * (u[l] * u[kk] * iW + (l == kk ? W : 0.0));
        A[1 + kk][M - 1] = c0 * W * u[kk];
    }
    A[M - 1][0] = W * W;
#pragma unroll
    for (int l = 0; l < NU; ++l) A[M - 1][1 + l] = 2.0 * rh * u[l];
    A[M - 1][M - 1] = c0 * W * W - 1.0;
}

// Pull a primitive cotangent back through con2prim (implicit-function rule) and
// U = Ucurv / J:
//   g_Ubar = (dUbar/dP)^{-T} g_P,  g_Ucurv = g_Ubar / J,  g_J = -(g_Ubar . Ucurv) / J^2.
// FOLD: g_P is the residual VJP's padded cotangent by direction (gsrc = gdir),
// ghost cotangents folded onto the interior nodes they copy; otherwise g_P is an
// interior field of m components (gsrc = the caller's cotangent).
template <int DIM, bool FOLD>
__global__ void __launch_bounds__(256) k_fold_con2prim_vjp(GridDev g, double G,
                                                           const double* __restrict__ prim,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ J,
                                                           const double* __restrict__ gsrc,
                                                           double* __restrict__ gU,
                                                           double* __restrict__ gJ) {
    constexpr int NU = DIM, M = DIM + 2;
    int i, j, k;
    if (!box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) return;
    const long long P = g.pnodes, N = g.nodes;
    const long long slab = (long long)M * P;
    const long long pi0 = pidx(g, i, j, k);
    const long long t = iidx(g, i, j, k);
    double gP[M];
#pragma unroll
    for (int c = 0; c < M; ++c) gP[c] = FOLD ? 0.0 : gsrc[c * N + t];
    const int ijk[3] = {i, j, k};
    const double* gdir = gsrc;
#pragma unroll
    for (int d = 0; d < (FOLD ? DIM : 0); ++d) {
        const double* gd = gdir + d * slab;
        const long long str = d == 0 ? 1 : (d == 1 ? (long long)g.P[0] : (long long)g.P[0] * g.P[1]);
        const int n = g.n[d], me = ijk[d];
#pragma unroll
        for (int c = 0; c < M; ++c) gP[c] += gd[c * P + pi0];
        // ghost positions along d that copy this node
#pragma unroll
        for (int q = 0; q < 2 * NG; ++q) {
            const int gpos = q < NG ? q - NG : n + (q - NG);
            if (map_sol(gpos, n, g.bc[d]) == me) {
                const long long gi = pi0 + (long long)(gpos - me) * str;
#pragma unroll
                for (int c = 0; c < M; ++c) gP[c] += gd[c * P + gi];
            }
        }
    }
    const double rho = prim[pi0], p = prim[(M - 1) * P + pi0];
    double u[NU];
#pragma unroll
    for (int c = 0; c < NU; ++c) u[c] = prim[(1 + c) * P + pi0];
    double A[M][M];
    rhd_dU_dP<DIM>(G, rho, u, p, A);
    double y[M];
    solve_transposed<M>(A, gP, y);
    const double Jv = J[t], iJ = 1.0 / Jv;
    double gj = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        gU[c * N + t] = y[c] * iJ;
        gj -= y[c] * U[c * N + t];
    }
    gJ[t] = gj * iJ * iJ;
}

// VJP of Ucurv = J U(P) at the interior nodes: g_P = J (dU/dP)^T g_Ucurv,
// g_J = U(P) . g_Ucurv (gJ may be null).  prim: interior, m comps (rho, u, p).
template <int DIM>
__global__ void __launch_bounds__(256) k_prim2con_vjp_rhd(GridDev g, double G,
                                                          const double* __restrict__ prim,
                                                          const double* __restrict__ J,
                                                          const double* __restrict__ gUc,
                                                          double* __restrict__ gP,
                                                          double* __restrict__ gJ) {
    constexpr int NU = DIM, M = DIM + 2;
    const long long t = gtid();
    if (t >= g.nodes) return;
    const long long N = g.nodes;
    const double rho = prim[t], p = prim[(M - 1) * N + t];
    double u[NU], uu = 0.0;
#pragma unroll
    for (int c = 0; c < NU; ++c) { u[c] = prim[(1 + c) * N + t]; uu += u[c] * u[c]; }
    double A[M][M];
    rhd_dU_dP<DIM>(G, rho, u, p, A);
    double gu[M];
#pragma unroll
    for (int r = 0; r < M; ++r) gu[r] = gUc[r * N + t];
    const double Jv = J[t];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < M; ++r) acc += A[r][c] * gu[r];
        gP[c * N + t] = Jv * acc;
    }
    if (gJ != nullptr) {
        // U(P): D = rho W, m = rho h W u, E = rho h W^2 - p
        const double W = sqrt(1.0 + uu);
        const double rh = rho + G / (G - 1.0) * p;
        double acc = rho * W * gu[0] + (rh * W * W - p) * gu[M - 1];
#pragma unroll
        for (int c = 0; c < NU; ++c) acc += rh * W * u[c] * gu[1 + c];
        gJ[t] = acc;
    }
}

// RK3 reverse sweep, elementwise over U (nU values) and J (nJ values).
// pre:  lamL = cL dt lam (U part), acc (=|+=) cA lam
__global__ void k_adj_pre(long long nU, long long nJ, double cL, double cA, int first,
                          const double* __restrict__ dt_dev, const double* __restrict__ lamU,
                          const double* __restrict__ lamJ, double* __restrict__ lamL,
                          double* __restrict__ accU, double* __restrict__ accJ) {
    const long long t = gtid();
    if (t >= nU + nJ) return;
    if (t < nU) {
        lamL[t] = cL * dt_dev[0] * lamU[t];
        accU[t] = (first ? 0.0 : accU[t]) + cA * lamU[t];
    } else {
        const long long q = t - nU;
        accJ[q] = (first ? 0.0 : accJ[q]) + cA * lamJ[q];
    }
}

// post: lam = cK lam + g
__global__ void k_adj_post(long long nU, long long nJ, double cK, double* __restrict__ lamU,
                           double* __restrict__ lamJ, const double* __restrict__ gU,
                           const double* __restrict__ gJ) {
    const long long t = gtid();
    if (t >= nU + nJ) return;
    if (t < nU) lamU[t] = cK * lamU[t] + gU[t];
    else { const long long q = t - nU; lamJ[q] = cK * lamJ[q] + gJ[q]; }
}

// final: out = acc + lam + g
__global__ void k_adj_final(long long nU, long long nJ, const double* __restrict__ accU,
                            const double* __restrict__ accJ, const double* __restrict__ lamU,
                            const double* __restrict__ lamJ, const double* __restrict__ gU,
                            const double* __restrict__ gJ, double* __restrict__ outU,
                            double* __restrict__ outJ) {
    const long long t = gtid();
    if (t >= nU + nJ) return;
    if (t < nU) outU[t] = accU[t] + lamU[t] + gU[t];
    else { const long long q = t - nU; outJ[q] = accJ[q] + lamJ[q] + gJ[q]; }
}

template <int DIM>
static void residual_vjp_all(const es_ctx* c, const double* prim, const double* met,
                             const double* lam, double* gdir, hipStream_t s) {
    const GridDev& g = c->g;
    AdjPlan pl{};
    long long nb = 0;
    for (int d = 0; d < DIM; ++d) {
        long long nl = 1;
        for (int a = 0; a < DIM; ++a)
            if (a != d) nl *= g.n[a];
        // every padded position of every line is an output; segments per sequence of
        // the longest sequence (flat where it saves an eighth of the wavefronts), one
        // block per segment offset
        const long long ml = (nl + ALINES - 1) / ALINES;
        const int plen = g.n[d] + 2 * NG;
        pl.flat[d] = seq_flat(plen, plen, ASEG, 0.875) ? 1 : 0;
        pl.nsl[d] = (plen + ASEG - 1) / ASEG;
        pl.nseg[d] = pl.flat[d] ? (int)((ml * plen + ASEG - 1) / ASEG) : (int)(ml * pl.nsl[d]);
        pl.nlines[d] = nl;
        pl.nblk[d] = pl.nseg[d];
        nb += pl.nblk[d];
    }
    const double G = c->scheme.gamma, eps = c->scheme.weno_eps;
    const unsigned thr = 64 * ALINES;
    const bool es = c->scheme.dissipation != 0;
    if (c->scheme.order_p == 2) {
        if (es)
            k_residual_vjp<DIM, true, 2><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl);
        else
            k_residual_vjp<DIM, false, 2><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl);
    } else if (es) {
        k_residual_vjp<DIM, true, 3><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl);
    } else {
        k_residual_vjp<DIM, false, 3><<<(unsigned)nb, thr, 0, s>>>(g, G, eps, prim, met, lam, gdir, pl);
    }
}

}  // namespace

hipError_t launch_state_residual_vjp(const es_ctx* c, const double* U, const double* J,
                                     const double* met, const double* lam, double* gU, double* gJ,
                                     hipStream_t s) {
    hipError_t e = launch_con2prim(c, U, J, c->prim, 0, s);
    if (e != hipSuccess) return e;
    if (c->scheme.phys == ES_RMHD) return launch_residual_fold_vjp_rmhd(c, U, J, met, lam, gU, gJ, s);
    if (c->g.dim == 2) residual_vjp_all<2>(c, c->prim, met, lam, c->gdir, s);
    else residual_vjp_all<3>(c, c->prim, met, lam, c->gdir, s);
    const GridDev& g = c->g;
    const dim3 gr = box_grid(g.n[0], g.n[1], g.n[2]);
    if (g.dim == 2) k_fold_con2prim_vjp<2, true><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, c->gdir, gU, gJ);
    else k_fold_con2prim_vjp<3, true><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, c->gdir, gU, gJ);
    return hipGetLastError();
}

hipError_t launch_con2prim_vjp(const es_ctx* c, const double* U, const double* J, const double* gprim,
                               double* gU, double* gJ, hipStream_t s) {
    hipError_t e = launch_con2prim(c, U, J, c->prim, 0, s);
    if (e != hipSuccess) return e;
    if (c->scheme.phys == ES_RMHD) return launch_con2prim_vjp_rmhd(c, U, J, gprim, gU, gJ, s);
    const GridDev& g = c->g;
    const dim3 gr = box_grid(g.n[0], g.n[1], g.n[2]);
    if (g.dim == 2) k_fold_con2prim_vjp<2, false><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, gprim, gU, gJ);
    else k_fold_con2prim_vjp<3, false><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, c->prim, U, J, gprim, gU, gJ);
    return hipGetLastError();
}

hipError_t launch_prim2con_vjp(const es_ctx* c, const double* prim, const double* J, const double* gUc,
                               double* gprim, double* gJ, hipStream_t s) {
    if (c->scheme.phys == ES_RMHD) return launch_prim2con_vjp_rmhd(c, prim, J, gUc, gprim, gJ, s);
    const GridDev& g = c->g;
    if (g.dim == 2) k_prim2con_vjp_rhd<2><<<grid_for(g.nodes), TPB, 0, s>>>(g, c->scheme.gamma, prim, J, gUc, gprim, gJ);
    else k_prim2con_vjp_rhd<3><<<grid_for(g.nodes), TPB, 0, s>>>(g, c->scheme.gamma, prim, J, gUc, gprim, gJ);
    return hipGetLastError();
}

hipError_t launch_rk3_vjp(const es_ctx* c, const double* ckpt, const double* lamU_in,
                          const double* lamJ_in, double* gU_out, double* gJ_out, hipStream_t s) {
    const GridDev& g = c->g;
    const long long N = g.nodes, nU = N * c->m, nJ = N;
    const Checkpoint k = checkpoint_layout(c, ckpt);
    static const double coef[3] = {0.0, 1.0, 0.5};
    // stage 2: U3 = 1/3 U0 + 2/3 (U2 + dt L2)
    // stage 1: U2 = 3/4 U0 + 1/4 (U1 + dt L1)
    // stage 0: U1 = U0 + dt L0
    static const double cL[3] = {1.0, 0.25, 2.0 / 3.0};
    static const double cA[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double cK[3] = {1.0, 0.25, 2.0 / 3.0};
    hipError_t e = launch_copy(c->adj_lamU, lamU_in, nU, s);
    if (e == hipSuccess) e = launch_copy(c->adj_lamJ, lamJ_in, nJ, s);
    if (e != hipSuccess) return e;
    for (int st = 2; st >= 0; --st) {
        k_adj_pre<<<grid_for(nU + nJ), TPB, 0, s>>>(nU, nJ, cL[st], cA[st], st == 2, k.dt, c->adj_lamU,
                                                     c->adj_lamJ, c->adj_lamL, c->adj_accU, c->adj_accJ);
        e = launch_metrics(c, k.x, k.xdot, k.dt, coef[st], c->met, nullptr, s);
        if (e == hipSuccess)
            e = launch_state_residual_vjp(c, k.U[st], k.J[st], c->met, c->adj_lamL, c->adj_gU, c->adj_gJ, s);
        if (e != hipSuccess) return e;
        if (st > 0)
            k_adj_post<<<grid_for(nU + nJ), TPB, 0, s>>>(nU, nJ, cK[st], c->adj_lamU, c->adj_lamJ, c->adj_gU,
                                                          c->adj_gJ);
        else
            k_adj_final<<<grid_for(nU + nJ), TPB, 0, s>>>(nU, nJ, c->adj_accU, c->adj_accJ, c->adj_lamU,
                                                           c->adj_lamJ, c->adj_gU, c->adj_gJ, gU_out, gJ_out);
    }
    return hipGetLastError();
}

}  // namespace es
