// RMHD kernels of libes.so (gfx950): primitive <-> conservative, the residual
// (EC pair fluxes, Godunov-Powell source, VCL, ES dissipation with the numeric
// eigen-structure), the CFL spectral radius and the FP64 diagnostics.  Same
// launch shapes and layouts as the RHD kernels; 8 conservative components,
// padded primitive fields (rho, u_1..3, p, B_1..3, ln rho, ln beta).
#include <float.h>
#include <math.h>

#include "es_internal.h"
#include "es_launch.h"
#include "es_rmhd.h"

namespace es {

namespace {

constexpr int MR = 8;              // RMHD conservative components

__global__ void k_prim2con_rmhd(GridDev g, double G, const double* __restrict__ prim,
                                const double* __restrict__ J, double* __restrict__ U) {
    const long long t = gtid();
    if (t >= g.nodes) return;
    const long long N = g.nodes;
    double P[MR], Uc[MR];
#pragma unroll
    for (int c = 0; c < MR; ++c) P[c] = prim[c * N + t];
    const StateRMHD<double> s = rmhd_state<double>(G, P);
    rmhd_cons<double>(s, Uc);
    const double Jv = J[t];
#pragma unroll
    for (int c = 0; c < MR; ++c) U[c * N + t] = Jv * Uc[c];
}

// con2prim on the padded box; with use_guess the previous Z = rho h W^2 of the
// node seeds the iteration.
__global__ void k_con2prim_rmhd(GridDev g, double G, StateSrc ss, double* prim, int use_guess,
                                unsigned long long* __restrict__ fail) {
    int i, j, k;
    if (!box_ijk(-g.ng, -g.ng, -g.g2, g.P[0], g.P[1], i, j, k)) return;
    const long long t = pidx(g, i, j, k);
    const int si = map_sol(i, g.n[0], g.bc[0]);
    const int sj = map_sol(j, g.n[1], g.bc[1]);
    const int sk = g.dim == 3 ? map_sol(k, g.n[2], g.bc[2]) : 0;
    const long long src = iidx(g, si, sj, sk);
    const long long N = g.nodes, P = g.pnodes;
    double Us[MR + 1];
#pragma unroll
    for (int c = 0; c <= MR; ++c) Us[c] = state_value(ss, g.dim, MR, N, c, src);
    if (ss.stage >= 0 && si == i && sj == j && sk == k) {
#pragma unroll
        for (int c = 0; c < MR; ++c) ss.Uout[c * N + src] = Us[c];
        ss.Jout[src] = Us[MR];
    }
    const double iJ = 1.0 / Us[MR];
    double Uc[MR], Pv[MR];
#pragma unroll
    for (int c = 0; c < MR; ++c) Uc[c] = Us[c] * iJ;
    double guess = -1.0;
    if (use_guess) {
        const double rho = prim[t], p = prim[4 * P + t];
        double uu = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) { const double u = prim[(1 + c) * P + t]; uu += u * u; }
        guess = (rho + G / (G - 1.0) * p) * (1.0 + uu);
    }
    const double Jv = Us[MR];
    const int st = Jv > 0.0 && Jv < INFINITY ? c2p_rmhd(G, Uc, guess, Pv) : FAIL_MESH;
    if (st != 0) {
#pragma unroll
        for (int c = 0; c < MR; ++c) Pv[c] = __builtin_nan("");
        if (si == i && sj == j && sk == k) record_failure(fail, st, src);
    }
#pragma unroll
    for (int c = 0; c < MR; ++c) prim[c * P + t] = Pv[c];
    prim[MR * P + t] = log(Pv[0]);
    prim[(MR + 1) * P + t] = log(Pv[0] / Pv[4]);
}

// ---------------------------------------------------------------------------
// residual: one wavefront per line segment of seg_nodes(p) nodes (as the RHD
// residual)
// ---------------------------------------------------------------------------
constexpr int RLINES = 2;

template <int DIM, int PO>
struct ResidualLDSM {
    static constexpr int NA = DIM + 1, NF = MR + 2 + NA;
    double sd[RLINES][NF][seg_loads(PO) + 1];
    double sp[RLINES][PO > 2 ? PO : 2][MR + 2][64];    // pair fluxes F (8), J and B~ values
};

struct SweepPlanM {
    int nseg[3];
    int nblk[3];
    long long nlines[3];
};

template <int DIM, int DIR, bool ES, bool MIXED, int PO>
__device__ __forceinline__ void residual_segment_rmhd(const GridDev& g, double G, double eps,
                                                      const double* __restrict__ prim,
                                                      const double* __restrict__ met,
                                                      double* __restrict__ out, int blk, int nseg,
                                                      long long nlines, ResidualLDSM<DIM, PO>& lds) {
    constexpr int NA = DIM + 1;
    constexpr int NGP = ghost_layers(PO), SEGP = seg_nodes(PO), NLOADP = seg_loads(PO);
    constexpr int F_LR = MR, F_LB = MR + 1, F_A = MR + 2;
    auto& sd = lds.sd;
    auto& sp = lds.sp;
    const int lane = threadIdx.x & 63;
    const int line = threadIdx.x >> 6;
    const int seg = blk % nseg;
    const long long lid = (long long)(blk / nseg) * RLINES + line;
    const bool active = lid < nlines;
    const int nAlong = g.n[DIR];
    const int s0 = seg * SEGP;
    const int s_end = min(s0 + SEGP, nAlong);
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

    // Lane q holds position q and, for q < NLOADP - 64, position 64 + q as well: the
    // loads of both are issued before either is used, from addresses that are always
    // valid and outside any branch (a position off the line reads node 0 and then
    // takes the far-field values instead), so the wavefront waits on memory once.
    static_assert(NLOADP > 64 && NLOADP <= 128, "two positions per lane");
    {
        constexpr int NV = MR + 2 + NA;
        const bool sec = lane < NLOADP - 64;
        const int sa = s0 - NGP + lane, sb = s0 - NGP + 64 + (sec ? lane : 0);
        const bool oka = active && sa < s_end + NGP, okb = sec && active && sb < s_end + NGP;
        const long long ia = oka ? pbase + (long long)sa * pstride : 0;
        const long long ib = okb ? pbase + (long long)sb * pstride : 0;
        double va[NV], vb[NV];
#pragma unroll
        for (int c = 0; c < MR + 2; ++c) {
            va[c] = prim[c * P + ia];
            vb[c] = prim[c * P + ib];
        }
#pragma unroll
        for (int c = 0; c < NA; ++c) {
            va[F_A + c] = met[(DIR * NA + c) * P + ia];
            vb[F_A + c] = met[(DIR * NA + c) * P + ib];
        }
        // every load issued before any of them is used
        __builtin_amdgcn_sched_barrier(0);
        // far field: rho = p = 1, the metric (0, 1, 0, ...), the rest 0
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const double far = (c == 0 || c == 4 || c == F_A + 1) ? 1.0 : 0.0;
            va[c] = oka ? va[c] : far;
            vb[c] = okb ? vb[c] : far;
        }
        // the lanes without a second position store their own again (the same
        // values): no branch, so the second loads are not sunk after the first wait
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            sd[line][c][lane] = va[c];
            sd[line][c][sec ? 64 + lane : lane] = sec ? vb[c] : va[c];
        }
    }
    __syncthreads();

    auto prim_at = [&](int q, double* Pq) {
#pragma unroll
        for (int c = 0; c < MR; ++c) Pq[c] = sd[line][c][q];
    };
    auto node_at = [&](int q) {
        double Pq[MR];
        prim_at(q, Pq);
        return node_rmhd(G, Pq, sd[line][F_LR][q], sd[line][F_LB][q]);
    };

    const int s_own = s0 - NGP + lane;
    if (active && s_own < s_end) {
        const NodeRMHD l = node_at(lane);
        double al[NA];
#pragma unroll
        for (int c = 0; c < NA; ++c) al[c] = sd[line][F_A + c][lane];
#pragma unroll 1
        for (int n = 1; n <= PO; ++n) {
            const NodeRMHD r = node_at(lane + n);
            double ar[NA];
#pragma unroll
            for (int c = 0; c < NA; ++c) ar[c] = sd[line][F_A + c][lane + n];
            double F[MR], Jt, Bt;
            pair_flux_rmhd<DIM, typename std::conditional<MIXED, float, double>::type>(G, l, r, al, ar, F, Jt,
                                                                                         Bt);
#pragma unroll
            for (int c = 0; c < MR; ++c) sp[line][n - 1][c][lane] = F[c];
            sp[line][n - 1][MR][lane] = Jt;
            sp[line][n - 1][MR + 1][lane] = Bt;
        }
    }
    __syncthreads();

    const bool owner = active && lane >= NGP && s_own < s_end;
    const double idxi = 1.0 / g.dxi[DIR];
    double R[MR + 1];
#pragma unroll
    for (int c = 0; c <= MR; ++c) R[c] = 0.0;
    if (owner) {
        double diff[MR + 2];
#pragma unroll
        for (int c = 0; c < MR + 2; ++c) {
            double s = 0.0;
#pragma unroll
            for (int n = 1; n <= PO; ++n)
                s += alpha_pn(PO, n) * (sp[line][n - 1][c][lane] - sp[line][n - 1][c][lane - n]);
            diff[c] = s * idxi;
        }
        // flux differences and the Godunov-Powell source -Phi'(V_i) (B~ differences)
        double Pq[MR];
        prim_at(lane, Pq);
        const StateRMHD<double> st = rmhd_state<double>(G, Pq);
        double Pp[MR];
        rmhd_phi_prime<double>(st, Pp);
#pragma unroll
        for (int c = 0; c < MR; ++c) R[c] = -diff[c] - Pp[c] * diff[MR + 1];
        R[MR] = -diff[MR];
    }

    if (ES) {
        __syncthreads();
        // the flux differences wait in the (now free) pair slot 1 while the face
        // dissipation runs (register pressure)
        if (owner) {
#pragma unroll
            for (int c = 0; c <= MR; ++c) sp[line][1][c][lane] = R[c];
        }
        if (active && lane >= PO - 1 && s_own < s_end) {
            double Pn[2 * PO][MR];
#pragma unroll
            for (int q = 0; q < 2 * PO; ++q) prim_at(lane - (PO - 1) + q, Pn[q]);
            double al[NA], ar[NA];
#pragma unroll
            for (int c = 0; c < NA; ++c) { al[c] = sd[line][F_A + c][lane]; ar[c] = sd[line][F_A + c][lane + 1]; }
            double d[MR];
            face_diss_rmhd<DIM, MIXED, PO>(G, eps, Pn, al, ar, d);
#pragma unroll
            for (int c = 0; c < MR; ++c) sp[line][0][c][lane] = d[c];
        }
        __syncthreads();
        if (owner) {
#pragma unroll
            for (int c = 0; c <= MR; ++c) R[c] = sp[line][1][c][lane];
#pragma unroll
            for (int c = 0; c < MR; ++c) R[c] += 0.5 * (sp[line][0][c][lane] - sp[line][0][c][lane - 1]) * idxi;
        }
    }

    if (owner) {
        const long long o = ibase + (long long)s_own * istride;
#pragma unroll
        for (int c = 0; c <= MR; ++c) out[c * N + o] = R[c];
    }
}

template <int DIM, bool ES, bool MIXED, int PO>
__global__ void __launch_bounds__(128) k_residual_rmhd(GridDev g, double G, double eps,
                                                       const double* __restrict__ prim,
                                                       const double* __restrict__ met,
                                                       double* __restrict__ Ld, SweepPlanM sw) {
    __shared__ ResidualLDSM<DIM, PO> lds;
    const long long slab = (long long)(MR + 1) * g.nodes;
    int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    if (b < sw.nblk[0]) {
        residual_segment_rmhd<DIM, 0, ES, MIXED, PO>(g, G, eps, prim, met, Ld, b, sw.nseg[0], sw.nlines[0], lds);
        return;
    }
    b -= sw.nblk[0];
    if (DIM == 2 || b < sw.nblk[1]) {
        residual_segment_rmhd<DIM, 1, ES, MIXED, PO>(g, G, eps, prim, met, Ld + slab, b, sw.nseg[1], sw.nlines[1], lds);
        return;
    }
    b -= sw.nblk[1];
    if (DIM == 3)
        residual_segment_rmhd<DIM, 2, ES, MIXED, PO>(g, G, eps, prim, met, Ld + 2 * slab, b, sw.nseg[2], sw.nlines[2], lds);
}

// CFL partial maxima: rho_k = L_k max_m |lambda_m| / J per direction (eq. cfl), the
// eigenvalues of the Godunov-Powell modified x_1 Jacobian at the state rotated
// to the metric normal of direction k.
template <int DIM>
__global__ void __launch_bounds__(256) k_cfl_partial_rmhd(GridDev g, double G, const double* __restrict__ prim,
                                                          const double* __restrict__ met,
                                                          const double* __restrict__ J,
                                                          double* __restrict__ partial) {
    constexpr int NA = DIM + 1;
    __shared__ double sh[8];
    double mx[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) mx[k] = 0.0;
    const long long P = g.pnodes;
    int i, j, k;
    if (box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) {
        const long long pi = pidx(g, i, j, k);
        double Pv[MR];
#pragma unroll
        for (int c = 0; c < MR; ++c) Pv[c] = prim[c * P + pi];
        const double iJ = 1.0 / J[iidx(g, i, j, k)];
#pragma unroll 1
        for (int kd = 0; kd < DIM; ++kd) {
            double ax[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < DIM; ++c) ax[c] = met[(kd * NA + 1 + c) * P + pi];
            const double L = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
            double n[3] = {ax[0] / L, ax[1] / L, ax[2] / L};
            double T[3][3];
            rotation<3>(n, T);
            double Pr[MR];
            rotate8<false>(T, Pv, Pr);
            const double r = L * rmhd_max_speed(G, Pr) * iJ;
            if (kd == 0) mx[0] = r;
            else if (kd == 1) mx[DIM > 1 ? 1 : 0] = r;
            else mx[DIM - 1] = r;
        }
    }
    const int nb = (int)(gridDim.x * gridDim.y * gridDim.z);
#pragma unroll
    for (int kd = 0; kd < DIM; ++kd) {
        const double r = block_reduce<0>(mx[kd], sh);
        if (flat_tid() == 0) partial[kd * nb + flat_block()] = r;
    }
}

// FP64 diagnostics: sum (V.dU - phi dJ), sum J eta, sum J, sum U (8 comps);
// phi = rho W + beta |b|^2 W / 2 (eq. EntropyPotential), eta = -rho W s/(G-1).
template <int DIM>
__global__ void __launch_bounds__(256) k_diag_partial_rmhd(GridDev g, double G, const double* __restrict__ prim,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ J,
                                                           const double* __restrict__ dU,
                                                           const double* __restrict__ dJ,
                                                           double* __restrict__ partial) {
    constexpr int NQ = 3 + MR;
    __shared__ double sh[8];
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const long long P = g.pnodes, N = g.nodes;
    int i, j, k;
    if (box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) {
        const long long t = iidx(g, i, j, k);
        const long long pi = pidx(g, i, j, k);
        double Pv[MR], V[MR];
#pragma unroll
        for (int c = 0; c < MR; ++c) Pv[c] = prim[c * P + pi];
        const StateRMHD<double> s = rmhd_state<double>(G, Pv);
        rmhd_entropy_vars<double>(G, s, V);
        const double phi = s.rho * s.W + 0.5 * s.beta * s.bsq * s.W;
        double ep = 0.0;
#pragma unroll
        for (int c = 0; c < MR; ++c) ep += V[c] * dU[c * N + t];
        ep -= phi * dJ[t];
        const double sth = log(s.p) - G * log(s.rho);
        const double eta = -s.rho * s.W * sth / (G - 1.0);
        acc[0] = ep;
        acc[1] = J[t] * eta;
        acc[2] = J[t];
#pragma unroll
        for (int c = 0; c < MR; ++c) acc[3 + c] = U[c * N + t];
    }
    const int nb = (int)(gridDim.x * gridDim.y * gridDim.z);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double r = block_reduce<2>(acc[q], sh);
        if (flat_tid() == 0) partial[q * nb + flat_block()] = r;
    }
}

template <int DIM>
static void residual_all_rmhd(const es_ctx* c, const double* prim, const double* met, double* Ld,
                              hipStream_t s) {
    const GridDev& g = c->g;
    SweepPlanM sw{};
    long long nb = 0;
    const int segn = seg_nodes(g.p);
    for (int d = 0; d < DIM; ++d) {
        sw.nseg[d] = (g.n[d] + segn - 1) / segn;
        long long nl = 1;
        for (int a = 0; a < DIM; ++a)
            if (a != d) nl *= g.n[a];
        sw.nlines[d] = nl;
        sw.nblk[d] = (int)(((nl + RLINES - 1) / RLINES) * sw.nseg[d]);
        nb += sw.nblk[d];
    }
    const double G = c->scheme.gamma, eps = c->scheme.weno_eps;
    const dim3 grid((unsigned)nb), block(64 * RLINES);
    const bool es = c->scheme.dissipation != 0, mixed = c->scheme.mixed != 0;
    if (c->scheme.order_p == 2) {
        if (es && mixed) k_residual_rmhd<DIM, true, true, 2><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        else if (es) k_residual_rmhd<DIM, true, false, 2><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        else if (mixed) k_residual_rmhd<DIM, false, true, 2><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        else k_residual_rmhd<DIM, false, false, 2><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        return;
    }
    if (c->scheme.order_p == 4) {
        if (es && mixed) k_residual_rmhd<DIM, true, true, 4><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        else if (es) k_residual_rmhd<DIM, true, false, 4><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        else if (mixed) k_residual_rmhd<DIM, false, true, 4><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        else k_residual_rmhd<DIM, false, false, 4><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
        return;
    }
    if (es && mixed) k_residual_rmhd<DIM, true, true, 3><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
    else if (es) k_residual_rmhd<DIM, true, false, 3><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
    else if (mixed) k_residual_rmhd<DIM, false, true, 3><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
    else k_residual_rmhd<DIM, false, false, 3><<<grid, block, 0, s>>>(g, G, eps, prim, met, Ld, sw);
}

}  // namespace

hipError_t launch_prim2con_rmhd(const es_ctx* c, const double* prim, const double* J, double* U,
                                hipStream_t s) {
    k_prim2con_rmhd<<<grid_for(c->g.nodes), TPB, 0, s>>>(c->g, c->scheme.gamma, prim, J, U);
    return hipGetLastError();
}

hipError_t launch_con2prim_rmhd(const es_ctx* c, const void* state_src, double* prim, int use_guess,
                                hipStream_t s) {
    const GridDev& g = c->g;
    const StateSrc ss = *static_cast<const StateSrc*>(state_src);
    k_con2prim_rmhd<<<box_grid(g.P[0], g.P[1], g.P[2]), box_block(), 0, s>>>(g, c->scheme.gamma, ss, prim,
                                                                              use_guess, c->fail);
    return hipGetLastError();
}

hipError_t launch_residual_dirs_rmhd(const es_ctx* c, const double* prim, const double* met, double* Ld,
                                     hipStream_t s) {
    if (c->g.dim == 2) residual_all_rmhd<2>(c, prim, met, Ld, s);
    else residual_all_rmhd<3>(c, prim, met, Ld, s);
    return hipGetLastError();
}

hipError_t launch_cfl_partial_rmhd(const es_ctx* c, const double* prim, const double* met,
                                   const double* J, hipStream_t s) {
    const GridDev& g = c->g;
    const dim3 gr = box_grid(g.n[0], g.n[1], g.n[2]);
    if (g.dim == 2) k_cfl_partial_rmhd<2><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, prim, met, J, c->red);
    else k_cfl_partial_rmhd<3><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, prim, met, J, c->red);
    return hipGetLastError();
}

hipError_t launch_diag_partial_rmhd(const es_ctx* c, const double* prim, const double* U, const double* J,
                                    const double* dU, const double* dJ, hipStream_t s) {
    const GridDev& g = c->g;
    const dim3 gr = box_grid(g.n[0], g.n[1], g.n[2]);
    if (g.dim == 2) k_diag_partial_rmhd<2><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, prim, U, J, dU, dJ, c->red);
    else k_diag_partial_rmhd<3><<<gr, box_block(), 0, s>>>(g, c->scheme.gamma, prim, U, J, dU, dJ, c->red);
    return hipGetLastError();
}

}  // namespace es
