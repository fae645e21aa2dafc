// HIP kernels of libes.so (gfx950) and their launchers.
//
// Node kernels use 64 x 4 thread blocks over an index box (no integer
// division in the index map).  The residual maps one 64-lane wavefront to a
// 61-node segment of a grid line plus its 3-node halo, stages the line in LDS
// and exchanges two-point fluxes and face dissipation between lanes through
// LDS.  All scalars that feed back into the step (dt, monitor maximum,
// Delta_tau) come from two-pass block reductions ending in a one-block kernel:
// max/min are exact in any order, sums are only used for diagnostics.
#include <float.h>
#include <math.h>

#include "es_internal.h"
#include "es_launch.h"
#include "es_rhd.h"

namespace es {

namespace {

// index in the mesh-extension box (6 layers beyond the interior on active axes)
__device__ __forceinline__ long long eidx(const GridDev& g, int i, int j, int k) {
    return ((long long)(k + g.g6) * g.E[1] + (j + 2 * g.ng)) * g.E[0] + (i + 2 * g.ng);
}

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void k_zero(double* __restrict__ p, long long n) {
    const long long t = gtid();
    if (t < n) p[t] = 0.0;
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, long long n) {
    const long long t = gtid();
    if (t < n) dst[t] = src[t];
}

// ---------------------------------------------------------------------------
// primitive -> conservative (eq. RMHDdiv2 with B = 0), times J
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void k_prim2con_rhd(GridDev g, double G, const double* __restrict__ prim,
                               const double* __restrict__ J, double* __restrict__ U) {
    constexpr int M = DIM + 2;
    const long long t = gtid();
    if (t >= g.nodes) return;
    const long long N = g.nodes;
    const double rho = prim[t];
    const double p = prim[(M - 1) * N + t];
    double u[DIM], uu = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { u[k] = prim[(1 + k) * N + t]; uu += u[k] * u[k]; }
    const double W = sqrt(1.0 + uu);
    const double h = 1.0 + G / (G - 1.0) * p / rho;
    const double Jv = J[t];
    U[t] = Jv * (rho * W);
#pragma unroll
    for (int k = 0; k < DIM; ++k) U[(1 + k) * N + t] = Jv * (rho * h * W * u[k]);
    U[(M - 1) * N + t] = Jv * (rho * h * W * W - p);
}

// ---------------------------------------------------------------------------
// conservative -> primitive on the padded box (ghosts by the solution rule).
// With use_guess the pressure already stored at the node (previous stage) seeds
// the Newton iteration when it lies inside the bracket.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void k_con2prim_rhd(GridDev g, double G, StateSrc ss, double* prim, int use_guess,
                               unsigned long long* __restrict__ fail) {
    constexpr int M = DIM + 2;
    int i, j, k;
    if (DIM == 3) {
        if (!plane_cell_xcd(g.P[0], g.P[1], i, j, k)) return;
        i -= g.ng; j -= g.ng; k -= g.g2;
    } else if (!box_ijk(-g.ng, -g.ng, -g.g2, g.P[0], g.P[1], i, j, k)) {
        return;
    }
    const long long t = pidx(g, i, j, k);
    const int si = map_sol(i, g.n[0], g.bc[0]);
    const int sj = map_sol(j, g.n[1], g.bc[1]);
    const int sk = DIM == 3 ? map_sol(k, g.n[2], g.bc[2]) : 0;
    const long long src = iidx(g, si, sj, sk);
    const long long N = g.nodes;
    const long long P = g.pnodes;
    double Uc[M + 1];
#pragma unroll
    for (int c = 0; c <= M; ++c) Uc[c] = state_value(ss, DIM, M, N, c, src);
    if (ss.stage >= 0 && si == i && sj == j && sk == k) {
#pragma unroll
        for (int c = 0; c < M; ++c) ss.Uout[c * N + src] = Uc[c];
        ss.Jout[src] = Uc[M];
    }
    const double Jv = Uc[M];
    const double D = Uc[0] / Jv;
    double m[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) m[c] = Uc[1 + c] / Jv;
    const double E = Uc[M - 1] / Jv;
    double rho, p, u[DIM];
    const double guess = use_guess ? prim[(M - 1) * P + t] : -1.0;
    // a non-positive (or non-finite) Jacobian is a tangled mesh: recorded as such
    const int st = Jv > 0.0 && Jv < INFINITY ? c2p_rhd<DIM>(G, D, m, E, guess, rho, u, p) : FAIL_MESH;
    if (st != 0) {
        rho = p = __builtin_nan("");
#pragma unroll
        for (int c = 0; c < DIM; ++c) u[c] = __builtin_nan("");
        if (si == i && sj == j && sk == k) record_failure(fail, st, src);
    }
    prim[t] = rho;
#pragma unroll
    for (int c = 0; c < DIM; ++c) prim[(1 + c) * P + t] = u[c];
    prim[(M - 1) * P + t] = p;
    prim[M * P + t] = log(rho);
    prim[(M + 1) * P + t] = log(rho / p);
}

// ---------------------------------------------------------------------------
// metrics (Section 3.3; 2D explicit form of Appendix B with 1/Delta xi)
// ---------------------------------------------------------------------------
// Stage mesh x + cdt xdot and mesh velocity on the extension box (2 ng layers):
// periodic copies with the coordinate shift, odd reflection on outflow axes.
// Flattened cells per plane of the extension box.
template <int DIM>
__global__ void k_mesh_extend(GridDev g, const double* __restrict__ x, const double* __restrict__ xd,
                              const double* __restrict__ dt_dev, double coef, double* __restrict__ xe,
                              double* __restrict__ ve) {
    int i, j, k;
    if (!plane_cell_xcd(g.E[0], g.E[1], i, j, k)) return;
    i -= 2 * g.ng; j -= 2 * g.ng; k -= g.g6;
    const long long t = eidx(g, i, j, k);
    const double cdt = dt_dev != nullptr ? coef * dt_dev[0] : 0.0;
    const double* xs = dt_dev != nullptr ? xd : nullptr;
    if (i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && (DIM == 2 || (k >= 0 && k < g.n[2]))) {
        // interior node: every load issued before the first use (mesh_value's value
        // for an interior node, the velocity loaded once for both outputs)
        const long long nd = iidx(g, i, j, DIM == 2 ? 0 : k);
        double xv[DIM], dv[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            xv[c] = x[c * g.nodes + nd];
            dv[c] = xd != nullptr ? xd[c * g.nodes + nd] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double v = xv[c];
            if (xs != nullptr) v += cdt * dv[c];
            xe[c * g.enodes + t] = v;
            if (ve != nullptr) ve[c * g.enodes + t] = dv[c];
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        xe[c * g.enodes + t] = mesh_value(g, x, xs, cdt, c, i, j, k, true);
        if (ve != nullptr) ve[c * g.enodes + t] = xd != nullptr ? mesh_value(g, xd, nullptr, 0.0, c, i, j, k, false) : 0.0;
    }
}

// 2D metrics with the stage-mesh extension fused in: a block stages the
// extended stage mesh x + c dt xdot of its 64 x 4 tile of padded nodes plus a
// 3-node halo in LDS (mesh_value, as k_mesh_extend) and forms the central
// differences of eq. SCLCoeff (2D form of Appendix B with 1/Delta xi) from
// there; the mesh velocity is read at the node.
constexpr int MTX = 64, MTY = 4, MBY = 4;
constexpr int MRX = MTX + 2 * NG_MAX, MRY = MTY + 2 * NG_MAX;

__global__ void __launch_bounds__(256) k_metrics2d_fused(GridDev g, const double* __restrict__ x,
                                                         const double* __restrict__ xd,
                                                         const double* __restrict__ dt_dev, double coef,
                                                         double* __restrict__ met, double* __restrict__ J0) {
    __shared__ double xs[2][MRY][MRX];
    const int tid = threadIdx.y * MTX + threadIdx.x;
    const int i0 = -g.ng + (int)blockIdx.x * MTX, j0 = -g.ng + (int)blockIdx.y * MTY;
    const double cdt = dt_dev != nullptr ? coef * dt_dev[0] : 0.0;
    const double* xsd = dt_dev != nullptr ? xd : nullptr;
    for (int q = tid; q < MRX * MRY; q += MTX * MBY) {
        const int ri = q % MRX, rj = q / MRX;
        const int i = i0 - g.ng + ri, j = j0 - g.ng + rj;
        // positions beyond the extension box are never needed by padded nodes
        const bool ok = i >= -2 * g.ng && i < g.n[0] + 2 * g.ng && j >= -2 * g.ng && j < g.n[1] + 2 * g.ng;
        xs[0][rj][ri] = ok ? mesh_value(g, x, xsd, cdt, 0, i, j, 0, true) : 0.0;
        xs[1][rj][ri] = ok ? mesh_value(g, x, xsd, cdt, 1, i, j, 0, true) : 0.0;
    }
    __syncthreads();
    const long long P = g.pnodes;
    const int i = i0 + (int)threadIdx.x;
    if (i >= g.n[0] + g.ng) return;
    const int ri = threadIdx.x + g.ng;
    for (int row = threadIdx.y; row < MTY; row += MBY) {
        const int j = j0 + row;
        if (j >= g.n[1] + g.ng) break;
        const int rj = row + g.ng;
        double dxi[2], deta[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double s = 0.0, r = 0.0;
#pragma unroll
            for (int n = 1; n <= NG_MAX; ++n) {
                if (n > g.p) break;
                const double a = 0.5 * alpha_pn(g.p, n);
                s += a * (xs[c][rj][ri + n] - xs[c][rj][ri - n]);
                r += a * (xs[c][rj + n][ri] - xs[c][rj - n][ri]);
            }
            dxi[c] = s;
            deta[c] = r;
        }
        const long long t = pidx(g, i, j, 0);
        const double xix = deta[1] / g.dxi[1];
        const double xiy = -deta[0] / g.dxi[1];
        const double etx = -dxi[1] / g.dxi[0];
        const double ety = dxi[0] / g.dxi[0];
        double at0 = 0.0, at1 = 0.0;
        if (xd != nullptr) {
            const double vx = mesh_value(g, xd, nullptr, 0.0, 0, i, j, 0, false);
            const double vy = mesh_value(g, xd, nullptr, 0.0, 1, i, j, 0, false);
            at0 = -(vx * xix + vy * xiy);
            at1 = -(vx * etx + vy * ety);
        }
        met[0 * P + t] = at0;
        met[1 * P + t] = xix;
        met[2 * P + t] = xiy;
        met[3 * P + t] = at1;
        met[4 * P + t] = etx;
        met[5 * P + t] = ety;
        if (J0 != nullptr && i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1])
            J0[iidx(g, i, j, 0)] = (dxi[0] * deta[1] - deta[0] * dxi[1]) / (g.dxi[0] * g.dxi[1]);
    }
}

// The three stage metrics of an RK3 step in one launch (2D): the extended mesh X
// = x (with the periodic shift) and its velocity V are staged once per tile, the
// stage meshes are X + c_s dt V (c = 0, 1, 1/2), and the differences and the
// temporal metrics (velocity V at the node) are those of k_metrics2d_fused.
constexpr int MSY = 3 * MTY;   // threads per column: one per (stage, tile row)

__global__ void __launch_bounds__(MTX * MSY) k_metrics2d_stages(GridDev g, const double* __restrict__ x,
                                                               const double* __restrict__ xd,
                                                               const double* __restrict__ dt_dev,
                                                               double* __restrict__ met0,
                                                               double* __restrict__ met1,
                                                               double* __restrict__ met2) {
    __shared__ double xs[2][MRY][MRX];
    __shared__ double vs[2][MRY][MRX];
    const int tid = threadIdx.y * MTX + threadIdx.x;
    const int i0 = -g.ng + (int)blockIdx.x * MTX, j0 = -g.ng + (int)blockIdx.y * MTY;
    for (int q = tid; q < MRX * MRY; q += MTX * MSY) {
        const int ri = q % MRX, rj = q / MRX;
        const int i = i0 - g.ng + ri, j = j0 - g.ng + rj;
        const bool ok = i >= -2 * g.ng && i < g.n[0] + 2 * g.ng && j >= -2 * g.ng && j < g.n[1] + 2 * g.ng;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            xs[c][rj][ri] = ok ? mesh_value(g, x, nullptr, 0.0, c, i, j, 0, true) : 0.0;
            vs[c][rj][ri] = ok ? mesh_value(g, xd, nullptr, 0.0, c, i, j, 0, false) : 0.0;
        }
    }
    __syncthreads();
    const long long P = g.pnodes;
    const int i = i0 + (int)threadIdx.x;
    const int row = (int)threadIdx.y % MTY, st = (int)threadIdx.y / MTY;
    const int j = j0 + row;
    if (i >= g.n[0] + g.ng || j >= g.n[1] + g.ng) return;
    const int ri = threadIdx.x + g.ng, rj = row + g.ng;
    const double cdt = (st == 0 ? 0.0 : (st == 1 ? 1.0 : 0.5)) * dt_dev[0];
    const long long t = pidx(g, i, j, 0);
    const double vx = vs[0][rj][ri], vy = vs[1][rj][ri];
    double dxi[2], deta[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double s = 0.0, r = 0.0;
#pragma unroll
        for (int n = 1; n <= NG_MAX; ++n) {
            if (n > g.p) break;
            const double a = 0.5 * alpha_pn(g.p, n);
            s += a * ((xs[c][rj][ri + n] + cdt * vs[c][rj][ri + n]) - (xs[c][rj][ri - n] + cdt * vs[c][rj][ri - n]));
            r += a * ((xs[c][rj + n][ri] + cdt * vs[c][rj + n][ri]) - (xs[c][rj - n][ri] + cdt * vs[c][rj - n][ri]));
        }
        dxi[c] = s;
        deta[c] = r;
    }
    const double xix = deta[1] / g.dxi[1];
    const double xiy = -deta[0] / g.dxi[1];
    const double etx = -dxi[1] / g.dxi[0];
    const double ety = dxi[0] / g.dxi[0];
    double* met = st == 0 ? met0 : (st == 1 ? met1 : met2);
    met[0 * P + t] = -(vx * xix + vy * xiy);
    met[1 * P + t] = xix;
    met[2 * P + t] = xiy;
    met[3 * P + t] = -(vx * etx + vy * ety);
    met[4 * P + t] = etx;
    met[5 * P + t] = ety;
}

// 3D conservative metric method (eq. SCLCoeff): with the products
//   Pi_{a,j} = delta_a[x_{j+1}] x_{j+2}   (indices mod 3)
// on the extension box, J dxi_k/dx_j = (delta_{k+2}[Pi_{k+1,j}] - delta_{k+1}[Pi_{k+2,j}])
// / (dxi_{k+1} dxi_{k+2}).  Pi_{a,.} is formed where the a-coordinate lies within
// 3 layers of the interior (the metric differences never read it elsewhere).
__global__ void k_cmm_products(GridDev g, const double* __restrict__ xe, double* __restrict__ pi) {
    int i, j, k;
    if (!plane_cell_xcd(g.E[0], g.E[1], i, j, k)) return;
    i -= 2 * g.ng; j -= 2 * g.ng; k -= 2 * g.ng;
    const long long e = eidx(g, i, j, k);
    const long long EN = g.enodes;
    const int c[3] = {i, j, k};
    const long long st[3] = {1, (long long)g.E[0], (long long)g.E[0] * g.E[1]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool valid = c[a] >= -g.ng && c[a] < g.n[a] + g.ng;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            const int j1 = (jj + 1) % 3, j2 = (jj + 2) % 3;
            double v = 0.0;
            if (valid) {
                const double* xc = xe + j1 * EN + e;
                double d = 0.0;
#pragma unroll
                for (int n = 1; n <= NG_MAX; ++n)
                    if (n <= g.p) d += 0.5 * alpha_pn(g.p, n) * (xc[n * st[a]] - xc[-n * st[a]]);
                v = d * xe[j2 * EN + e];
            }
            pi[(a * 3 + jj) * EN + e] = v;
        }
    }
}

__global__ void k_metrics3d(GridDev g, const double* __restrict__ xe, const double* __restrict__ ve,
                            const double* __restrict__ pi, double* __restrict__ met,
                            double* __restrict__ J0) {
    int i, j, k;
    if (!box_ijk_xcd(-g.ng, -g.ng, -g.ng, g.P[0], g.P[1], i, j, k)) return;
    const long long t = pidx(g, i, j, k);
    const long long e = eidx(g, i, j, k);
    const long long EN = g.enodes;
    const long long P = g.pnodes;
    const long long st[3] = {1, (long long)g.E[0], (long long)g.E[0] * g.E[1]};
    double m[3][3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const int k1 = (kk + 1) % 3, k2 = (kk + 2) % 3;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            const double* pa = pi + (k1 * 3 + jj) * EN + e;   // Pi_{k1, j}, differenced along k2
            const double* pb = pi + (k2 * 3 + jj) * EN + e;   // Pi_{k2, j}, differenced along k1
            double ta = 0.0, tb = 0.0;
#pragma unroll
            for (int n = 1; n <= NG_MAX; ++n) {
                if (n > g.p) break;
                const double a = 0.5 * alpha_pn(g.p, n);
                ta += a * (pa[n * st[k2]] - pa[-n * st[k2]]);
                tb += a * (pb[n * st[k1]] - pb[-n * st[k1]]);
            }
            m[kk][jj] = (ta - tb) / (g.dxi[k1] * g.dxi[k2]);
        }
    }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        double at = 0.0;
        if (ve != nullptr) {
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) at -= ve[jj * EN + e] * m[kk][jj];
        }
        met[(kk * 4) * P + t] = at;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) met[(kk * 4 + 1 + jj) * P + t] = m[kk][jj];
    }
    if (J0 != nullptr && i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2]) {
        // J = sum_k (J dxi_k/dx_1) delta_k[x_1] / dxi_k
        double Jv = 0.0;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            double d = 0.0;
#pragma unroll
            for (int n = 1; n <= NG_MAX; ++n)
                if (n <= g.p) d += 0.5 * alpha_pn(g.p, n) * (xe[e + n * st[kk]] - xe[e - n * st[kk]]);
            Jv += m[kk][0] * d / g.dxi[kk];
        }
        J0[iidx(g, i, j, k)] = Jv;
    }
}

// The 3D metric differences in one pass after the stage mesh is extended: from the
// extended stage mesh (and mesh velocity) straight to the 12 padded metric
// components, the CMM products (eq. SCLCoeff) formed on the fly instead of in HBM.
// A block owns a 16 x 16 tile of padded (i, j) columns and marches through kz
// planes, with three threads per column, one per mesh component c (and, for the
// products Pi_{a,jj}, one per jj = c).  Each thread keeps its component of the stage
// mesh at planes k - H .. k + H for its own column and for one position of the
// H-wide cross-shaped halo, and the products Pi_{0,jj}, Pi_{1,jj} of its own column
// at the same planes (they are differenced along xi_3), in registers.  Per plane
// the block stages in LDS the mesh at the leading plane k + H (tile and cross), the
// mesh at the centre plane k (whole square: the corners are read directly) and its
// xi_3 differences (tile and cross), and the products Pi_{2,.} (tile and cross),
// Pi_{0,.} (tile and xi_2 strips) and Pi_{1,.} (tile and xi_1 strips) at the centre
// plane; the temporal part J dxi_k/dt = -sum_jj xdot_jj (J dxi_k/dx_jj) is summed
// from the row of spatial metrics left in LDS, at the start of the next plane.  The
// sums (in n order), the products and the temporal sum (in jj order) are those of
// k_cmm_products + k_metrics3d; the metric differences are scaled by the reciprocal
// of dxi_{k+1} dxi_{k+2}.  Every global load of a plane is issued one plane ahead,
// from clamped (always valid) addresses and outside any branch, so that its wait
// falls in the next plane.  The kernel is bound by LDS traffic (about 1.5 KB per
// node and plane); the three-kernel form it replaces (products in HBM, then a
// marching difference kernel reading them through L1/L2) took about twice as long.
constexpr int MT = 16;
constexpr int MT_THREADS = 3 * MT * MT;

template <int H>
struct MetTile {
    double xl[3][MT + 2 * H][MT + 2 * H];   // mesh at the leading plane (tile and cross)
    double xc[3][MT + 2 * H][MT + 2 * H];   // mesh at the centre plane (whole square)
    double dz[3][MT + 2 * H][MT + 2 * H];   // delta_3 of the mesh, centre plane (tile and cross)
    double p2[3][MT + 2 * H][MT + 2 * H];   // Pi_{2,.}, centre plane (tile and cross)
    double p0[3][MT + 2 * H][MT];           // Pi_{0,.}, centre plane (tile and xi_2 strips)
    double p1[3][MT][MT + 2 * H];           // Pi_{1,.}, centre plane (tile and xi_1 strips)
    double m[3][3][MT * MT];                // J dxi_kk/dx_jj of the centre plane, [kk][jj][column]
};

// offset of extension-box node (i, j, 0), each index clamped into the box
__device__ __forceinline__ long long eidx_clamped(const GridDev& g, int i, int j) {
    const int e = 2 * g.ng;
    return eidx(g, min(max(i, -e), g.n[0] + e - 1), min(max(j, -e), g.n[1] + e - 1), 0);
}

template <int H>
__global__ void __launch_bounds__(MT_THREADS) k_metrics3d_tile(GridDev g, const double* __restrict__ xe,
                                                               const double* __restrict__ ve,
                                                               double* __restrict__ met, int kz, int tiles0,
                                                               int tiles1) {
    constexpr int NCROSS = 4 * H * MT;
    constexpr int NCORNER = 4 * H * H;
    static_assert(NCROSS <= MT * MT && NCORNER <= MT * MT, "one halo position of each kind per thread");
    __shared__ MetTile<H> sm;
    const int c = (int)threadIdx.x / (MT * MT);   // mesh component (and jj) of this thread
    const int u = (int)threadIdx.x % (MT * MT);   // column of the tile
    const int j1 = (c + 1) % 3, j2 = (c + 2) % 3;
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int bx = lb % tiles0, by = (lb / tiles0) % tiles1, bz = lb / (tiles0 * tiles1);
    const int i0 = -g.ng + bx * MT, j0 = -g.ng + by * MT;
    const int kb = -g.ng + bz * kz, ke = min(kb + kz, g.n[2] + g.ng);
    // own column: square position (H + tx, H + ty)
    const int tx = u % MT, ty = u / MT;
    const int oi = i0 + tx, oj = j0 + ty;
    const bool store = oi < g.n[0] + g.ng && oj < g.n[1] + g.ng;
    // cross position: the xi_2 strips (rows 0..H-1 and MT+H..MT+2H-1 of the square)
    // first, then the xi_1 strips
    const bool has_c = u < NCROSS;
    const bool ystrip = u < 2 * H * MT;
    int cx = H, cy = H;
    if (ystrip) {
        const int r = u / MT;
        cx = H + u % MT;
        cy = r < H ? r : MT + r;
    } else if (has_c) {
        const int v = u - 2 * H * MT, r = v % (2 * H);
        cy = H + v / (2 * H);
        cx = r < H ? r : MT + r;
    }
    // corner position
    const bool has_k = u < NCORNER;
    int kx = 0, ky = 0;
    if (has_k) {
        const int r = u / (2 * H), q = u % (2 * H);
        ky = r < H ? r : MT + r;
        kx = q < H ? q : MT + q;
    }
    double a[H + 1];
#pragma unroll
    for (int n = 1; n <= H; ++n) a[n] = 0.5 * alpha_pn(g.p, n);
    const double c01 = 1.0 / (g.dxi[1] * g.dxi[2]), c20 = 1.0 / (g.dxi[2] * g.dxi[0]),
                 c12 = 1.0 / (g.dxi[0] * g.dxi[1]);
    const long long P = g.pnodes, EN = g.enodes;
    const long long tz = (long long)g.P[0] * g.P[1], sz = (long long)g.E[0] * g.E[1];
    // plane-0 offsets of the positions in the extension box (clamped: the positions
    // outside it belong to the ragged edge of the last tiles and are never used)
    const long long eo = eidx_clamped(g, oi, oj);
    const long long ec = eidx_clamped(g, i0 - H + cx, j0 - H + cy);
    const long long ek = eidx_clamped(g, i0 - H + kx, j0 - H + ky);
    const double* vsrc = ve != nullptr ? ve : xe;
    const double* xec = xe + c * EN;
    const int zlo = -2 * g.ng, zhi = g.n[2] + 2 * g.ng - 1;
    // windows (planes L - 2H .. L of the leading plane L): component c of the mesh at
    // the own column and at the cross position; Pi_{0,c}, Pi_{1,c} of the own column
    double wo[2 * H + 1], wc[2 * H + 1], w0[2 * H + 1], w1[2 * H + 1];
#pragma unroll
    for (int q = 0; q <= 2 * H; ++q) wo[q] = wc[q] = w0[q] = w1[q] = 0.0;
    // loads of leading plane L: component c of the mesh at the own column and the
    // cross position, of the corner's mesh at the centre plane L - H, and the three
    // components of the mesh velocity at the own column on the centre plane
    double no, nc, nk, nv[3];
    auto prefetch = [&](int L) {
        const long long zl = (long long)min(max(L, zlo), zhi) * sz;
        const long long zk = (long long)min(max(L - H, zlo), zhi) * sz;
        no = xec[eo + zl];
        nc = xec[ec + zl];
        nk = xec[ek + zk];
#pragma unroll
        for (int q = 0; q < 3; ++q) nv[q] = vsrc[q * EN + eo + zk];
    };
    // temporal metric kk = c of the plane whose spatial metrics are in sm.m
    auto temporal = [&](const double* v, long long t) {
        double at = 0.0;
        if (ve != nullptr) {
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) at -= v[jj] * sm.m[c][jj][u];
        }
        __builtin_nontemporal_store(at, &met[(c * 4) * P + t]);
    };
    prefetch(kb - H);
    long long tout = pidx(g, oi, oj, kb);
    double vp[3] = {0.0, 0.0, 0.0};   // mesh velocity of the previous centre plane
    for (int L = kb - H; L < ke + H; ++L) {
        const int k = L - H;
        const bool centre = k >= kb;
        // the previous centre plane's temporal metric (its row of sm.m is complete)
        if (k - 1 >= kb && store) temporal(vp, tout - tz);
#pragma unroll
        for (int q = 0; q < 2 * H; ++q) {
            wo[q] = wo[q + 1];
            wc[q] = wc[q + 1];
            w0[q] = w0[q + 1];
            w1[q] = w1[q + 1];
        }
        wo[2 * H] = no;
        wc[2 * H] = nc;
        const double kv = nk;
        double vv[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) vv[q] = nv[q];
        prefetch(L + 1);
        // leading plane (tile and cross) and, from the first centre plane on, the
        // centre mesh and its xi_3 differences
        sm.xl[c][H + ty][H + tx] = wo[2 * H];
        if (has_c) sm.xl[c][cy][cx] = wc[2 * H];
        if (centre) {
            sm.xc[c][H + ty][H + tx] = wo[H];
            if (has_c) sm.xc[c][cy][cx] = wc[H];
            if (has_k) sm.xc[c][ky][kx] = kv;
            double d = 0.0, e = 0.0;
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                d += a[n] * (wo[H + n] - wo[H - n]);
                e += a[n] * (wc[H + n] - wc[H - n]);
            }
            sm.dz[c][H + ty][H + tx] = d;
            if (has_c) sm.dz[c][cy][cx] = e;
        }
        __syncthreads();
        // Pi_{0,c} and Pi_{1,c} of the own column at the leading plane
        {
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                d0 += a[n] * (sm.xl[j1][H + ty][H + tx + n] - sm.xl[j1][H + ty][H + tx - n]);
                d1 += a[n] * (sm.xl[j1][H + ty + n][H + tx] - sm.xl[j1][H + ty - n][H + tx]);
            }
            const double x2 = sm.xl[j2][H + ty][H + tx];
            w0[2 * H] = d0 * x2;
            w1[2 * H] = d1 * x2;
        }
        if (centre) {
            // centre-plane Pi_{2,c} = delta_3[x_{c+1}] x_{c+2} (tile and cross), Pi_{0,c}
            // (tile from the window, xi_2 strips) and Pi_{1,c} (tile, xi_1 strips)
            sm.p2[c][H + ty][H + tx] = sm.dz[j1][H + ty][H + tx] * sm.xc[j2][H + ty][H + tx];
            sm.p0[c][H + ty][tx] = w0[H];
            sm.p1[c][ty][H + tx] = w1[H];
            if (has_c) {
                sm.p2[c][cy][cx] = sm.dz[j1][cy][cx] * sm.xc[j2][cy][cx];
                double d = 0.0;
                if (ystrip) {
#pragma unroll
                    for (int n = 1; n <= H; ++n) d += a[n] * (sm.xc[j1][cy][cx + n] - sm.xc[j1][cy][cx - n]);
                    sm.p0[c][cy][cx - H] = d * sm.xc[j2][cy][cx];
                } else {
#pragma unroll
                    for (int n = 1; n <= H; ++n) d += a[n] * (sm.xc[j1][cy + n][cx] - sm.xc[j1][cy - n][cx]);
                    sm.p1[c][cy - H][cx] = d * sm.xc[j2][cy][cx];
                }
            }
        }
        __syncthreads();
        if (centre && store) {
            double ta0 = 0.0, tb0 = 0.0, ta1 = 0.0, tb1 = 0.0, ta2 = 0.0, tb2 = 0.0;
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                // row 0: Pi_{1,c} along xi_3 minus Pi_{2,c} along xi_2
                ta0 += a[n] * (w1[H + n] - w1[H - n]);
                tb0 += a[n] * (sm.p2[c][H + ty + n][H + tx] - sm.p2[c][H + ty - n][H + tx]);
                // row 1: Pi_{2,c} along xi_1 minus Pi_{0,c} along xi_3
                ta1 += a[n] * (sm.p2[c][H + ty][H + tx + n] - sm.p2[c][H + ty][H + tx - n]);
                tb1 += a[n] * (w0[H + n] - w0[H - n]);
                // row 2: Pi_{0,c} along xi_2 minus Pi_{1,c} along xi_1
                ta2 += a[n] * (sm.p0[c][H + ty + n][tx] - sm.p0[c][H + ty - n][tx]);
                tb2 += a[n] * (sm.p1[c][ty][H + tx + n] - sm.p1[c][ty][H + tx - n]);
            }
            const double m0 = (ta0 - tb0) * c01, m1 = (ta1 - tb1) * c20, m2 = (ta2 - tb2) * c12;
            sm.m[0][c][u] = m0;
            sm.m[1][c][u] = m1;
            sm.m[2][c][u] = m2;
            __builtin_nontemporal_store(m0, &met[(0 * 4 + 1 + c) * P + tout]);
            __builtin_nontemporal_store(m1, &met[(1 * 4 + 1 + c) * P + tout]);
            __builtin_nontemporal_store(m2, &met[(2 * 4 + 1 + c) * P + tout]);
        }
        if (centre) {
            tout += tz;
#pragma unroll
            for (int q = 0; q < 3; ++q) vp[q] = vv[q];
        }
        __syncthreads();
    }
    if (store) temporal(vp, tout - tz);
}

// Temporal metrics J dxi_k/dt = -sum_j xdot_j (J dxi_k/dx_j) of a mesh whose
// spatial metrics are already in met (padded nodes; the mesh velocity extended
// as in k_mesh_extend): stage 0 of a 3D step, whose mesh is x^n.
__global__ void k_temporal_metrics3d(GridDev g, const double* __restrict__ xd, double* __restrict__ met) {
    int i, j, k;
    if (!plane_cell_xcd(g.P[0], g.P[1], i, j, k)) return;
    i -= g.ng; j -= g.ng; k -= g.ng;
    const long long t = pidx(g, i, j, k);
    const long long P = g.pnodes;
    // the spatial metrics, then the mesh velocity (loaded together at interior nodes)
    double m[3][3], v[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) m[kk][jj] = met[(kk * 4 + 1 + jj) * P + t];
    if (i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2]) {
        const long long nd = iidx(g, i, j, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = xd[c * g.nodes + nd];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = mesh_value(g, xd, nullptr, 0.0, c, i, j, k, false);
    }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        double at = 0.0;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) at -= v[jj] * m[kk][jj];
        met[(kk * 4) * P + t] = at;
    }
}

// ---------------------------------------------------------------------------
// residual: all direction sweeps in one launch
// ---------------------------------------------------------------------------
constexpr int LINES = 4;           // line segments (wavefronts) per block

template <int DIM, int PO>
struct ResidualLDS {
    static constexpr int NU = DIM, M = DIM + 2, NA = DIM + 1, NF = 6 + NU + NA;
    double sd[LINES][NF][seg_loads(PO) + 1];
    // 3D: the flux differences of each lane wait here while the face dissipation
    // runs (register pressure)
    double rs[DIM == 3 ? LINES : 1][M + 1][64];
};

// Orders the LDS accesses of one wavefront: its lanes exchange data only among
// themselves (each wavefront owns its line of the LDS buffer), so no block
// barrier is needed.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront per segment of the lines along DIR: loads the segment with its
// halo into LDS, evaluates the two-point fluxes owned by each node, the face
// dissipation and the flux differences, and writes this direction's part of the
// residual (m components and J) to out.  The fluxes F(s-n, s) and the
// dissipation of face s-1/2 come from the lanes that own them (lane shuffles).
//
// The lines are dealt to LINES sequences so that the wavefronts of a block work on
// adjacent lines (es_seq.h); segment w of a sequence holds 64 consecutive positions
// and owns the interior nodes among its lanes ng..63.  Flat layout: the positions
// of the lines' padded node sequences (n + 2 ng nodes each) laid end to end, so a
// segment may run across the end of one line into the next; every stencil an owned
// node uses stays within its own line's padded nodes, and the pair fluxes and faces
// that straddle two lines are computed and never used.  Aligned layout: ceil(n / SEG)
// segments per line.  Flat is taken where it saves at least an eighth of the
// wavefronts: aligned, a line of n = 128 nodes would take three, the third with 6
// owned nodes but the full instruction stream.
template <int DIM, int DIR, bool ES, bool MIXED, int PO>
__device__ __forceinline__ void residual_segment(const GridDev& g, double G, double eps,
                                                 const double* __restrict__ prim,
                                                 const double* __restrict__ met,
                                                 double* __restrict__ out, int blk, int nseg,
                                                 long long nlines, bool flat, int nsl,
                                                 ResidualLDS<DIM, PO>& lds) {
    constexpr int NU = DIM, M = DIM + 2, NA = DIM + 1;
    constexpr int NGP = ghost_layers(PO), SEGP = seg_nodes(PO), NLOADP = seg_loads(PO);
    constexpr int F_RHO = 0, F_P = 1, F_BETA = 2, F_W = 3, F_LR = 4, F_LB = 5, F_U = 6,
                  F_A = 6 + NU;
    auto& sd = lds.sd;

    const int lane = threadIdx.x & 63;
    const int line = threadIdx.x >> 6;
    // segment w (nseg of them per sequence) of sequence `line`; blk numbers this
    // sweep's blocks
    const long long w = blk;
    if (w >= nseg) return;
    const int nAlong = g.n[DIR];
    const int PL = nAlong + 2 * NGP;                    // padded nodes of a line
    const long long f0 = w * SEGP;                      // sequence position of lane 0
    const long long pstride = DIR == 0 ? 1 : (DIR == 1 ? (long long)g.P[0] : (long long)g.P[0] * g.P[1]);
    const long long istride = DIR == 0 ? 1 : (DIR == 1 ? (long long)g.n[0] : (long long)g.n[0] * g.n[1]);
    const long long P = g.pnodes;
    const long long N = g.nodes;
    // line and along-coordinate s (-ng .. n + ng - 1) of sequence position f0 + q,
    // and the padded / interior index of the line's node 0
    const int nf = DIR == 0 ? g.n[1] : g.n[0];
    const SeqBase sb = flat ? seq_base(f0, PL, NGP, nf, LINES, line)
                            : seq_base_aligned(w, nsl, SEGP, 0, NGP, nf, LINES, line);
    auto locate = [&](int q, long long& lid, int& s, long long& pbase, long long& ibase) {
        int fa, fb;
        seq_at(sb, q, flat, PL, NGP, nf, LINES, line, lid, s, fa, fb);
        if (s >= nAlong + NGP) lid = nlines;   // past the line's padded end (aligned)
        const int ci = DIR == 0 ? 0 : fa, cj = DIR == 0 ? fa : (DIR == 1 ? 0 : fb), ck = DIR == 2 ? 0 : fb;
        pbase = pidx(g, ci, cj, ck);
        ibase = iidx(g, ci, cj, ck);
    };

    // ---- load the segment with its halo into LDS.  Lane q holds position q and,
    // for q < NLOADP - 64, position 64 + q as well; the loads of both positions are
    // issued before the first of them is used, from addresses that are always valid
    // and outside any branch (a position off the lines reads node 0 and then takes
    // the far-field values instead), so the wavefront waits on memory once.
    static_assert(NLOADP > 64 && NLOADP <= 128, "two positions per lane");
    constexpr int NV = M + 2 + NA;   // rho, u, p, ln rho, ln beta, then the metrics
    auto index = [&](int q, bool use, long long& qlid, int& s, bool& ok) {
        long long pb, ib;
        locate(q, qlid, s, pb, ib);
        (void)ib;
        ok = use && qlid < nlines;
        return ok ? pb + (long long)s * pstride : 0;
    };
    auto fetch = [&](long long idx, double* v) {
#pragma unroll
        for (int c = 0; c < M + 2; ++c) v[c] = prim[c * P + idx];
#pragma unroll
        for (int c = 0; c < NA; ++c) v[M + 2 + c] = met[(DIR * NA + c) * P + idx];
    };
    auto stash = [&](int q, bool ok, const double* v) {
        const double rho = ok ? v[0] : 1.0, p = ok ? v[M - 1] : 1.0;
        double u[NU], uu = 0.0;
#pragma unroll
        for (int c = 0; c < NU; ++c) {
            u[c] = ok ? v[1 + c] : 0.0;
            uu += u[c] * u[c];
        }
        sd[line][F_RHO][q] = rho;
        sd[line][F_P][q] = p;
        sd[line][F_BETA][q] = rho * frcp(p);
        sd[line][F_W][q] = psqrt(1.0 + uu);
        sd[line][F_LR][q] = ok ? v[M] : 0.0;
        sd[line][F_LB][q] = ok ? v[M + 1] : 0.0;
#pragma unroll
        for (int c = 0; c < NU; ++c) sd[line][F_U + c][q] = u[c];
#pragma unroll
        for (int c = 0; c < NA; ++c) sd[line][F_A + c][q] = ok ? v[M + 2 + c] : (c == 1 ? 1.0 : 0.0);
    };
    // this lane's own node (position lane): only flags stay live (the output index
    // is formed again at the store)
    bool active, owner, face;
    {
        constexpr int NSEC = NLOADP - 64;
        const bool sec = lane < NSEC;
        double v0[NV], v1[NV];
        long long lid_own, lid1;
        int s_own, s1;
        bool ok0, ok1;
        const long long i0 = index(lane, true, lid_own, s_own, ok0);
        const long long i1 = index(64 + (sec ? lane : 0), sec, lid1, s1, ok1);
        fetch(i0, v0);
        fetch(i1, v1);
        // every load issued before any of them is used
        __builtin_amdgcn_sched_barrier(0);
        active = lid_own < nlines;
        owner = active && lane >= NGP && s_own >= 0 && s_own < nAlong;
        face = active && lane >= NGP - 1 && s_own >= -1 && s_own < nAlong;
        stash(lane, ok0, v0);
        // the lanes without a second position store their own again (the same
        // values): no branch, so the second loads are not sunk after the first wait
#pragma unroll
        for (int c = 0; c < NV; ++c) v1[c] = sec ? v1[c] : v0[c];
        stash(sec ? 64 + lane : lane, sec ? ok1 : ok0, v1);
    }
    wave_lds_sync();

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

    // ---- two-point fluxes (s, s+n), n = 1..p, owned by the lane of node s, and
    // flux differences R_s = -(1/dxi) sum_n alpha_n [F(s,s+n) - F(s-n,s)]
    const bool valid = active;
    const double idxi = 1.0 / g.dxi[DIR];
    double R[M + 1];
#pragma unroll
    for (int c = 0; c <= M; ++c) R[c] = 0.0;
    {
        NodeRHD<NU> l;
        double al[NA];
        if (valid) {
            l = node_at(lane);
#pragma unroll
            for (int c = 0; c < NA; ++c) al[c] = sd[line][F_A + c][lane];
        }
#pragma unroll
        for (int n = 1; n <= PO; ++n) {
            double F[M + 1];
#pragma unroll
            for (int c = 0; c <= M; ++c) F[c] = 0.0;
            if (valid) {
                const NodeRHD<NU> r = node_at(lane + n);
                double ar[NA];
#pragma unroll
                for (int c = 0; c < NA; ++c) ar[c] = sd[line][F_A + c][lane + n];
                if (MIXED) pair_flux_rhd_mixed<NU>(G, l, r, al, ar, F, F[M]);
                else pair_flux_rhd<NU>(G, l, r, al, ar, F, F[M]);
            }
            // all lanes take part in the shuffle; owners (lane >= ng) read F(s-n, s)
#pragma unroll
            for (int c = 0; c <= M; ++c) R[c] += alpha_pn(PO, n) * (F[c] - __shfl_up(F[c], n, 64));
            // one pair at a time (interleaving the three raises register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int c = 0; c <= M; ++c) R[c] = owner ? -R[c] * idxi : 0.0;

    if (ES) {
        constexpr bool STASH = DIM == 3;
        if (STASH) {
#pragma unroll
            for (int c = 0; c <= M; ++c) lds.rs[line][c][lane] = R[c];
        }
        // the fence makes the dissipation reload its stencil from LDS instead of
        // keeping the flux phase's node values live (register pressure)
        wave_lds_sync();
        // ---- face dissipation at s+1/2 for faces s in [-1, n) of the lane's line
        double d[M];
#pragma unroll
        for (int c = 0; c < M; ++c) d[c] = 0.0;
        if (face) {
            // the stencil states are read from LDS where they are used
            if (MIXED) {
                // FP32 dissipation from FP32 copies of the stencil states and metrics
                auto node_f = [&](int q) {
                    const int k = lane - (PO - 1) + q;
                    NodeRHD<NU, float> nd;
                    nd.rho = (float)sd[line][F_RHO][k];
                    nd.p = (float)sd[line][F_P][k];
                    nd.beta = (float)sd[line][F_BETA][k];
                    nd.W = (float)sd[line][F_W][k];
                    nd.lr = (float)sd[line][F_LR][k];
                    nd.lb = (float)sd[line][F_LB][k];
#pragma unroll
                    for (int c = 0; c < NU; ++c) nd.u[c] = (float)sd[line][F_U + c][k];
                    return nd;
                };
                float al[NA], ar[NA];
#pragma unroll
                for (int c = 0; c < NA; ++c) {
                    al[c] = (float)sd[line][F_A + c][lane];
                    ar[c] = (float)sd[line][F_A + c][lane + 1];
                }
                float df[M];
                face_diss_rhd_fn<DIM, float, PO>((float)G, (float)eps, node_f, al, ar, df);
#pragma unroll
                for (int c = 0; c < M; ++c) d[c] = (double)df[c];
            } else {
                double al[NA], ar[NA];
#pragma unroll
                for (int c = 0; c < NA; ++c) { al[c] = sd[line][F_A + c][lane]; ar[c] = sd[line][F_A + c][lane + 1]; }
                face_diss_rhd_fn<DIM, double, PO>(G, eps, [&](int q) { return node_at(lane - (PO - 1) + q); }, al, ar,
                                                  d);
            }
        }
        if (STASH) {
#pragma unroll
            for (int c = 0; c <= M; ++c) R[c] = lds.rs[line][c][lane];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double dm = __shfl_up(d[c], 1, 64);
            if (owner) R[c] += 0.5 * (d[c] - dm) * idxi;
        }
    }

    if (owner) {
        long long lid_own, pb, ib;
        int s_own;
        locate(lane, lid_own, s_own, pb, ib);
        const long long o = ib + (long long)s_own * istride;
#pragma unroll
        for (int c = 0; c <= M; ++c) out[c * N + o] = R[c];
    }
}

// Residual of all directions: logical blocks [0, nb0) sweep x, [nb0, nb0 + nb1)
// sweep y, the rest z; direction k writes slab k of Ld (m + 1 components each).
struct SweepPlan {
    int nseg[3];          // segments per sequence (blocks of the sweep)
    int nblk[3];          // blocks of the sweep
    long long nlines[3];  // lines of the sweep
    int flat[3];          // flat (1) or aligned (0) layout of the segments
    int nsl[3];           // segments per line of the aligned layout
};

template <int DIM, bool ES, bool MIXED, int PO>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_residual_rhd(GridDev g, double G, double eps,
                                                      const double* __restrict__ prim,
                                                      const double* __restrict__ met,
                                                      double* __restrict__ Ld, SweepPlan sw) {
    constexpr int M = DIM + 2;
    __shared__ ResidualLDS<DIM, PO> lds;
    const long long slab = (long long)(M + 1) * g.nodes;
    int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    if (b < sw.nblk[0]) {
        residual_segment<DIM, 0, ES, MIXED, PO>(g, G, eps, prim, met, Ld, b, sw.nseg[0], sw.nlines[0], sw.flat[0], sw.nsl[0], lds);
        return;
    }
    b -= sw.nblk[0];
    if (DIM == 2 || b < sw.nblk[1]) {
        residual_segment<DIM, 1, ES, MIXED, PO>(g, G, eps, prim, met, Ld + slab, b, sw.nseg[1], sw.nlines[1], sw.flat[1], sw.nsl[1], lds);
        return;
    }
    b -= sw.nblk[1];
    if (DIM == 3)
        residual_segment<DIM, 2, ES, MIXED, PO>(g, G, eps, prim, met, Ld + 2 * slab, b, sw.nseg[2], sw.nlines[2], sw.flat[2], sw.nsl[2], lds);
}

// dU = sum_k Ld_k (components 0..m-1), dJ = sum_k Ld_k (component m), summed in
// direction order.
__global__ void k_sum_dirs(long long N, int M, int dim, const double* __restrict__ Ld,
                           double* __restrict__ dU, double* __restrict__ dJ) {
    const long long t = gtid();
    if (t >= N * (M + 1)) return;
    const long long slab = (long long)(M + 1) * N;
    double v = Ld[t] + Ld[slab + t];
    if (dim == 3) v += Ld[2 * slab + t];
    if (t < N * M) dU[t] = v; else dJ[t - N * M] = v;
}

// Monitor at interior node (i, j, k) (Section 5): |grad sigma| from central
// differences in computational space (one-sided at outflow edges), stored in w
// as omega = sqrt(1 + alpha |grad sigma|^2) (sqgrad) or as |grad sigma| for the
// later normalisation by its maximum; returns the value that enters that maximum.
template <int DIM>
__device__ __forceinline__ double monitor_node(const GridDev& g, int M, int sigma_ln, int sqgrad, double alpha,
                                               const double* __restrict__ prim, double* __restrict__ w,
                                               int i, int j, int k) {
    const long long P = g.pnodes;
    const int c[3] = {i, j, k};
    const long long pc = pidx(g, i, j, k);
    const long long off = sigma_ln ? M * P : 0;
    const long long strides[3] = {1, (long long)g.P[0], (long long)g.P[0] * g.P[1]};
    double g2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        // neighbours through the solution rule: ghosts of the padded box hold
        // the periodic copies, so only outflow edges need the one-sided form
        const double sp = prim[off + pc + strides[a]];
        const double sm = prim[off + pc - strides[a]];
        const double s0 = prim[off + pc];
        double d;
        if (g.bc[a] == ES_BC_PERIODIC || (c[a] > 0 && c[a] < g.n[a] - 1)) d = (sp - sm) / (2.0 * g.dxi[a]);
        else if (c[a] == 0) d = (sp - s0) / g.dxi[a];
        else d = (s0 - sm) / g.dxi[a];
        g2 += d * d;
    }
    const long long t = iidx(g, i, j, k);
    if (sqgrad) {
        w[t] = sqrt(1.0 + alpha * g2);
        return 0.0;
    }
    const double gn = sqrt(g2);
    w[t] = gn;
    return gn;
}

// ---------------------------------------------------------------------------
// CFL (eq. cfl): per-direction maxima of rho_k = L_k max|lambda| / J
// ---------------------------------------------------------------------------
// rho_k = L_k max|lambda_pm| / J at padded node pi for the spatial metrics ax[k]
// (the acoustic speeds bound |v_n|)
template <int DIM>
__device__ __forceinline__ void cfl_node(double G, const double* __restrict__ prim, long long P,
                                         long long pi, double Jv, const double (&ax)[DIM][DIM],
                                         double* mx) {
    constexpr int M = DIM + 2;
    const double rho = prim[pi], p = prim[(M - 1) * P + pi];
    double u[DIM], uu = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) { u[c] = prim[(1 + c) * P + pi]; uu += u[c] * u[c]; }
    const double W = sqrt(1.0 + uu);
    const double v2 = uu / (W * W);
    const double h = 1.0 + G / (G - 1.0) * p / rho;
    const double cs2 = G * p / (rho * h);
    const double cs = sqrt(cs2);
    const double iJ = 1.0 / Jv;
#pragma unroll
    for (int kd = 0; kd < DIM; ++kd) {
        double L2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) L2 += ax[kd][c] * ax[kd][c];
        const double L = sqrt(L2);
        double vn = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) vn += ax[kd][c] * u[c];
        vn = vn / (L * W);
        const double disc = sqrt((1.0 - v2) * (1.0 - v2 * cs2 - vn * vn * (1.0 - cs2)));
        const double iden = 1.0 / (1.0 - v2 * cs2);
        const double lm = (vn * (1.0 - cs2) - cs * disc) * iden;
        const double lp = (vn * (1.0 - cs2) + cs * disc) * iden;
        mx[kd] = L * fmax(fabs(lm), fabs(lp)) * iJ;
    }
}

template <int DIM>
__global__ void __launch_bounds__(256) k_cfl_partial(GridDev g, double G, const double* __restrict__ prim,
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
        double ax[DIM][DIM];
#pragma unroll
        for (int kd = 0; kd < DIM; ++kd)
#pragma unroll
            for (int c = 0; c < DIM; ++c) ax[kd][c] = met[(kd * NA + 1 + c) * P + pi];
        cfl_node<DIM>(G, prim, P, pi, J[iidx(g, i, j, k)], ax, mx);
    }
    const int nb = (int)(gridDim.x * gridDim.y * gridDim.z);
#pragma unroll
    for (int kd = 0; kd < DIM; ++kd) {
        const double r = block_reduce<0>(mx[kd], sh);
        if (flat_tid() == 0) partial[kd * nb + flat_block()] = r;
    }
}

// CFL maxima with the spatial metrics of x formed in the kernel (2D): a block
// stages the extended mesh of its 64 x 4 interior tile plus a 3-node halo in
// LDS (as k_metrics2d_fused) and evaluates the metrics at its nodes from there.
struct MonitorArgs {
    int enabled, M, sigma_ln, sqgrad;
    double alpha;
    double* w;         // interior omega (or |grad sigma|)
    double* partial;   // block maxima of |grad sigma|
};

// 64 x 8 threads per 64 x 4 tile: all stage the mesh (about two positions each);
// rows 0-3 then evaluate the CFL speeds, rows 4-7 the monitor.
constexpr int CBY = 8;

__global__ void __launch_bounds__(MTX * CBY) k_cfl_partial2d_mesh(GridDev g, double G,
                                                                 const double* __restrict__ prim,
                                                                 const double* __restrict__ x,
                                                                 const double* __restrict__ J,
                                                                 double* __restrict__ partial, MonitorArgs mon) {
    __shared__ double xs[2][MRY][MRX];
    __shared__ double sh[MTX * CBY / 64];
    const int tid = threadIdx.y * MTX + threadIdx.x;
    const int i0 = (int)blockIdx.x * MTX, j0 = (int)blockIdx.y * MBY;
    const int role = (int)threadIdx.y / MBY;       // 0: CFL, 1: monitor, 2: staging only
    const int i = i0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y % MBY;
    const bool inside = i < g.n[0] && j < g.n[1];
    // the monitor needs no metrics: its loads overlap the mesh staging
    double gmx = 0.0;
    if (role == 1 && mon.enabled && inside)
        gmx = monitor_node<2>(g, mon.M, mon.sigma_ln, mon.sqgrad, mon.alpha, prim, mon.w, i, j, 0);
    for (int q = tid; q < MRX * (MBY + 2 * g.ng); q += MTX * CBY) {
        const int ri = q % MRX, rj = q / MRX;
        const int ii = i0 - g.ng + ri, jj = j0 - g.ng + rj;
        const bool ok = ii < g.n[0] + 2 * g.ng && jj < g.n[1] + 2 * g.ng;
        xs[0][rj][ri] = ok ? mesh_value(g, x, nullptr, 0.0, 0, ii, jj, 0, true) : 0.0;
        xs[1][rj][ri] = ok ? mesh_value(g, x, nullptr, 0.0, 1, ii, jj, 0, true) : 0.0;
    }
    __syncthreads();
    double mx[2] = {0.0, 0.0};
    if (role == 0 && inside) {
        const int ri = threadIdx.x + g.ng, rj = threadIdx.y + g.ng;
        double dxi[2], deta[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double s = 0.0, r = 0.0;
#pragma unroll
            for (int n = 1; n <= NG_MAX; ++n) {
                if (n > g.p) break;
                const double a = 0.5 * alpha_pn(g.p, n);
                s += a * (xs[c][rj][ri + n] - xs[c][rj][ri - n]);
                r += a * (xs[c][rj + n][ri] - xs[c][rj - n][ri]);
            }
            dxi[c] = s;
            deta[c] = r;
        }
        const double ax[2][2] = {{deta[1] / g.dxi[1], -deta[0] / g.dxi[1]},
                                 {-dxi[1] / g.dxi[0], dxi[0] / g.dxi[0]}};
        cfl_node<2>(G, prim, g.pnodes, pidx(g, i, j, 0), J[iidx(g, i, j, 0)], ax, mx);
    }
    const int nb = (int)(gridDim.x * gridDim.y);
#pragma unroll
    for (int kd = 0; kd < 2; ++kd) {
        const double r = block_reduce<0>(mx[kd], sh);
        if (tid == 0) partial[kd * nb + flat_block()] = r;
    }
    if (mon.enabled) {
        const double r = block_reduce<0>(gmx, sh);
        if (tid == 0) mon.partial[flat_block()] = r;
    }
}

// Final reduction of the CFL partial maxima into dt (one block; every thread of
// the block must call it).
struct DtFinal {
    const double* partial;   // dim slabs of nb block maxima
    int nb, dim;
    double cfl, dx[3];
    const double* fixed_dt;  // optional prescribed dt
    double* dt_out;
};

template <int RU>
__device__ __forceinline__ void finalize_dt(const DtFinal& f, double* sh) {
    // a prescribed dt needs no reduction (the same branch for the whole block)
    if (f.fixed_dt != nullptr) {
        if (flat_tid() == 0) f.dt_out[0] = f.fixed_dt[0];
        return;
    }
    // RU partials per slab and thread are loaded before any is used (RU sized so
    // that one pass covers the caller's typical count); an index past the last
    // partial reads the last one again, which leaves a maximum unchanged (the three
    // slabs are allocated in 2D too; the third is not used there)
    const int tid = flat_tid(), nt = (int)(blockDim.x * blockDim.y * blockDim.z);
    double m[3] = {0.0, 0.0, 0.0};
    for (int b0 = tid; b0 < f.nb; b0 += RU * nt) {
        double q[3][RU];
#pragma unroll
        for (int kd = 0; kd < 3; ++kd)
#pragma unroll
            for (int u = 0; u < RU; ++u) q[kd][u] = f.partial[kd * f.nb + min(b0 + u * nt, f.nb - 1)];
#pragma unroll
        for (int kd = 0; kd < 3; ++kd)
#pragma unroll
            for (int u = 0; u < RU; ++u) m[kd] = fmax(m[kd], q[kd][u]);
    }
    double tot = 0.0;
    for (int kd = 0; kd < f.dim; ++kd) tot += block_reduce<0>(m[kd], sh) / f.dx[kd];
    if (tid == 0) f.dt_out[0] = f.fixed_dt != nullptr ? f.fixed_dt[0] : f.cfl / tot;
}

constexpr int FINAL_TPB = 1024;   // threads of the one-block final reductions

__global__ void __launch_bounds__(FINAL_TPB) k_cfl_final(DtFinal f) {
    __shared__ double sh[FINAL_TPB / 64];
    finalize_dt<8>(f, sh);
}

// ---------------------------------------------------------------------------
// mesh redistribution (Section 5)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256) k_monitor_grad(GridDev g, int M, int sigma_ln, int sqgrad,
                                                      double alpha, const double* __restrict__ prim,
                                                      double* __restrict__ w, double* __restrict__ partial) {
    __shared__ double sh[8];
    double mx = 0.0;
    int i, j, k;
    if (box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) mx = monitor_node<DIM>(g, M, sigma_ln, sqgrad, alpha, prim, w, i, j, k);
    const double r = block_reduce<0>(mx, sh);
    if (flat_tid() == 0) partial[flat_block()] = r;
}

// |Lap_xi sigma| at an interior node (eq. RMHD_2DVortex_Monitor): three-point
// second differences, central where both neighbours are on the axis (ghosts of
// periodic axes hold the periodic copies), else the three nearest nodes
template <int DIM>
__device__ __forceinline__ double laplacian_node(const GridDev& g, int M, int sigma_ln,
                                                 const double* __restrict__ prim, int i, int j, int k) {
    const long long P = g.pnodes;
    const int c[3] = {i, j, k};
    const long long pc = pidx(g, i, j, k);
    const long long off = sigma_ln ? M * P : 0;
    const long long strides[3] = {1, (long long)g.P[0], (long long)g.P[0] * g.P[1]};
    double lap = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        long long ctr = pc;
        if (g.bc[a] != ES_BC_PERIODIC) {
            if (c[a] == 0) ctr += strides[a];
            else if (c[a] == g.n[a] - 1) ctr -= strides[a];
        }
        const double d2 = prim[off + ctr + strides[a]] - 2.0 * prim[off + ctr] + prim[off + ctr - strides[a]];
        lap += d2 / (g.dxi[a] * g.dxi[a]);
    }
    return fabs(lap);
}

// gradient + Laplacian monitor: |grad sigma| into w, |Lap sigma| into w2 and the
// block maxima of both (partial: grad slab, then Laplacian slab of nb entries)
template <int DIM>
__global__ void __launch_bounds__(256) k_monitor_gradlap(GridDev g, int M, int sigma_ln,
                                                         const double* __restrict__ prim,
                                                         double* __restrict__ w, double* __restrict__ w2,
                                                         double* __restrict__ pgrad, double* __restrict__ plap) {
    __shared__ double sh[8];
    double mg = 0.0, ml = 0.0;
    int i, j, k;
    if (box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) {
        mg = monitor_node<DIM>(g, M, sigma_ln, 0, 0.0, prim, w, i, j, k);
        ml = laplacian_node<DIM>(g, M, sigma_ln, prim, i, j, k);
        w2[iidx(g, i, j, k)] = ml;
    }
    const double rg = block_reduce<0>(mg, sh);
    if (flat_tid() == 0) pgrad[flat_block()] = rg;
    const double rl = block_reduce<0>(ml, sh);
    if (flat_tid() == 0) plap[flat_block()] = rl;
}

// omega = sqrt(1 + alpha g / max g + alpha2 l / max l), a term with a zero maximum dropped
__global__ void k_monitor_apply_gradlap(long long n, double alpha, double alpha2,
                                        const double* __restrict__ gmax, const double* __restrict__ lmax,
                                        double* __restrict__ w, const double* __restrict__ w2) {
    const long long t = gtid();
    if (t >= n) return;
    const double mg = gmax[0], ml = lmax[0];
    double v = 1.0;
    if (mg > 0.0) v += alpha * w[t] / mg;
    if (ml > 0.0) v += alpha2 * w2[t] / ml;
    w[t] = sqrt(v);
}

// one-block reduction of partial maxima (op 0) or minima capped at 1 (op 1)
__global__ void __launch_bounds__(FINAL_TPB) k_reduce_final(int op, int nb, const double* __restrict__ partial,
                                                            double* __restrict__ out) {
    __shared__ double sh[FINAL_TPB / 64];
    double v = op == 0 ? 0.0 : 1.0;
    // RU partials per thread loaded before any is used; an index past the last
    // partial reads the last one again (maximum and minimum are unchanged by it)
    constexpr int RU = 8;
    const int nt = (int)blockDim.x;
    for (int b0 = threadIdx.x; b0 < nb; b0 += RU * nt) {
        double q[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) q[u] = partial[min(b0 + u * nt, nb - 1)];
#pragma unroll
        for (int u = 0; u < RU; ++u) v = op == 0 ? fmax(v, q[u]) : fmin(v, q[u]);
    }
    v = op == 0 ? block_reduce<0>(v, sh) : block_reduce<1>(v, sh);
    if (threadIdx.x == 0) out[0] = v;
}

__global__ void k_monitor_apply(long long n, double alpha, const double* __restrict__ gmax,
                                double* __restrict__ w) {
    const long long t = gtid();
    if (t >= n) return;
    const double m = gmax[0];
    w[t] = m == 0.0 ? 1.0 : sqrt(1.0 + alpha * w[t] / m);
}

template <int DIM>
__global__ void k_filter(GridDev g, const double* __restrict__ win, double* __restrict__ wout) {
    int i, j, k;
    if (!box_ijk_xcd(0, 0, 0, g.n[0], g.n[1], i, j, k)) return;
    double s = 0.0;
    if (DIM == 2) {
        for (int o0 = -1; o0 <= 1; ++o0) {
            const int ii = map_sol(i + o0, g.n[0], g.bc[0]);
            for (int o1 = -1; o1 <= 1; ++o1) {
                const int jj = map_sol(j + o1, g.n[1], g.bc[1]);
                const int e = abs(o0) + abs(o1) + 2;
                s += ldexp(1.0, -e) * win[iidx(g, ii, jj, 0)];
            }
        }
    } else {
        // the 27 neighbour indices (map_sol of an interior index +- 1, without its
        // branches), then all loads before the first use, then the sum in the order
        // o0, o1, o2
        const int* n = g.n;
        auto nb = [&](int v, int a) {
            const bool per = g.bc[a] == ES_BC_PERIODIC;
            return v < 0 ? (per ? n[a] - 1 : 0) : (v >= n[a] ? (per ? 0 : n[a] - 1) : v);
        };
        int ia[3], ja[3], ka[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            ia[o] = nb(i + o - 1, 0);
            ja[o] = nb(j + o - 1, 1);
            ka[o] = nb(k + o - 1, 2);
        }
        double v[27];
#pragma unroll
        for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
            for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2) v[(o0 * 3 + o1) * 3 + o2] = win[iidx(g, ia[o0], ja[o1], ka[o2])];
        // every load issued before any of them is used
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
            for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2) {
                    const int e = (o0 != 1) + (o1 != 1) + (o2 != 1) + 3;
                    s += ldexp(1.0, -e) * v[(o0 * 3 + o1) * 3 + o2];
                }
    }
    wout[iidx(g, i, j, k)] = s;
}

// Monitor normalisation and up to FH low-pass filter passes in one launch (2D):
// a block stages its 64 x 4 tile of omega plus an FH-node halo in LDS, applies
// omega = sqrt(1 + alpha |grad sigma| / max |grad sigma|) at load (paper form;
// apply = 0 when the input already holds omega) and the 3x3 filter of k_filter
// `passes` times on the shrinking valid region.  Neighbours beyond an outflow
// edge read the clamped edge value (the zero-gradient ghost); periodic copies
// are filtered as the originals.
constexpr int FTX = 64, FTY = 4, FH = 5;
constexpr int FRX = FTX + 2 * FH, FRY = FTY + 2 * FH;
constexpr int FBY = 8;    // 64 x 8 threads: about two region positions per thread

// With apply, every block reduces the nb partial maxima of |grad sigma| itself
// (no separate reduction launch); with dt_fin, block 0 also finalises dt.
__global__ void __launch_bounds__(FTX * FBY) k_monitor_filter2d(GridDev g, int apply, double alpha,
                                                          const double* __restrict__ gpart, int nb,
                                                          int passes, const double* __restrict__ win,
                                                          double* __restrict__ wout, DtFinal dt_fin) {
    __shared__ double ws[2][FRY][FRX];
    __shared__ double sh[FTX * FBY / 64];
    const int tid = threadIdx.y * FTX + threadIdx.x;
    const int i0 = (int)blockIdx.x * FTX - FH, j0 = (int)blockIdx.y * FTY - FH;
    const int n0 = g.n[0], n1 = g.n[1];
    if (dt_fin.dt_out != nullptr && blockIdx.x == 0 && blockIdx.y == 0) finalize_dt<2>(dt_fin, sh);
    double m = 0.0;
    if (apply) {
        for (int b = tid; b < nb; b += FTX * FBY) m = fmax(m, gpart[b]);
        m = block_reduce<0>(m, sh);
    }
    for (int q = tid; q < FRX * FRY; q += FTX * FBY) {
        const int ri = q % FRX, rj = q / FRX;
        const int ii = map_sol(i0 + ri, n0, g.bc[0]), jj = map_sol(j0 + rj, n1, g.bc[1]);
        double v = win[(long long)jj * n0 + ii];
        if (apply) v = m == 0.0 ? 1.0 : sqrt(1.0 + alpha * v / m);
        ws[0][rj][ri] = v;
    }
    __syncthreads();
    const bool per0 = g.bc[0] == ES_BC_PERIODIC, per1 = g.bc[1] == ES_BC_PERIODIC;
    // region index of the neighbour read: outflow positions clamp to the domain
    auto rx = [&](int ri, int o) {
        int gi = i0 + ri + o;
        if (!per0) gi = gi < 0 ? 0 : (gi >= n0 ? n0 - 1 : gi);
        return gi - i0;
    };
    auto ry = [&](int rj, int o) {
        int gj = j0 + rj + o;
        if (!per1) gj = gj < 0 ? 0 : (gj >= n1 ? n1 - 1 : gj);
        return gj - j0;
    };
    int cur = 0;
    for (int ps = 1; ps <= passes; ++ps) {
        for (int q = tid; q < FRX * FRY; q += FTX * FBY) {
            const int ri = q % FRX, rj = q / FRX;
            double v = ws[cur][rj][ri];
            if (ri >= ps && ri < FRX - ps && rj >= ps && rj < FRY - ps) {
                double s = 0.0;
                for (int o0 = -1; o0 <= 1; ++o0) {
                    const int xi = rx(ri, o0);
                    for (int o1 = -1; o1 <= 1; ++o1) {
                        const int e = abs(o0) + abs(o1) + 2;
                        s += ldexp(1.0, -e) * ws[cur][ry(rj, o1)][xi];
                    }
                }
                v = s;
            }
            ws[cur ^ 1][rj][ri] = v;
        }
        cur ^= 1;
        __syncthreads();
    }
    const int gi = (int)blockIdx.x * FTX + threadIdx.x, gj = (int)blockIdx.y * FTY + threadIdx.y;
    if (threadIdx.y < FTY && gi < n0 && gj < n1)
        wout[(long long)gj * n0 + gi] = ws[cur][threadIdx.y + FH][threadIdx.x + FH];
}

// Value of mesh component q at the neighbour c + s e_a of interior node c: a
// direct load inside the box, the periodic copy with its shift across a
// periodic edge (the Jacobi and limiter rules never look across an outflow edge).
template <int DIM>
__device__ __forceinline__ double mesh_nb(const GridDev& g, const double* __restrict__ x, int q,
                                          const int* c, int a, int s) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[a] += s;
    double shift = 0.0;
    if (cc[a] < 0) { cc[a] += g.n[a]; if (q == a) shift = -g.period[a]; }
    else if (cc[a] >= g.n[a]) { cc[a] -= g.n[a]; if (q == a) shift = g.period[a]; }
    return x[(long long)q * g.nodes + iidx(g, cc[0], cc[1], cc[2])] + shift;
}

// One Jacobi sweep of the mesh equations over the axes along which a node is free.
// The neighbours c +- e_a are wrapped across the box (the periodic copies, with the
// coordinate shift of component a); along an outflow axis only the nodes off its
// edges are free, and their neighbours never wrap (a fixed node's wrapped
// neighbours are loaded and not used).  Every load is issued before the first is
// used, with no branch around them, so that a sweep waits on memory once.
template <int DIM>
__global__ void k_jacobi(GridDev g, const double* __restrict__ w, const double* __restrict__ xin,
                         double* __restrict__ xout) {
    int i, j, k;
    if (!box_ijk_xcd(0, 0, 0, g.n[0], g.n[1], i, j, k)) return;
    const int c[3] = {i, j, k};
    const long long t = iidx(g, i, j, k);
    const long long N = g.nodes;
    const long long stride[3] = {1, (long long)g.n[0], (long long)g.n[0] * g.n[1]};
    bool fr[3];
    long long tp[3], tm[3];
    double sp[3], sm[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        fr[a] = g.bc[a] == ES_BC_PERIODIC || (c[a] > 0 && c[a] < g.n[a] - 1);
        const bool wrap_p = c[a] + 1 >= g.n[a], wrap_m = c[a] < 1;
        tp[a] = t + (wrap_p ? (long long)(1 - g.n[a]) : 1LL) * stride[a];
        tm[a] = t + (wrap_m ? (long long)(g.n[a] - 1) : -1LL) * stride[a];
        sp[a] = wrap_p ? g.period[a] : 0.0;
        sm[a] = wrap_m ? -g.period[a] : 0.0;
    }
    const double wc = w[t];
    double wp[3], wm[3], xp[3][3], xm[3][3], xc[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        wp[a] = w[tp[a]];
        wm[a] = w[tm[a]];
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
            xp[a][q] = xin[q * N + tp[a]];
            xm[a][q] = xin[q * N + tm[a]];
        }
    }
#pragma unroll
    for (int q = 0; q < DIM; ++q) xc[q] = xin[q * N + t];
    // every load issued before any of them is used
    __builtin_amdgcn_sched_barrier(0);
    double den = 0.0, num[DIM];
#pragma unroll
    for (int q = 0; q < DIM; ++q) num[q] = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dn = den + (2.0 * wc + wp[a] + wm[a]);
        den = fr[a] ? dn : den;
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
            const double xpv = xp[a][q] + (q == a ? sp[a] : 0.0);
            const double xmv = xm[a][q] + (q == a ? sm[a] : 0.0);
            const double nq = num[q] + ((wc + wp[a]) * xpv + (wc + wm[a]) * xmv);
            num[q] = fr[a] ? nq : num[q];
        }
    }
#pragma unroll
    for (int q = 0; q < DIM; ++q) xout[q * N + t] = (fr[q] && den > 0.0) ? num[q] / den : xc[q];
}

// Largest admissible pseudo-time fraction at interior node c (index t) for the
// relaxed coordinates xm_a (eq. dtau): a node moves at most half-way towards its
// neighbour along each coordinate direction.
template <int DIM>
__device__ __forceinline__ double dtau_bound(const GridDev& g, const double* __restrict__ x,
                                             const int* c, long long t, const double* xm) {
    double best = 1.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const long long o = (long long)a * g.nodes + t;
        const double dk = xm[a] - x[o];
        if (dk == 0.0) continue;       // fixed coordinates (outflow edges) never move
        const double nb = mesh_nb<DIM>(g, x, a, c, a, dk > 0.0 ? 1 : -1);
        const double b = dk < 0.0 ? -(x[o] - nb) / (2.0 * dk) : (nb - x[o]) / (2.0 * dk);
        best = fmin(best, b);
    }
    return best;
}

// Several Jacobi sweeps in one launch (2D): a block stages its TX x TY tile of
// outputs with a halo of JS nodes (x and omega) in LDS and applies the sweep of
// k_jacobi `sweeps` <= JS times to the shrinking valid region; periodic copies
// carry the coordinate shift (the sweep is an average with weights summing to
// one, so shifted copies evolve as the shifted originals); positions outside an
// outflow edge are never read by the nodes a sweep updates.
constexpr int JTX = 64, JTY = 8, JS = 5;
constexpr int JRX = JTX + 2 * JS, JRY = JTY + 2 * JS;
constexpr int JNT = 1024;   // threads per block: about one region position per thread

// With dtau_part (last launch), each block also writes the minimum of the
// Delta tau bound over its tile (x0: the mesh before the sweeps).
__global__ void __launch_bounds__(JNT) k_jacobi_multi2d(GridDev g, int sweeps, const double* __restrict__ w,
                                                        const double* __restrict__ xin,
                                                        double* __restrict__ xout,
                                                        const double* __restrict__ x0,
                                                        double* __restrict__ dtau_part) {
    __shared__ double xs[2][2][JRY][JRX];
    __shared__ double ws[JRY][JRX];
    __shared__ double sh[JNT / 64];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * JTX - JS, j0 = blockIdx.y * JTY - JS;
    const int n0 = g.n[0], n1 = g.n[1];
    const bool per0 = g.bc[0] == ES_BC_PERIODIC, per1 = g.bc[1] == ES_BC_PERIODIC;
    for (int q = tid; q < JRX * JRY; q += JNT) {
        const int ri = q % JRX, rj = q / JRX;
        int gi = i0 + ri, gj = j0 + rj;
        double sh0 = 0.0, sh1 = 0.0;
        bool ok = true;
        if (gi < 0 || gi >= n0) {
            if (per0) { const int wr = floordiv(gi, n0); gi -= wr * n0; sh0 = wr * g.period[0]; }
            else ok = false;
        }
        if (gj < 0 || gj >= n1) {
            if (per1) { const int wr = floordiv(gj, n1); gj -= wr * n1; sh1 = wr * g.period[1]; }
            else ok = false;
        }
        double a = 0.0, b = 0.0, ww = 0.0;
        if (ok) {
            const long long t = (long long)gj * n0 + gi;
            a = xin[t] + sh0;
            b = xin[g.nodes + t] + sh1;
            ww = w[t];
        }
        xs[0][0][rj][ri] = a;
        xs[0][1][rj][ri] = b;
        ww = ok ? ww : 1.0;
        ws[rj][ri] = ww;
    }
    __syncthreads();
    // each thread keeps the sweep coefficients of its region positions in
    // registers: x_new = sum_k c_k x_k over the four neighbours, c_k = (w_c +
    // w_k) / den over the free axes; flags: bit 0 / 1 = component 0 / 1 is
    // updated (its axis is free and den > 0), bits 2.. = depth in the region
    // (the position is valid for sweeps up to its depth)
    constexpr int NQ = (JRX * JRY + JNT - 1) / JNT;
    double cf[NQ][4];
    int fl[NQ];
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const int q = tid + JNT * r;
        cf[r][0] = cf[r][1] = cf[r][2] = cf[r][3] = 0.0;
        fl[r] = 0;
        if (q < JRX * JRY) {
            const int ri = q % JRX, rj = q / JRX;
            const int depth = min(min(ri, JRX - 1 - ri), min(rj, JRY - 1 - rj));
            if (depth >= 1) {
                const int gi = i0 + ri, gj = j0 + rj;
                const bool fr0 = per0 || (gi > 0 && gi < n0 - 1);
                const bool fr1 = per1 || (gj > 0 && gj < n1 - 1);
                const double wc = ws[rj][ri];
                double den = 0.0;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                if (fr0) {
                    const double wp = ws[rj][ri + 1], wm = ws[rj][ri - 1];
                    den += 2.0 * wc + wp + wm;
                    a0 = wc + wp;
                    a1 = wc + wm;
                }
                if (fr1) {
                    const double wp = ws[rj + 1][ri], wm = ws[rj - 1][ri];
                    den += 2.0 * wc + wp + wm;
                    a2 = wc + wp;
                    a3 = wc + wm;
                }
                if (den > 0.0) {
                    const double id = 1.0 / den;
                    cf[r][0] = a0 * id;
                    cf[r][1] = a1 * id;
                    cf[r][2] = a2 * id;
                    cf[r][3] = a3 * id;
                    fl[r] = (fr0 ? 1 : 0) | (fr1 ? 2 : 0);
                }
                fl[r] |= depth << 2;
            }
        }
    }
    int cur = 0;
    for (int sw = 1; sw <= sweeps; ++sw) {
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            const int q = tid + JNT * r;
            if (q < JRX * JRY) {
                const int ri = q % JRX, rj = q / JRX;
                double v0 = xs[cur][0][rj][ri], v1 = xs[cur][1][rj][ri];
                if ((fl[r] >> 2) >= sw) {
                    if (fl[r] & 1)
                        v0 = cf[r][0] * xs[cur][0][rj][ri + 1] + cf[r][1] * xs[cur][0][rj][ri - 1] +
                             cf[r][2] * xs[cur][0][rj + 1][ri] + cf[r][3] * xs[cur][0][rj - 1][ri];
                    if (fl[r] & 2)
                        v1 = cf[r][0] * xs[cur][1][rj][ri + 1] + cf[r][1] * xs[cur][1][rj][ri - 1] +
                             cf[r][2] * xs[cur][1][rj + 1][ri] + cf[r][3] * xs[cur][1][rj - 1][ri];
                }
                xs[cur ^ 1][0][rj][ri] = v0;
                xs[cur ^ 1][1][rj][ri] = v1;
            }
        }
        cur ^= 1;
        __syncthreads();
    }
    double best = 1.0;
    for (int q = tid; q < JTX * JTY; q += JNT) {
        const int oi = q % JTX, oj = q / JTX;
        const int gi = blockIdx.x * JTX + oi, gj = blockIdx.y * JTY + oj;
        if (gi < n0 && gj < n1) {
            const long long t = (long long)gj * n0 + gi;
            const double xm[2] = {xs[cur][0][oj + JS][oi + JS], xs[cur][1][oj + JS][oi + JS]};
            xout[t] = xm[0];
            xout[g.nodes + t] = xm[1];
            if (dtau_part != nullptr) {
                const int c[3] = {gi, gj, 0};
                best = fmin(best, dtau_bound<2>(g, x0, c, t, xm));
            }
        }
    }
    if (dtau_part != nullptr) {
        best = block_reduce<1>(best, sh);
        if (tid == 0) dtau_part[blockIdx.y * gridDim.x + blockIdx.x] = best;
    }
}

template <int DIM>
__global__ void __launch_bounds__(256) k_dtau_partial(GridDev g, const double* __restrict__ x,
                                                      const double* __restrict__ xm,
                                                      double* __restrict__ partial) {
    __shared__ double sh[8];
    double best = 1.0;
    int i, j, k;
    if (box_ijk_xcd(0, 0, 0, g.n[0], g.n[1], i, j, k)) {
        const int c[3] = {i, j, k};
        const long long t = iidx(g, i, j, k);
        double xv[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) xv[a] = xm[(long long)a * g.nodes + t];
        best = dtau_bound<DIM>(g, x, c, t, xv);
    }
    const double r = block_reduce<1>(best, sh);
    if (flat_tid() == 0) partial[flat_block()] = r;
}

// x^{n+1} = x + dtau (xm - x), xdot = dtau (xm - x) / dt.  With nb > 0 every
// block reduces the nb partial minima of the Delta tau bound itself (capped at
// 1) and block 0 stores the result in dtau; otherwise dtau holds it.
__global__ void __launch_bounds__(256) k_mesh_update(long long n, const double* __restrict__ x,
                                                     const double* __restrict__ xm, double* __restrict__ dtau,
                                                     const double* __restrict__ part, int nb,
                                                     const double* __restrict__ dt, double* __restrict__ xnew,
                                                     double* __restrict__ xdot) {
    __shared__ double sh[8];
    double a;
    if (nb > 0) {
        a = 1.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) a = fmin(a, part[b]);
        a = block_reduce<1>(a, sh);
        if (blockIdx.x == 0 && threadIdx.x == 0) dtau[0] = a;
    } else {
        a = dtau[0];
    }
    const long long t = gtid();
    if (t >= n) return;
    const double dx = xm[t] - x[t];
    xnew[t] = x[t] + a * dx;
    xdot[t] = a * dx / dt[0];
}

__global__ void k_zero_mesh_velocity(long long n, const double* __restrict__ x, double* __restrict__ xnew,
                                     double* __restrict__ xdot) {
    const long long t = gtid();
    if (t >= n) return;
    xnew[t] = x[t];
    xdot[t] = 0.0;
}

__global__ void k_mesh_advance(long long n, const double* __restrict__ x, const double* __restrict__ xdot,
                               const double* __restrict__ dt_dev, double* __restrict__ xnew) {
    const long long t = gtid();
    if (t >= n) return;
    xnew[t] = x[t] + dt_dev[0] * xdot[t];
}

// ---------------------------------------------------------------------------
// SSP-RK3 stage combinations (Shu-Osher form)
// ---------------------------------------------------------------------------
// out may alias U0 (last stage writes the new state in place), so no __restrict__.
// Threads [0, nU) combine Ucurv, threads [nU, nU + nJ) combine J.
// Shu-Osher SSP-RK3 stage combination of U (nU = m N values) and J (nJ = N) with
// the residual L = sum_k Ld_k summed from the direction slabs in direction order
// (slab k holds the m components followed by J, so U value t and J value t map
// to Ld index t and nU + t).
__global__ void k_rk_combine(long long nU, long long nJ, int dim, int stage, const double* U0,
                             const double* Us, const double* J0, const double* Js,
                             const double* __restrict__ Ld, const double* __restrict__ dt_dev,
                             double* outU, double* outJ, long long nX, const double* __restrict__ xsrc,
                             double* __restrict__ xdst) {
    long long t = gtid();
    if (t >= nU + nJ) {
        // threads beyond the state copy the new mesh (end of the step)
        t -= nU + nJ;
        if (t < nX) xdst[t] = xsrc[t];
        return;
    }
    const long long slab = nU + nJ;
    double l = Ld[t] + Ld[slab + t];
    if (dim == 3) l += Ld[2 * slab + t];
    const double* a = U0;
    const double* b = Us;
    double* o = outU;
    if (t >= nU) { t -= nU; a = J0; b = Js; o = outJ; }
    const double dt = dt_dev[0];
    if (stage == 0) o[t] = a[t] + dt * l;
    else if (stage == 1) o[t] = 0.75 * a[t] + 0.25 * (b[t] + dt * l);
    else o[t] = a[t] / 3.0 + 2.0 / 3.0 * (b[t] + dt * l);
}

// ---------------------------------------------------------------------------
// diagnostics (FP64 sums)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256) k_diag_partial(GridDev g, double G, const double* __restrict__ prim,
                                                      const double* __restrict__ U,
                                                      const double* __restrict__ J,
                                                      const double* __restrict__ dU,
                                                      const double* __restrict__ dJ,
                                                      double* __restrict__ partial) {
    constexpr int M = DIM + 2;
    constexpr int NQ = 3 + M;
    __shared__ double sh[8];
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const long long P = g.pnodes, N = g.nodes;
    int i, j, k;
    if (box_ijk(0, 0, 0, g.n[0], g.n[1], i, j, k)) {
        const long long t = iidx(g, i, j, k);
        const long long pi = pidx(g, i, j, k);
        const double rho = prim[pi], p = prim[(M - 1) * P + pi];
        const double lr = prim[M * P + pi], lb = prim[(M + 1) * P + pi];
        double u[DIM], uu = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) { u[c] = prim[(1 + c) * P + pi]; uu += u[c] * u[c]; }
        const double W = sqrt(1.0 + uu);
        const double beta = rho / p;
        double V[M];
        V[0] = G / (G - 1.0) + lr + lb / (G - 1.0) + beta;
#pragma unroll
        for (int c = 0; c < DIM; ++c) V[1 + c] = beta * u[c];
        V[M - 1] = -beta * W;
        const double phi = rho * W;
        double ep = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) ep += V[c] * dU[c * N + t];
        ep -= phi * dJ[t];
        const double s = log(p) - G * lr;
        const double eta = -rho * W * s / (G - 1.0);
        acc[0] = ep;
        acc[1] = J[t] * eta;
        acc[2] = J[t];
#pragma unroll
        for (int c = 0; c < M; ++c) acc[3 + c] = U[c * N + t];
    }
    const int nb = (int)(gridDim.x * gridDim.y * gridDim.z);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double r = block_reduce<2>(acc[q], sh);
        if (flat_tid() == 0) partial[q * nb + flat_block()] = r;
    }
}

__global__ void __launch_bounds__(256) k_diag_final(int nq, int nb, const double* __restrict__ partial,
                                                    double* __restrict__ out) {
    __shared__ double sh[8];
    for (int q = 0; q < nq; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[q * nb + b];
        s = block_reduce<2>(s, sh);
        if (threadIdx.x == 0) out[q] = s;
    }
}

inline dim3 interior_grid(const GridDev& g) { return box_grid(g.n[0], g.n[1], g.n[2]); }
inline int interior_blocks(const GridDev& g) {
    const dim3 b = interior_grid(g);
    return (int)(b.x * b.y * b.z);
}

}  // namespace

int reduction_blocks(const GridDev& g) { return interior_blocks(g); }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t s) {
    k_fill_u64<<<grid_for(n), TPB, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, long long n, hipStream_t s) {
    k_zero<<<grid_for(n), TPB, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, long long n, hipStream_t s) {
    k_copy<<<grid_for(n), TPB, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_prim2con(const es_ctx* c, const double* prim, const double* J, double* U,
                           hipStream_t s) {
    const double G = c->scheme.gamma;
    if (c->scheme.phys == ES_RMHD) return launch_prim2con_rmhd(c, prim, J, U, s);
    if (c->g.dim == 2) k_prim2con_rhd<2><<<grid_for(c->g.nodes), TPB, 0, s>>>(c->g, G, prim, J, U);
    else k_prim2con_rhd<3><<<grid_for(c->g.nodes), TPB, 0, s>>>(c->g, G, prim, J, U);
    return hipGetLastError();
}

static hipError_t con2prim_from(const es_ctx* c, const StateSrc& ss, double* prim, int use_guess,
                                hipStream_t s) {
    const double G = c->scheme.gamma;
    const GridDev& g = c->g;
    if (c->scheme.phys == ES_RMHD) return launch_con2prim_rmhd(c, &ss, prim, use_guess, s);
    const dim3 gr = box_grid(g.P[0], g.P[1], g.P[2]);
    if (g.dim == 2) k_con2prim_rhd<2><<<gr, box_block(), 0, s>>>(g, G, ss, prim, use_guess, c->fail);
    else k_con2prim_rhd<3><<<plane_grid(g.P[0], g.P[1], g.P[2]), TPB, 0, s>>>(g, G, ss, prim, use_guess, c->fail);
    return hipGetLastError();
}

hipError_t launch_con2prim(const es_ctx* c, const double* U, const double* J, double* prim,
                           int use_guess, hipStream_t s) {
    StateSrc ss{};
    ss.U = U;
    ss.J = J;
    ss.stage = -1;
    return con2prim_from(c, ss, prim, use_guess, s);
}

hipError_t launch_combine_con2prim(const es_ctx* c, int stage, const double* U0, const double* J0,
                                   const double* Us, const double* Js, const double* Ld,
                                   const double* dt_dev, double* Uout, double* Jout, double* prim,
                                   hipStream_t s) {
    StateSrc ss{};
    ss.stage = stage;
    ss.U0 = U0;
    ss.J0 = J0;
    ss.Us = Us;
    ss.Js = Js;
    ss.Ld = Ld;
    ss.dt = dt_dev;
    ss.Uout = Uout;
    ss.Jout = Jout;
    return con2prim_from(c, ss, prim, 1, s);
}

bool metrics_stages_batched(const es_ctx* c) { return c->g.dim == 2; }

// planes per block of the 3D metric tile kernel: one block per compute unit at a
// time (its LDS), so the runs of planes are cut to fill the 256 compute units once
// (128^3: 9 x 9 tiles x 3 runs of 45 planes), and are at least 2H + 1 planes long
static int metric_tile_planes(const GridDev& g) {
    const int tiles = ((g.P[0] + MT - 1) / MT) * ((g.P[1] + MT - 1) / MT);
    const int runs = tiles >= 256 ? 1 : 256 / tiles;
    const int kz = (g.P[2] + runs - 1) / runs;
    return kz < 2 * NG_MAX + 1 ? 2 * NG_MAX + 1 : kz;
}

hipError_t launch_metrics_stages(const es_ctx* c, const double* x, const double* xdot,
                                 const double* dt_dev, double* met0, double* met1, double* met2,
                                 hipStream_t s) {
    const GridDev& g = c->g;
    const dim3 gm((unsigned)((g.P[0] + MTX - 1) / MTX), (unsigned)((g.P[1] + MTY - 1) / MTY), 1);
    k_metrics2d_stages<<<gm, dim3(MTX, MSY, 1), 0, s>>>(g, x, xdot, dt_dev, met0, met1, met2);
    return hipGetLastError();
}

hipError_t launch_temporal_metrics3d(const es_ctx* c, const double* xdot, double* met, hipStream_t s) {
    const GridDev& g = c->g;
    k_temporal_metrics3d<<<plane_grid(g.P[0], g.P[1], g.P[2]), TPB, 0, s>>>(g, xdot, met);
    return hipGetLastError();
}

hipError_t launch_metrics(const es_ctx* c, const double* x, const double* xdot,
                          const double* dt_dev, double coef, double* met, double* J0,
                          hipStream_t s, bool ve_ready) {
    const GridDev& g = c->g;
    const dim3 ge = plane_grid(g.E[0], g.E[1], g.E[2]);
    double* ve = xdot != nullptr ? c->ve : nullptr;
    if (g.dim == 2) {
        (void)ve;
        const dim3 gm((unsigned)((g.P[0] + MTX - 1) / MTX), (unsigned)((g.P[1] + MTY - 1) / MTY), 1);
        k_metrics2d_fused<<<gm, dim3(MTX, MBY, 1), 0, s>>>(g, x, xdot, dt_dev, coef, met, J0);
    } else {
        if (J0 != nullptr) {
            // with the Jacobian J^0 (set-up, not a stage): extended mesh and products in HBM
            k_mesh_extend<3><<<ge, TPB, 0, s>>>(g, x, xdot, dt_dev, coef, c->xe, ve);
            k_cmm_products<<<ge, TPB, 0, s>>>(g, c->xe, c->pi);
            k_metrics3d<<<box_grid(g.P[0], g.P[1], g.P[2]), box_block(), 0, s>>>(g, c->xe, ve, c->pi, met, J0);
        } else {
            // the extended mesh velocity is left in c->ve by an earlier call with the same xdot
            k_mesh_extend<3><<<ge, TPB, 0, s>>>(g, x, xdot, dt_dev, coef, c->xe, ve_ready ? nullptr : ve);
            const int t0 = (g.P[0] + MT - 1) / MT, t1 = (g.P[1] + MT - 1) / MT;
            const int kz = metric_tile_planes(g);
            const unsigned nb = (unsigned)(t0 * t1 * ((g.P[2] + kz - 1) / kz));
            if (g.ng == 4) k_metrics3d_tile<4><<<nb, MT_THREADS, 0, s>>>(g, c->xe, ve, met, kz, t0, t1);
            else k_metrics3d_tile<3><<<nb, MT_THREADS, 0, s>>>(g, c->xe, ve, met, kz, t0, t1);
        }
    }
    return hipGetLastError();
}

template <int DIM, int PO>
static void residual_launch(bool es_, bool mixed, unsigned nb, hipStream_t s, const GridDev& g, double G,
                            double eps, const double* prim, const double* met, double* Ld, const SweepPlan& sw) {
    if (es_ && mixed) k_residual_rhd<DIM, true, true, PO><<<nb, 256, 0, s>>>(g, G, eps, prim, met, Ld, sw);
    else if (es_) k_residual_rhd<DIM, true, false, PO><<<nb, 256, 0, s>>>(g, G, eps, prim, met, Ld, sw);
    else if (mixed) k_residual_rhd<DIM, false, true, PO><<<nb, 256, 0, s>>>(g, G, eps, prim, met, Ld, sw);
    else k_residual_rhd<DIM, false, false, PO><<<nb, 256, 0, s>>>(g, G, eps, prim, met, Ld, sw);
}

template <int DIM>
static void residual_all(const es_ctx* c, const double* prim, const double* met, double* Ld,
                         hipStream_t s) {
    const GridDev& g = c->g;
    SweepPlan sw{};
    long long nb = 0;
    const int segn = seg_nodes(g.p);
    for (int d = 0; d < DIM; ++d) {
        long long nl = 1;
        for (int a = 0; a < DIM; ++a)
            if (a != d) nl *= g.n[a];
        // segments per sequence (the lines dealt to LINES sequences): flat, until the
        // one owning the longest sequence's last interior node; aligned, ceil(n / SEG)
        // per line.  One block per segment offset, one wavefront per sequence.
        const long long pl = g.n[d] + 2 * g.ng, ml = (nl + LINES - 1) / LINES;
        sw.flat[d] = seq_flat(g.n[d], (int)pl, segn, 0.875) ? 1 : 0;
        sw.nsl[d] = (g.n[d] + segn - 1) / segn;
        sw.nseg[d] = sw.flat[d] ? (int)(((ml - 1) * pl + g.n[d] - 1) / segn + 1) : (int)(ml * sw.nsl[d]);
        sw.nlines[d] = nl;
        sw.nblk[d] = sw.nseg[d];
        nb += sw.nblk[d];
    }
    const double G = c->scheme.gamma, eps = c->scheme.weno_eps;
    const bool es_ = c->scheme.dissipation != 0, mixed = c->scheme.mixed != 0;
    if (g.p == 2) residual_launch<DIM, 2>(es_, mixed, (unsigned)nb, s, g, G, eps, prim, met, Ld, sw);
    else if (g.p == 4) residual_launch<DIM, 4>(es_, mixed, (unsigned)nb, s, g, G, eps, prim, met, Ld, sw);
    else residual_launch<DIM, 3>(es_, mixed, (unsigned)nb, s, g, G, eps, prim, met, Ld, sw);
}

hipError_t launch_residual_dirs(const es_ctx* c, const double* prim, const double* met, double* Ld,
                                hipStream_t s) {
    if (c->scheme.phys == ES_RMHD) return launch_residual_dirs_rmhd(c, prim, met, Ld, s);
    if (c->g.dim == 2) residual_all<2>(c, prim, met, Ld, s);
    else residual_all<3>(c, prim, met, Ld, s);
    return hipGetLastError();
}

hipError_t launch_residual(const es_ctx* c, const double* prim, const double* met, double* dU,
                           double* dJ, hipStream_t s) {
    hipError_t e = launch_residual_dirs(c, prim, met, c->L, s);
    if (e != hipSuccess) return e;
    const long long n = c->g.nodes * (c->m + 1);
    k_sum_dirs<<<grid_for(n), TPB, 0, s>>>(c->g.nodes, c->m, c->g.dim, c->L, dU, dJ);
    return hipGetLastError();
}

// reduction partials in c->red: CFL maxima (dim slabs), monitor maxima, Delta tau
// minima, Laplacian maxima of the gradient + Laplacian monitor
inline double* red_cfl(const es_ctx* c) { return c->red; }
inline double* red_monitor(const es_ctx* c) { return c->red + 3 * (long long)c->red_blocks; }
inline double* red_dtau(const es_ctx* c) { return c->red + 4 * (long long)c->red_blocks; }
inline double* red_laplacian(const es_ctx* c) { return c->red + 5 * (long long)c->red_blocks; }

inline DtFinal cfl_final_args(const es_ctx* c, const double* fixed_dt_dev, double* dt_dev) {
    const GridDev& g = c->g;
    DtFinal f;
    f.partial = red_cfl(c);
    f.nb = interior_blocks(g);
    f.dim = g.dim;
    f.cfl = c->scheme.cfl;
    f.dx[0] = g.dxi[0];
    f.dx[1] = g.dxi[1];
    f.dx[2] = g.dxi[2];
    f.fixed_dt = fixed_dt_dev;
    f.dt_out = dt_dev;
    return f;
}

hipError_t launch_cfl_mesh(const es_ctx* c, const double* prim, const double* x, const double* J,
                           double* dt_dev, const double* fixed_dt_dev, hipStream_t s, bool defer_final,
                           bool with_monitor, bool* monitor_done) {
    const GridDev& g = c->g;
    if (monitor_done != nullptr) *monitor_done = false;
    if (c->scheme.phys == ES_RMHD || g.dim != 2) {
        if (fixed_dt_dev != nullptr) {
            // a prescribed dt: no speeds needed (finalised here or by the mesh launches)
            if (!defer_final) k_cfl_final<<<1, FINAL_TPB, 0, s>>>(cfl_final_args(c, fixed_dt_dev, dt_dev));
            return hipGetLastError();
        }
        const hipError_t e = launch_metrics(c, x, nullptr, nullptr, 0.0, c->met, nullptr, s);
        if (e != hipSuccess) return e;
        return launch_cfl(c, prim, c->met, J, dt_dev, fixed_dt_dev, s, defer_final);
    }
    MonitorArgs mon{};
    // the gradient + Laplacian monitor is formed by the mesh launches
    if (with_monitor && c->monitor.form != ES_MON_GRADLAP) {
        mon.enabled = 1;
        mon.M = c->m;
        mon.sigma_ln = c->monitor.sigma == ES_SIGMA_LNRHO;
        mon.sqgrad = c->monitor.form == ES_MON_SQGRAD;
        mon.alpha = c->monitor.alpha;
        mon.w = c->wa;
        mon.partial = red_monitor(c);
    }
    k_cfl_partial2d_mesh<<<interior_grid(g), dim3(MTX, CBY, 1), 0, s>>>(g, c->scheme.gamma, prim, x, J, red_cfl(c),
                                                                         mon);
    if (!defer_final) k_cfl_final<<<1, FINAL_TPB, 0, s>>>(cfl_final_args(c, fixed_dt_dev, dt_dev));
    if (monitor_done != nullptr) *monitor_done = mon.enabled != 0;
    return hipGetLastError();
}

hipError_t launch_cfl(const es_ctx* c, const double* prim, const double* met, const double* J,
                      double* dt_dev, const double* fixed_dt_dev, hipStream_t s, bool defer_final) {
    const GridDev& g = c->g;
    const double G = c->scheme.gamma;
    if (c->scheme.phys == ES_RMHD) {
        const hipError_t e = launch_cfl_partial_rmhd(c, prim, met, J, s);
        if (e != hipSuccess) return e;
    } else if (g.dim == 2) {
        k_cfl_partial<2><<<interior_grid(g), box_block(), 0, s>>>(g, G, prim, met, J, red_cfl(c));
    } else {
        k_cfl_partial<3><<<interior_grid(g), box_block(), 0, s>>>(g, G, prim, met, J, red_cfl(c));
    }
    if (!defer_final) k_cfl_final<<<1, FINAL_TPB, 0, s>>>(cfl_final_args(c, fixed_dt_dev, dt_dev));
    return hipGetLastError();
}

hipError_t launch_zero_mesh_velocity(const es_ctx* c, const double* x, double* x_new, double* xdot,
                                     hipStream_t s) {
    const long long n = c->g.nodes * c->g.dim;
    k_zero_mesh_velocity<<<grid_for(n), TPB, 0, s>>>(n, x, x_new, xdot);
    return hipGetLastError();
}

hipError_t launch_mesh_advance(const es_ctx* c, const double* x, const double* xdot,
                               const double* dt_dev, double* x_new, hipStream_t s) {
    const long long n = c->g.nodes * c->g.dim;
    k_mesh_advance<<<grid_for(n), TPB, 0, s>>>(n, x, xdot, dt_dev, x_new);
    return hipGetLastError();
}

hipError_t launch_mesh(const es_ctx* c, const double* prim, const double* x, const double* dt_dev,
                       double* x_new, double* xdot, double* dtau_dev, hipStream_t s, bool dt_pending,
                       const double* fixed_dt_dev, bool grad_done) {
    const GridDev& g = c->g;
    const es_monitor& mo = c->monitor;
    const int nb = interior_blocks(g);
    const dim3 gr = interior_grid(g);
    const int sig_ln = mo.sigma == ES_SIGMA_LNRHO;
    const int sq = mo.form == ES_MON_SQGRAD;
    const bool gradlap = mo.form == ES_MON_GRADLAP;
    double* w = c->wa;
    double* w2 = c->wb;
    double* gpart = red_monitor(c);
    // 2D: the first filter launch finalises a pending dt (block 0); 3D: a launch of its own
    // (dt_dev is written only when dt is pending: the step's own buffer)
    DtFinal dt_fin = cfl_final_args(c, fixed_dt_dev, dt_pending ? const_cast<double*>(dt_dev) : nullptr);
    if (dt_pending && g.dim != 2) k_cfl_final<<<1, FINAL_TPB, 0, s>>>(dt_fin);
    if (grad_done) {
        // omega (or |grad sigma|) in c->wa and its block maxima came with the CFL launch
    } else if (gradlap) {
        // omega formed here; the filter passes below take it as it is
        if (g.dim == 2)
            k_monitor_gradlap<2><<<gr, box_block(), 0, s>>>(g, c->m, sig_ln, prim, w, w2, gpart, red_laplacian(c));
        else
            k_monitor_gradlap<3><<<gr, box_block(), 0, s>>>(g, c->m, sig_ln, prim, w, w2, gpart, red_laplacian(c));
        k_reduce_final<<<1, FINAL_TPB, 0, s>>>(0, nb, gpart, c->scal + SCAL_GMAX);
        k_reduce_final<<<1, FINAL_TPB, 0, s>>>(0, nb, red_laplacian(c), c->scal + SCAL_LMAX);
        k_monitor_apply_gradlap<<<grid_for(g.nodes), TPB, 0, s>>>(g.nodes, mo.alpha, mo.alpha2, c->scal + SCAL_GMAX,
                                                                   c->scal + SCAL_LMAX, w, w2);
    } else if (g.dim == 2) {
        k_monitor_grad<2><<<gr, box_block(), 0, s>>>(g, c->m, sig_ln, sq, mo.alpha, prim, w, gpart);
    } else {
        k_monitor_grad<3><<<gr, box_block(), 0, s>>>(g, c->m, sig_ln, sq, mo.alpha, prim, w, gpart);
    }
    if (g.dim == 2) {
        // normalisation (maximum reduced in each block) and filter passes, FH per launch
        int apply = !sq && !gradlap, left = mo.filter_passes;
        do {
            const int k = min(FH, left);
            k_monitor_filter2d<<<box_grid(g.n[0], g.n[1], 1), dim3(FTX, FBY, 1), 0, s>>>(
                g, apply, mo.alpha, gpart, nb, k, w, w2, dt_fin);
            double* tmp = w; w = w2; w2 = tmp;
            apply = 0;
            dt_fin.dt_out = nullptr;
            left -= k;
        } while (left > 0);
    } else {
        if (!sq && !gradlap) {
            k_reduce_final<<<1, FINAL_TPB, 0, s>>>(0, nb, gpart, c->scal + SCAL_GMAX);
            k_monitor_apply<<<grid_for(g.nodes), TPB, 0, s>>>(g.nodes, mo.alpha, c->scal + SCAL_GMAX, w);
        }
        for (int f = 0; f < mo.filter_passes; ++f) {
            k_filter<3><<<gr, box_block(), 0, s>>>(g, w, w2);
            double* tmp = w; w = w2; w2 = tmp;
        }
    }
    const double* xin = x;
    double* xo = c->xa;
    double* xalt = c->xb;
    double* dtau = dtau_dev != nullptr ? dtau_dev : c->scal + SCAL_DTAU;
    const long long n = g.nodes * g.dim;
    int nbt = 0;   // Delta tau partials left for k_mesh_update to reduce
    if (g.dim == 2 && mo.sweeps > 0) {
        // the last multi-sweep launch also forms the Delta tau block minima
        const dim3 gj((unsigned)((g.n[0] + JTX - 1) / JTX), (unsigned)((g.n[1] + JTY - 1) / JTY), 1);
        for (int done = 0; done < mo.sweeps; done += JS) {
            const int k = min(JS, mo.sweeps - done);
            const bool last = done + k >= mo.sweeps;
            k_jacobi_multi2d<<<gj, JNT, 0, s>>>(g, k, w, xin, xo, x, last ? red_dtau(c) : nullptr);
            xin = xo;
            double* tmp = xo; xo = xalt; xalt = tmp;
        }
        nbt = (int)(gj.x * gj.y);
    } else {
        for (int it = 0; it < mo.sweeps; ++it) {
            if (g.dim == 2) k_jacobi<2><<<gr, box_block(), 0, s>>>(g, w, xin, xo);
            else k_jacobi<3><<<gr, box_block(), 0, s>>>(g, w, xin, xo);
            xin = xo;
            double* tmp = xo; xo = xalt; xalt = tmp;
        }
        if (g.dim == 2) k_dtau_partial<2><<<gr, box_block(), 0, s>>>(g, x, xin, red_dtau(c));
        else k_dtau_partial<3><<<gr, box_block(), 0, s>>>(g, x, xin, red_dtau(c));
        k_reduce_final<<<1, FINAL_TPB, 0, s>>>(1, nb, red_dtau(c), dtau);
    }
    k_mesh_update<<<grid_for(n), TPB, 0, s>>>(n, x, xin, dtau, red_dtau(c), nbt, dt_dev, x_new, xdot);
    return hipGetLastError();
}

hipError_t launch_rk_combine(const es_ctx* c, int stage, const double* U0, const double* J0,
                             double* Us, double* Js, const double* Ld, const double* dt_dev,
                             hipStream_t s, const double* xsrc, double* xdst) {
    const long long nU = c->g.nodes * c->m;
    const long long nJ = c->g.nodes;
    const long long nX = xsrc != nullptr ? c->g.nodes * c->g.dim : 0;
    // stage 2 writes the new state over U0/J0 (the caller passes them as outputs)
    double* outU = stage == 2 ? const_cast<double*>(U0) : Us;
    double* outJ = stage == 2 ? const_cast<double*>(J0) : Js;
    k_rk_combine<<<grid_for(nU + nJ + nX), TPB, 0, s>>>(nU, nJ, c->g.dim, stage, U0, Us, J0, Js, Ld, dt_dev,
                                                        outU, outJ, nX, xsrc, xdst);
    return hipGetLastError();
}

hipError_t launch_diagnostics(const es_ctx* c, const double* prim, const double* U,
                              const double* J, const double* dU, const double* dJ, double* out,
                              hipStream_t s) {
    const GridDev& g = c->g;
    const int nb = interior_blocks(g);
    const double G = c->scheme.gamma;
    if (c->scheme.phys == ES_RMHD) {
        const hipError_t e = launch_diag_partial_rmhd(c, prim, U, J, dU, dJ, s);
        if (e != hipSuccess) return e;
    } else if (g.dim == 2) {
        k_diag_partial<2><<<interior_grid(g), box_block(), 0, s>>>(g, G, prim, U, J, dU, dJ, c->red);
    } else {
        k_diag_partial<3><<<interior_grid(g), box_block(), 0, s>>>(g, G, prim, U, J, dU, dJ, c->red);
    }
    k_diag_final<<<1, 256, 0, s>>>(3 + c->m, nb, c->red, out);
    return hipGetLastError();
}

}  // namespace es
