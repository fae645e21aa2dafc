// Device-side grid description, index maps and boundary rules shared by all
// kernels of libes.so.  Layouts are those documented in include/es.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "es.h"

namespace es {

// Ghost layers of the padded box: the 2p-th order stencils reach p nodes past an
// edge (the EC pairs (i, i+n), n <= p; the metrics' central differences; WENO of
// order 2p - 1 on nodes i-p+1..i+p), so ng = 3 for p = 2 and p = 3 (one layout)
// and ng = 4 for p = 4.  NG_MAX sizes the fixed-size staging arrays.
constexpr int NG = 3;
constexpr int NG_MAX = 4;
constexpr int RED_BLOCK = 256;   // threads per block of the reduction kernels

__device__ __host__ constexpr int ghost_layers(int p) { return p > NG ? p : NG; }

// Line segments of the residual kernels (one wavefront each): ng = ghost_layers(p)
// halo nodes on each side of 64 - ng owned nodes (61 for p <= 3, 60 for p = 4), so
// that every owned node's stencil lies within the 64 + ng loaded slots.
__host__ __device__ constexpr int seg_nodes(int po) { return 64 - ghost_layers(po); }
__host__ __device__ constexpr int seg_loads(int po) { return seg_nodes(po) + 2 * ghost_layers(po); }

// 2p-th order coefficients alpha_{3,n} of eq. HOCoeff: (3/2, -3/10, 1/30).
__device__ __host__ constexpr double alpha3(int n) {
    return n == 1 ? 1.5 : (n == 2 ? -0.3 : (n == 3 ? 1.0 / 30.0 : 0.0));
}

// alpha_{p,n} of eq. HOCoeff for p = 2 (4/3, -1/6), p = 3 and p = 4 (8/5, -2/5, 8/105,
// -1/140), zero for n > p.
__device__ __host__ constexpr double alpha_pn(int p, int n) {
    return p == 2   ? (n == 1 ? 4.0 / 3.0 : (n == 2 ? -1.0 / 6.0 : 0.0))
           : p == 4 ? (n == 1 ? 1.6 : (n == 2 ? -0.4 : (n == 3 ? 8.0 / 105.0 : (n == 4 ? -1.0 / 140.0 : 0.0))))
                    : alpha3(n);
}

struct GridDev {
    int dim;
    int n[3];
    int bc[3];
    double dxi[3];
    double period[3];
    int P[3];               // padded extents (n + 2 ng, or 1 for the unused 3rd axis in 2D)
    int g2;                 // ghost offset of the third axis (ng in 3D, 0 in 2D)
    int E[3];               // mesh-extension box extents (n + 4 ng, or 1)
    int g6;                 // extension offset of the third axis (2 ng in 3D, 0 in 2D)
    long long nodes;        // interior nodes
    long long pnodes;       // padded nodes
    long long enodes;       // mesh-extension box nodes
    int p;                  // order parameter: 2p-th order EC flux and metrics (2, 3 or 4)
    int ng;                 // ghost layers, ghost_layers(p)
};

__device__ __forceinline__ long long pidx(const GridDev& g, int i, int j, int k) {
    return ((long long)(k + g.g2) * g.P[1] + (j + g.ng)) * g.P[0] + (i + g.ng);
}

__device__ __forceinline__ long long iidx(const GridDev& g, int i, int j, int k) {
    return ((long long)k * g.n[1] + j) * g.n[0] + i;
}

__device__ __forceinline__ int floordiv(int a, int n) {
    return (a >= 0) ? a / n : -((-a + n - 1) / n);
}

// Solution boundary rule: periodic wrap or zero-gradient copy (outflow).
__device__ __forceinline__ int map_sol(int i, int n, int bc) {
    if (bc == ES_BC_PERIODIC) {
        int q = floordiv(i, n);
        return i - q * n;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Mesh extension along one axis: periodic copy (with a count of wraps for the
// coordinate shift) or odd reflection x_{-a} = 2 x_0 - x_a, x_{n-1+a} = 2 x_{n-1} - x_{n-1-a}.
struct AxisTerms {
    int idx[2];
    double w[2];
    int nt;
    int wraps;
};

__device__ __forceinline__ AxisTerms axis_terms(int i, int n, int bc) {
    AxisTerms t;
    t.wraps = 0;
    if (bc == ES_BC_PERIODIC) {
        int q = floordiv(i, n);
        t.idx[0] = i - q * n; t.w[0] = 1.0; t.nt = 1; t.wraps = q;
        t.idx[1] = 0; t.w[1] = 0.0;
    } else if (i < 0) {
        t.idx[0] = 0; t.w[0] = 2.0; t.idx[1] = -i; t.w[1] = -1.0; t.nt = 2;
    } else if (i >= n) {
        t.idx[0] = n - 1; t.w[0] = 2.0; t.idx[1] = 2 * (n - 1) - i; t.w[1] = -1.0; t.nt = 2;
    } else {
        t.idx[0] = i; t.w[0] = 1.0; t.nt = 1; t.idx[1] = 0; t.w[1] = 0.0;
    }
    return t;
}

// Value of component c of the (stage) mesh x + cdt * xd at index (i, j, k),
// which may lie up to 2 ng outside the interior box.  With shift = false the
// periodic coordinate shift is omitted (mesh velocity).
__device__ __forceinline__ double mesh_value(const GridDev& g, const double* __restrict__ x,
                                             const double* __restrict__ xd, double cdt, int c,
                                             int i, int j, int k, bool shift) {
    if (i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && (g.dim == 2 || (k >= 0 && k < g.n[2]))) {
        const long long nd = (long long)c * g.nodes + iidx(g, i, j, g.dim == 2 ? 0 : k);
        double xv = x[nd];
        if (xd != nullptr) xv += cdt * xd[nd];
        return xv;
    }
    AxisTerms a = axis_terms(i, g.n[0], g.bc[0]);
    AxisTerms b = axis_terms(j, g.n[1], g.bc[1]);
    AxisTerms e;
    if (g.dim == 3) {
        e = axis_terms(k, g.n[2], g.bc[2]);
    } else {
        e.idx[0] = 0; e.w[0] = 1.0; e.nt = 1; e.wraps = 0; e.idx[1] = 0; e.w[1] = 0.0;
    }
    const long long off = (long long)c * g.nodes;
    double v = 0.0;
    // fully unrolled over the (at most) two terms per axis so the term arrays
    // stay in registers
#pragma unroll
    for (int te = 0; te < 2; ++te) {
        if (te >= e.nt) break;
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
            if (tb >= b.nt) break;
#pragma unroll
            for (int ta = 0; ta < 2; ++ta) {
                if (ta >= a.nt) break;
                const double w = a.w[ta] * b.w[tb] * e.w[te];
                const long long nd = off + iidx(g, a.idx[ta], b.idx[tb], e.idx[te]);
                double xv = x[nd];
                if (xd != nullptr) xv += cdt * xd[nd];
                v += w * xv;
            }
        }
    }
    if (shift) {
        const int wr = (c == 0) ? a.wraps : (c == 1 ? b.wraps : e.wraps);
        v += wr * g.period[c];
    }
    return v;
}

// Failure record of the conservative-to-primitive recovery (device array of 4
// unsigned 64-bit counters): [0] inadmissible states, [1] iterations that did not
// converge, [2] smallest failing interior node index, [3] nodes whose evolved
// Jacobian is not positive (a tangled mesh).  Codes: 1 inadmissible, 2 no
// convergence, FAIL_MESH non-positive Jacobian.
constexpr int FAIL_MESH = 3;
__device__ __forceinline__ void record_failure(unsigned long long* fail, int st, long long node) {
    atomicAdd(&fail[st == 1 ? 0 : (st == FAIL_MESH ? 3 : 1)], 1ull);
    atomicMin(&fail[2], (unsigned long long)node);
}

// Exact max/min reductions of non-negative doubles: order independent.
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace es
