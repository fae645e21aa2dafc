// Launch-shape helpers shared by the kernel files: 256-thread 1D grids and
// 64 x 4 box grids over an index box (no integer division in the index map).
#pragma once

#include "es_common.h"
#include "es_seq.h"

namespace es {
namespace {

constexpr int TPB = 256;
constexpr int BX = 64, BY = 4;

inline unsigned grid_for(long long n, int tpb = TPB) {
    return (unsigned)((n + tpb - 1) / tpb);
}

inline dim3 box_grid(int e0, int e1, int e2) {
    return dim3((unsigned)((e0 + BX - 1) / BX), (unsigned)((e1 + BY - 1) / BY), (unsigned)e2);
}

inline dim3 box_block() { return dim3(BX, BY, 1); }

__device__ __forceinline__ long long gtid() {
    return (long long)blockIdx.x * blockDim.x + threadIdx.x;
}

// (i, j, k) of this thread in the box [lo, lo + e); false outside
__device__ __forceinline__ bool box_ijk(int lo0, int lo1, int lo2, int e0, int e1, int& i, int& j,
                                        int& k) {
    i = lo0 + (int)(blockIdx.x * BX + threadIdx.x);
    j = lo1 + (int)(blockIdx.y * BY + threadIdx.y);
    k = lo2 + (int)blockIdx.z;
    return i < lo0 + e0 && j < lo1 + e1;
}

__device__ __forceinline__ int flat_block() {
    return (int)((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
}

__device__ __forceinline__ int flat_tid() { return (int)(threadIdx.y * blockDim.x + threadIdx.x); }

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8), each
// with its own L2.  The logical block index gives every XCD one contiguous range
// of logical blocks, so neighbouring lines, whose halos and cache lines overlap,
// are read through the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, k = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + k;
}

// box_ijk with the blocks of a (BX, BY, 1) x (gx, gy, gz) launch renumbered so that
// each XCD owns one contiguous range of (x fastest, then y, then z) blocks: stencils
// that reach across neighbouring z planes then read them through the same L2.
__device__ __forceinline__ bool box_ijk_xcd(int lo0, int lo1, int lo2, int e0, int e1, int& i, int& j,
                                            int& k) {
    const int gx = (int)gridDim.x, gy = (int)gridDim.y;
    const int nb = gx * gy * (int)gridDim.z;
    const int b = (int)((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
    const int lb = xcd_block(b, nb);
    const int bx = lb % gx, by = (lb / gx) % gy, bz = lb / (gx * gy);
    i = lo0 + bx * BX + (int)threadIdx.x;
    j = lo1 + by * BY + (int)threadIdx.y;
    k = lo2 + bz;
    return i < lo0 + e0 && j < lo1 + e1;
}


// Block reductions of one double over the whole block (wavefronts of 64).
// Flattened cells (c0, c1) of a w0 x w1 plane, c0 fastest: TPB consecutive cells
// per block (rows wrap inside a block, so no lane idles at a row end and a
// wave's stores to one component are one contiguous run); blockIdx.y numbers
// the planes (or runs of planes), and the logical blocks are taken in
// XCD-contiguous ranges.  Launch with plane_grid() and TPB threads.
__device__ __forceinline__ bool plane_cell_xcd(int w0, int w1, int& c0, int& c1, int& plane) {
    const int gx = (int)gridDim.x;
    const int nb = gx * (int)gridDim.y;
    const int lb = xcd_block((int)(blockIdx.y * gridDim.x + blockIdx.x), nb);
    const int cell = (lb % gx) * TPB + (int)threadIdx.x;
    plane = lb / gx;
    if (cell >= w0 * w1) return false;
    c0 = cell % w0;
    c1 = cell / w0;
    return true;
}

inline dim3 plane_grid(int w0, int w1, int planes) {
    return dim3(grid_for((long long)w0 * w1), (unsigned)planes, 1);
}

template <int OP>   // 0 max, 1 min, 2 sum
__device__ __forceinline__ double block_reduce(double v, double* sh) {
    v = OP == 0 ? wave_max(v) : (OP == 1 ? wave_min(v) : wave_sum(v));
    const int tid = flat_tid();
    const int w = tid >> 6;
    if ((tid & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    const int nw = (int)(blockDim.x * blockDim.y) >> 6;
    for (int q = 1; q < nw; ++q) r = OP == 0 ? fmax(r, sh[q]) : (OP == 1 ? fmin(r, sh[q]) : r + sh[q]);
    __syncthreads();
    return r;
}

// Conservative state read by con2prim: (U, J) directly (stage < 0), or the
// Shu-Osher combination of Runge-Kutta stage 0 or 1 formed on the fly from U0,
// the previous stage state Us (stage 1) and the residual L = sum_k Ld_k (slab k
// holds m components then J), in the order of the stage-combination kernel; the
// interior nodes also store the combined state in (Uout, Jout).
struct StateSrc {
    const double* U;
    const double* J;
    int stage;
    const double* U0;
    const double* J0;
    const double* Us;
    const double* Js;
    const double* Ld;
    const double* dt;
    double* Uout;
    double* Jout;
};

__device__ __forceinline__ double rk_stage_value(int stage, double a, double b, double l, double dt) {
    if (stage == 0) return a + dt * l;
    if (stage == 1) return 0.75 * a + 0.25 * (b + dt * l);
    return a / 3.0 + 2.0 / 3.0 * (b + dt * l);
}

// Component c (0..m-1: U, m: J) of the state at interior node t.
__device__ __forceinline__ double state_value(const StateSrc& s, int dim, int m, long long N, int c,
                                              long long t) {
    if (s.stage < 0) return c < m ? s.U[c * N + t] : s.J[t];
    const long long slab = (long long)(m + 1) * N;
    const long long q = (long long)c * N + t;
    double l = s.Ld[q] + s.Ld[slab + q];
    if (dim == 3) l += s.Ld[2 * slab + q];
    const double a = c < m ? s.U0[q] : s.J0[t];
    const double b = s.stage == 0 ? 0.0 : (c < m ? s.Us[q] : s.Js[t]);
    return rk_stage_value(s.stage, a, b, l, s.dt[0]);
}

}  // namespace
}  // namespace es
