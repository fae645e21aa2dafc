// Host-side context and kernel launchers of libes.so.
#pragma once

#include <hip/hip_runtime.h>

#include "es.h"
#include "es_common.h"

struct es_ctx {
    es_grid grid;
    es_scheme scheme;
    es_monitor monitor;
    es::GridDev g;
    int m;          // conserved variables
    int nprim;      // padded primitive comps (m + 2)
    int nmet;       // metric comps d(d+1)
    int device;
    // workspace (device)
    double* prim;   // padded, nprim comps
    double* met;    // padded, nmet comps
    double* met1;   // padded, nmet comps (stage-1 metrics, 2D)
    double* met2;   // padded, nmet comps (stage-2 metrics)
    double* L;      // interior, d slabs of m + 1 comps (stage residual by direction, J last)
    double* Us;     // interior, m comps (stage-1 state)
    double* Js;     // interior
    double* Us2;    // interior, m comps (stage-2 state)
    double* Js2;    // interior
    double* xnew;   // interior, d comps
    double* xa;     // interior, d comps (Jacobi ping)
    double* xb;     // interior, d comps (Jacobi pong)
    double* wa;     // interior (monitor ping)
    double* wb;     // interior (monitor pong)
    double* xe;     // stage mesh on the extension box (d comps)
    double* ve;     // mesh velocity on the extension box (d comps)
    double* pi;     // 3D: conservative-metric products on the extension box (9 comps; the
                    // metrics with J^0)
    double* red;    // reduction partials
    double* scal;   // device scalars: [0] dt, [1] gmax, [2] dtau, [3..] spare
    unsigned long long* fail;   // [0] count inadmissible, [1] count no-convergence, [2] first index
    int red_blocks;
    // adjoint workspace (allocated by the first adjoint call)
    double* adj_lamU;   // interior, m comps: cotangent of the current stage state
    double* adj_lamJ;   // interior
    double* adj_lamL;   // interior, m comps: cotangent of the stage residual
    double* adj_accU;   // interior, m comps: accumulated cotangent of U^n
    double* adj_accJ;   // interior
    double* adj_gU;     // interior, m comps: stage residual VJP
    double* adj_gJ;     // interior
    double* gdir;       // padded, d slabs of m comps: primitive cotangents by direction
    double* adj_eig;    // RMHD ES: face eigen-structure held by the residual VJP (face_eig_doubles_rmhd)
    // HIP graph of one es_rk3_step (replayed while the argument pointers stay the same)
    int use_graph;
    hipStream_t cap;            // capture stream (default priority)
    hipGraphExec_t gexec;
    const void* gkey[7];
};

namespace es {

constexpr int SCAL_DT = 0;
constexpr int SCAL_GMAX = 1;
constexpr int SCAL_DTAU = 2;
constexpr int SCAL_LMAX = 3;
constexpr int NSCAL = 8;

hipError_t launch_prim2con(const es_ctx* c, const double* prim, const double* J, double* U,
                           hipStream_t s);
hipError_t launch_con2prim(const es_ctx* c, const double* U, const double* J, double* prim,
                           int use_guess, hipStream_t s);
int reduction_blocks(const GridDev& g);
hipError_t launch_temporal_metrics3d(const es_ctx* c, const double* xdot, double* met, hipStream_t s);
// ve_ready: the extended mesh velocity of this xdot is already in the context
// (3D; an earlier call of the same step), so it is not formed again
hipError_t launch_metrics(const es_ctx* c, const double* x, const double* xdot,
                          const double* dt_dev, double coef, double* met, double* J0,
                          hipStream_t s, bool ve_ready = false);
// the metrics of the three stage meshes x + c dt xdot (c = 0, 1, 1/2) in one launch
bool metrics_stages_batched(const es_ctx* c);
hipError_t launch_metrics_stages(const es_ctx* c, const double* x, const double* xdot,
                                 const double* dt_dev, double* met0, double* met1, double* met2,
                                 hipStream_t s);
// residual by direction: slab k of Ld (dim slabs of m + 1 components) holds direction k's part
hipError_t launch_residual_dirs(const es_ctx* c, const double* prim, const double* met, double* Ld,
                                hipStream_t s);
// dU, dJ = sum over directions (through the context's slabs)
hipError_t launch_residual(const es_ctx* c, const double* prim, const double* met, double* dU,
                           double* dJ, hipStream_t s);
// defer_final: only the per-block CFL maxima are formed; launch_mesh with
// dt_pending finalises dt before its first use.
hipError_t launch_cfl(const es_ctx* c, const double* prim, const double* met, const double* J,
                      double* dt_dev, const double* fixed_dt_dev, hipStream_t s, bool defer_final = false);
// CFL step from the mesh x (spatial metrics formed on the fly; c->met is used as
// workspace where they are not).  with_monitor: the launch may also form the
// monitor gradient for launch_mesh; *monitor_done tells whether it did.
hipError_t launch_cfl_mesh(const es_ctx* c, const double* prim, const double* x, const double* J,
                           double* dt_dev, const double* fixed_dt_dev, hipStream_t s, bool defer_final,
                           bool with_monitor, bool* monitor_done);
hipError_t launch_mesh(const es_ctx* c, const double* prim, const double* x, const double* dt_dev,
                       double* x_new, double* xdot, double* dtau_dev, hipStream_t s,
                       bool dt_pending = false, const double* fixed_dt_dev = nullptr,
                       bool grad_done = false);
hipError_t launch_mesh_advance(const es_ctx* c, const double* x, const double* xdot,
                               const double* dt_dev, double* x_new, hipStream_t s);
hipError_t launch_zero_mesh_velocity(const es_ctx* c, const double* x, double* x_new, double* xdot,
                                     hipStream_t s);
// xsrc/xdst (optional): copy the new mesh in the same launch (last stage)
hipError_t launch_rk_combine(const es_ctx* c, int stage, const double* U0, const double* J0,
                             double* Us, double* Js, const double* Ld, const double* dt_dev,
                             hipStream_t s, const double* xsrc = nullptr, double* xdst = nullptr);
// stage 0 or 1 combination formed inside con2prim: (Uout, Jout) = combined state,
// prim = con2prim of it (previous stage's pressure as the Newton guess)
hipError_t launch_combine_con2prim(const es_ctx* c, int stage, const double* U0, const double* J0,
                                   const double* Us, const double* Js, const double* Ld,
                                   const double* dt_dev, double* Uout, double* Jout, double* prim,
                                   hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, long long n, hipStream_t s);
hipError_t launch_diagnostics(const es_ctx* c, const double* prim, const double* U,
                              const double* J, const double* dU, const double* dJ, double* out,
                              hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t s);

// RMHD kernels (es_kernels_rmhd.hip), dispatched from the launchers above
hipError_t launch_prim2con_rmhd(const es_ctx* c, const double* prim, const double* J, double* U,
                                hipStream_t s);
// state_src: the StateSrc of the launcher (declared with the kernels)
hipError_t launch_con2prim_rmhd(const es_ctx* c, const void* state_src, double* prim, int use_guess,
                                hipStream_t s);
hipError_t launch_residual_dirs_rmhd(const es_ctx* c, const double* prim, const double* met, double* Ld,
                                     hipStream_t s);
// residual VJP of the RMHD system on c->prim (con2prim done by the caller), with
// the ghost folding and the con2prim pull-back into (gU, gJ)
size_t face_eig_doubles_rmhd(const es_ctx* c);
hipError_t launch_residual_fold_vjp_rmhd(const es_ctx* c, const double* U, const double* J, const double* met,
                                         const double* lam, double* gU, double* gJ, hipStream_t s);
hipError_t launch_cfl_partial_rmhd(const es_ctx* c, const double* prim, const double* met,
                                   const double* J, hipStream_t s);
hipError_t launch_diag_partial_rmhd(const es_ctx* c, const double* prim, const double* U, const double* J,
                                    const double* dU, const double* dJ, hipStream_t s);

// Checkpoint of one RK3 step for the adjoint (one caller buffer of
// checkpoint_doubles() doubles): stage states U^(0..2) (m comps each), J^(0..2),
// the mesh x^n and its velocity (d comps each) and the time step.
struct Checkpoint {
    const double* U[3];
    const double* J[3];
    const double* x;
    const double* xdot;
    const double* dt;
};
inline long long checkpoint_doubles(const es_ctx* c) {
    const long long N = c->g.nodes;
    return 3 * (long long)(c->m + 1) * N + 2LL * c->g.dim * N + 1;
}
inline Checkpoint checkpoint_layout(const es_ctx* c, const double* base) {
    const long long N = c->g.nodes;
    Checkpoint k;
    for (int s = 0; s < 3; ++s) k.U[s] = base + (long long)s * c->m * N;
    const double* j0 = base + 3LL * c->m * N;
    for (int s = 0; s < 3; ++s) k.J[s] = j0 + (long long)s * N;
    k.x = j0 + 3 * N;
    k.xdot = k.x + (long long)c->g.dim * N;
    k.dt = k.xdot + (long long)c->g.dim * N;
    return k;
}
// VJP of L(U, J) = residual(con2prim(U, J), met) (state part): gU, gJ = (dL/d(U, J))^T lam
hipError_t launch_state_residual_vjp(const es_ctx* c, const double* U, const double* J,
                                     const double* met, const double* lam, double* gU, double* gJ,
                                     hipStream_t s);
// VJP of one RK3 step with the mesh trajectory and the time step held fixed
hipError_t launch_rk3_vjp(const es_ctx* c, const double* ckpt, const double* lamU_in,
                          const double* lamJ_in, double* gU_out, double* gJ_out, hipStream_t s);
// con2prim VJP at the interior nodes (con2prim of (U, J) into c->prim first):
// gU = (dU/dP)^{-T} gprim / J, gJ = -(that . Ucurv) / J^2
hipError_t launch_con2prim_vjp(const es_ctx* c, const double* U, const double* J, const double* gprim,
                               double* gU, double* gJ, hipStream_t s);
hipError_t launch_con2prim_vjp_rmhd(const es_ctx* c, const double* U, const double* J, const double* gprim,
                                    double* gU, double* gJ, hipStream_t s);
// prim2con VJP: gprim = J (dU/dP)^T gUc, gJ = U(P) . gUc (gJ may be null)
hipError_t launch_prim2con_vjp(const es_ctx* c, const double* prim, const double* J, const double* gUc,
                               double* gprim, double* gJ, hipStream_t s);
hipError_t launch_prim2con_vjp_rmhd(const es_ctx* c, const double* prim, const double* J, const double* gUc,
                                    double* gprim, double* gJ, hipStream_t s);
hipError_t launch_zero(double* p, long long n, hipStream_t s);

}  // namespace es
