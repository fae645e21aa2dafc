/*
 * es.h -- C ABI of libes.so: the entropy-stable adaptive moving-mesh finite
 * difference residual of Duan & Tang, "High-order accurate entropy stable
 * adaptive moving mesh finite difference schemes for special relativistic
 * (magneto)hydrodynamics" (arXiv 2107.12027), on one MI355X (gfx950) GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every array argument is a DEVICE pointer owned by the caller; the
 *   library never frees it and keeps no reference after the call returns.
 *   Scalars that feed back into the computation (time step, mesh-move limiter)
 *   stay in device memory ("*_dev" arguments) so a whole step runs without a
 *   host synchronisation.  Only es_ctx_status() synchronises.
 * Streams.  Work is enqueued on the given hipStream_t; calls on one stream
 *   are ordered.  Calls that share an es_ctx use its workspace and must not
 *   run concurrently on different streams.
 * Layout.  All fields are float64, component-major structure-of-arrays:
 *   a[c * nodes + node].  Interior node fields ("interior", nodes = n0*n1*n2)
 *   index node = (k*n1 + j)*n0 + i with i fastest along xi_1.  Padded fields
 *   ("padded") cover the box grown by ng ghost layers on each side of every
 *   active axis, ng = es_ghost_layers() = 3 for p = 2 and p = 3 and 4 for p = 4
 *   (the 2p-th order stencils reach p nodes past an edge): P0 = n0+2ng,
 *   P1 = n1+2ng, P2 = n2+2ng (3D) or 1 (2D), node = ((k+g)*P1 + (j+ng))*P0 + (i+ng)
 *   with g = ng in 3D and 0 in 2D.
 * Variables.  m = es_nvars(): 2D RHD (D, m1, m2, E); 3D RHD (D, m1, m2, m3, E);
 *   RMHD (D, m1, m2, m3, E, B1, B2, B3) (eq. RMHDdiv2).  Ucurv = J U (eq. RMHDCurv).
 *   Primitive interior input (es_prim2con): (rho, u_1..u_nu, p[, B1, B2, B3])
 *   with u = W v (nu = dim for RHD, 3 for RMHD) -- the same slots as U.
 *   Padded primitive output of es_con2prim has es_nprim() = m + 2 components:
 *   the m primitive slots, then ln(rho) and ln(beta), beta = rho/p.
 *   Metrics (es_nmet() = d(d+1) padded components): comp k*(d+1) is
 *   J dxi_k/dt, comp k*(d+1)+1+j is J dxi_k/dx_j (Section 3.3).
 * Errors.  Every entry point returns es_status; no C++ exception crosses the
 *   ABI.  Invalid arguments give ES_EINVAL before anything is enqueued.  A HIP
 *   launch error gives ES_EHIP.  Conservative-to-primitive failures, and
 *   nodes whose Jacobian is not positive, are recorded on the device (count
 *   and first failing interior node, the primitive output is NaN there) and
 *   reported by es_ctx_status().
 */
#ifndef ES_H
#define ES_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ES_OK = 0,
    ES_EINVAL = 1,        /* bad argument (sizes, null pointer, unsupported option) */
    ES_EADMISSIBLE = 2,   /* a state outside the admissible set reached con2prim */
    ES_ENOCONV = 3,       /* con2prim iteration did not converge */
    ES_EMESH = 4,         /* non-positive Jacobian (tangled mesh), reported by es_ctx_status */
    ES_EHIP = 5,          /* HIP runtime error */
    ES_EUNSUPPORTED = 6,  /* valid option not built into this library */
    ES_ETOOLARGE = 7      /* grid exceeds the static scratch of an allocation-free entry point */
} es_status;

enum { ES_RHD = 0, ES_RMHD = 1 };
enum { ES_BC_PERIODIC = 0, ES_BC_OUTFLOW = 1 };
enum { ES_SIGMA_RHO = 0, ES_SIGMA_LNRHO = 1 };
enum { ES_MON_PAPER = 0, ES_MON_SQGRAD = 1, ES_MON_GRADLAP = 2 };

/* Computational grid: a fixed orthogonal index box with constant spacing
 * (Section 3.2).  Periodic axes wrap the solution and shift the mesh
 * coordinate of that axis by period[k]; outflow axes copy the solution
 * (zero gradient) and extend the mesh by odd reflection. */
typedef struct {
    int dim;            /* 2 or 3 */
    int n[3];           /* interior nodes per axis, n[2] = 1 in 2D; >= 7 on outflow axes */
    int bc[3];          /* ES_BC_PERIODIC / ES_BC_OUTFLOW */
    double dxi[3];      /* computational spacing Delta xi_k */
    double period[3];   /* physical period of periodic axes */
} es_grid;

/* Scheme parameters (Sections 3-4, eq. cfl). */
typedef struct {
    int phys;           /* ES_RHD / ES_RMHD */
    double gamma;       /* adiabatic index of the ideal EOS (eq. EOS) */
    int order_p;        /* p of the 2p-th order EC flux and metrics with WENO of order
                           2p - 1 (Section 4): p = 2, 3 or 4 (RHD and RMHD, FP64 and
                           FP32-mixed; the adjoint entry points take p = 2 and 3 and
                           give ES_EUNSUPPORTED for p = 4); outflow axes need at
                           least 2 ng + 1 nodes (ES_EINVAL); other p give
                           ES_EUNSUPPORTED */
    int dissipation;    /* 0: entropy conservative, 1: entropy stable (WENO-(2p-1)) */
    int mixed;          /* 0: FP64 throughout.  1: FP32-mixed residual: the two-point
                           pair algebra (except the small-jump branch of the
                           logarithmic means) in FP32; the face dissipation in FP32
                           (RHD: state, eigenvectors, WENO, switch; RMHD: the
                           projections, WENO and switch, the numeric eigen-structure
                           staying FP64); metrics, their contraction with the pair
                           algebra, the Godunov-Powell source pair, the VCL, the
                           residual accumulation, con2prim, CFL, mesh and state in FP64 */
    double weno_eps;    /* WENO-JS epsilon */
    double cfl;         /* CFL number of eq. cfl */
} es_scheme;

/* Adaptive mesh redistribution (Section 5). */
typedef struct {
    int enabled;        /* 0: static mesh (xdot = 0) */
    int sigma;          /* ES_SIGMA_RHO / ES_SIGMA_LNRHO: monitored variable */
    int form;           /* ES_MON_PAPER: sqrt(1 + alpha |grad s| / max |grad s|) (eq. monitor);
                           ES_MON_SQGRAD: sqrt(1 + alpha |grad s|^2);
                           ES_MON_GRADLAP: sqrt(1 + alpha |grad s| / max |grad s|
                             + alpha2 |Lap s| / max |Lap s|) (eq. RMHD_2DVortex_Monitor),
                           gradient and Laplacian in xi by second-order central
                           differences (one-sided on outflow edges); a term whose
                           maximum is zero is dropped */
    double alpha;
    int filter_passes;  /* low-pass filter passes */
    int sweeps;         /* Jacobi sweeps mu */
    double alpha2;      /* Laplacian weight of ES_MON_GRADLAP (unused by the other forms) */
} es_monitor;

typedef struct es_ctx es_ctx;

/* Validate the options and allocate the context workspace (device memory
 * sized for one grid).  *out receives the context; free with es_destroy. */
es_status es_create(const es_grid* grid, const es_scheme* scheme, const es_monitor* monitor,
                    es_ctx** out);
es_status es_destroy(es_ctx* ctx);

size_t es_nvars(const es_ctx* ctx);          /* m */
size_t es_nprim(const es_ctx* ctx);          /* m + 2 */
size_t es_nmet(const es_ctx* ctx);           /* d (d + 1) */
size_t es_nodes(const es_ctx* ctx);          /* interior nodes */
size_t es_padded_nodes(const es_ctx* ctx);   /* padded nodes */
size_t es_ghost_layers(const es_ctx* ctx);   /* ng of the padded layout: 3 (p <= 3) or 4 (p = 4) */

/* Ucurv = J U(prim) on the interior (eq. RMHDdiv2, eq. RMHDCurv).
 * prim: interior, m comps (rho, u, p[, B]); J: interior; Ucurv: interior, m comps. */
es_status es_prim2con(es_ctx* ctx, const double* prim, const double* J, double* Ucurv,
                      hipStream_t stream);

/* Discrete metrics (Section 3.3, eq. SCLCoeff, eq. VCLCoeff; Appendix B in 2D)
 * with the 2p-th order central difference delta_k, evaluated on the padded box
 * from the mesh x (interior, d comps) extended by the boundary rule.
 * xdot: interior mesh velocity (d comps) or NULL for zero temporal metrics.
 * met: padded, d(d+1) comps.  J0: NULL, or interior output of the initial
 * Jacobian (2D: (delta_xi[x] delta_eta[y] - delta_eta[x] delta_xi[y])/(dxi deta);
 * 3D: sum_k (J dxi_k/dx_1) delta_k[x_1]/dxi_k). */
es_status es_metrics(es_ctx* ctx, const double* x, const double* xdot, double* met, double* J0,
                     hipStream_t stream);

/* Conservative-to-primitive recovery (Section 1: the nonlinear algebraic
 * equation; solver of this build: safeguarded Newton on p for RHD) at every
 * padded node, ghosts filled by the boundary rule.  Ucurv, J: interior.
 * prim: padded, m + 2 comps. */
es_status es_con2prim(es_ctx* ctx, const double* Ucurv, const double* J, double* prim,
                      hipStream_t stream);

/* Semi-discrete right-hand side (eq. RMHDSemiU_O2p_ES, eq. RMHDSemiJ_O2p_ES):
 * 2p-th order EC flux differences built from two-point EC fluxes (Proposition
 * 4.1), ES dissipation (eq. ESFlux_HO) when scheme.dissipation = 1, the
 * Godunov-Powell source for RMHD and the VCL.  prim, met: padded (from
 * es_con2prim / es_metrics).  dUcurv: interior m comps; dJ: interior. */
es_status es_residual(es_ctx* ctx, const double* prim, const double* met, double* dUcurv,
                      double* dJ, hipStream_t stream);

/* CFL time step (eq. cfl): dt = CFL / sum_k max_i rho_{k,i}/dxi_k with
 * rho_{k,i} = L_k max_m |lambda_m| / J_i (fluid speeds on the current mesh).
 * prim, met: padded; J: interior; dt_dev: one device double (output). */
es_status es_cfl(es_ctx* ctx, const double* prim, const double* met, const double* J,
                 double* dt_dev, hipStream_t stream);

/* Allocation-free CFL step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the computation of es_cfl on a grid and scheme given directly,
 * without a context.  The per-block maxima of the reduction live in a static
 * device array of 3 * ES_CFL_STATIC_MAX_BLOCKS doubles (3 MiB) that every GPU
 * the library runs on holds until the process ends; no call allocates or frees
 * memory.  Grids needing more blocks than ES_CFL_STATIC_MAX_BLOCKS
 * (es_cfl_static_blocks: ceil(n0/64) * ceil(n1/4) * n2) return ES_ETOOLARGE
 * before anything is enqueued.  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (different streams or threads without ordering)
 * race and must not be issued.  The array needs no clearing: each call writes
 * every entry it reads.  prim, met: padded (es_con2prim / es_metrics layouts);
 * J: interior; dt_dev: one device double (output).  Other errors as es_cfl. */
#define ES_CFL_STATIC_MAX_BLOCKS 131072
size_t es_cfl_static_blocks(const es_grid* grid);
es_status es_cfl_noalloc(const es_grid* grid, const es_scheme* scheme, const double* prim,
                         const double* met, const double* J, double* dt_dev, hipStream_t stream);

/* Mesh redistribution (Section 5): monitor, low-pass filter, Jacobi sweeps,
 * move limiter Delta_tau, x_new = x + Delta_tau (x^[mu] - x),
 * xdot = Delta_tau (x^[mu] - x) / dt.  prim: padded; x: interior (d comps);
 * dt_dev: device double; x_new, xdot: interior outputs (d comps);
 * dtau_dev: NULL or device double output.  x_new must not alias x. */
es_status es_mesh_redistribute(es_ctx* ctx, const double* prim, const double* x,
                               const double* dt_dev, double* x_new, double* xdot,
                               double* dtau_dev, hipStream_t stream);

/* One third-order SSP Runge-Kutta step of the whole scheme (con2prim, CFL,
 * mesh redistribution when enabled, three stages with metrics recomputed on
 * the stage meshes x + c dt xdot, c = 0, 1, 1/2), in place on Ucurv, J, x
 * (interior).  xdot: interior output (d comps).  dt_dev: device double output.
 * If fixed_dt_dev is not NULL the step uses that device value instead of the
 * CFL step. */
es_status es_rk3_step(es_ctx* ctx, double* Ucurv, double* J, double* x, double* xdot,
                      double* dt_dev, const double* fixed_dt_dev, hipStream_t stream);

/* One SSP-RK3 step on a prescribed moving mesh (the accuracy tests of Section 6
 * move the nodes by a given formula instead of the redistribution of Section 5):
 * as es_rk3_step, with the mesh velocity xdot (interior, d comps, device, read
 * only) given by the caller and held over the step; the stage meshes are
 * x + c dt xdot and x is advanced in place to x + dt xdot.  The monitor of the
 * context is not used.  Errors as es_rk3_step. */
es_status es_rk3_step_moving(es_ctx* ctx, double* Ucurv, double* J, double* x, const double* xdot,
                             double* dt_dev, const double* fixed_dt_dev, hipStream_t stream);

/* Adjoint (FP64 form only, p = 3 or p = 2; ES_EUNSUPPORTED for scheme.mixed = 1 or p = 4).
 * For RMHD the ES dissipation's face eigen-structure (the columns of R and
 * lambda^) is held at its forward value as well: the pair fluxes, the
 * Godunov-Powell source and the projections/WENO/accumulation of the dissipation
 * are differentiated, the numeric eigen-decomposition is not.  The
 * derivatives are those of the step with the mesh trajectory (x^n, xdot), the
 * time step dt and every branch decision (the sign switch Y of eq. ESFlux_HO,
 * the maximum in lambda^, the log-mean series branch) held at their forward
 * values; for a static mesh (monitor disabled) with a fixed dt this is the
 * exact derivative of the step.  con2prim is differentiated by the
 * implicit-function rule, dP/dU = (dU/dP)^{-1}.  The first adjoint call on a
 * context allocates its adjoint workspace.
 *
 * es_ckpt_doubles: size (in doubles) of the checkpoint of one step: the stage
 * states Ucurv^(0..2) (m comps each) and J^(0..2), x^n, xdot (d comps each) and
 * dt, all interior.
 *
 * es_rk3_step_save: es_rk3_step (always launched eagerly, not as a graph) that
 * also writes that checkpoint into ckpt (device, caller-owned). */
size_t es_ckpt_doubles(const es_ctx* ctx);
es_status es_rk3_step_save(es_ctx* ctx, double* Ucurv, double* J, double* x, double* xdot,
                           double* dt_dev, const double* fixed_dt_dev, double* ckpt,
                           hipStream_t stream);

/* Vector-Jacobian product of one saved step: given the cotangents lamU (m
 * comps) and lamJ of (Ucurv^{n+1}, J^{n+1}), writes the cotangents gU, gJ of
 * (Ucurv^n, J^n).  ckpt: from es_rk3_step_save on the same context.  Uses the
 * context's metrics and primitive workspace.  All arrays interior, device. */
es_status es_rk3_step_vjp(es_ctx* ctx, const double* ckpt, const double* lamU, const double* lamJ,
                          double* gU, double* gJ, hipStream_t stream);

/* Vector-Jacobian product of the state residual L(Ucurv, J) = residual(
 * con2prim(Ucurv, J), met) (its m state components; the VCL part does not
 * depend on the state): gU = (dL/dUcurv)^T lamU, gJ = (dL/dJ)^T lamU.
 * Ucurv, lamU, gU: interior m comps; J, gJ: interior; met: padded (es_metrics).
 * Overwrites the context's primitive workspace. */
es_status es_residual_vjp(es_ctx* ctx, const double* Ucurv, const double* J, const double* met,
                          const double* lamU, double* gU, double* gJ, hipStream_t stream);

/* Vector-Jacobian product of the conservative-to-primitive recovery at the
 * interior nodes (the implicit-function rule, as inside the adjoint): with
 * P(U) the primitive state (rho, u, p[, B]) that con2prim recovers from
 * U = Ucurv / J, gU = (dP/dUcurv)^T gprim and gJ = (dP/dJ)^T gprim, i.e.
 * y = (dU/dP)^{-T} gprim at the converged state, gU = y / J, gJ = -(y . Ucurv) / J^2.
 * Ucurv, gU: interior m comps; J, gJ: interior; gprim: interior, m comps in the
 * primitive slots (the layout es_prim2con reads).  Runs es_con2prim into the
 * context's primitive workspace first; failures are recorded as there
 * (es_ctx_status).  Any scheme of the context (FP64 or mixed, any p). */
es_status es_con2prim_vjp(es_ctx* ctx, const double* Ucurv, const double* J, const double* gprim,
                          double* gU, double* gJ, hipStream_t stream);

/* Vector-Jacobian product of es_prim2con, Ucurv = J U(prim) (eq. RMHDdiv2,
 * eq. RMHDCurv): gprim = J (dU/dP)^T gUcurv and, if gJ is not NULL,
 * gJ = U(prim) . gUcurv.  prim: interior, m comps (as es_prim2con); J: interior;
 * gUcurv: interior m comps; gprim: interior m comps (output). */
es_status es_prim2con_vjp(es_ctx* ctx, const double* prim, const double* J, const double* gUcurv,
                          double* gprim, double* gJ, hipStream_t stream);

/* Replay es_rk3_step and es_rk3_step_moving as a HIP graph (default 1) or
 * launch their kernels one by one (0).  In graph mode the step is captured on
 * the context's own stream the first time it is called with a given set of
 * array pointers (captured again when they change) and the graph is launched
 * into the caller's stream, ordered with its other work; the results are those
 * of the eager launch sequence. */
es_status es_set_graph(es_ctx* ctx, int enable);

/* FP64 diagnostics on the interior (Theorem 4.1 / 5.1, Section 6 total entropy):
 * out_dev[0] = sum_i (V_i . dUcurv_i - phi_i dJ_i)   (entropy production rate)
 * out_dev[1] = sum_i J_i eta_i                         (total entropy)
 * out_dev[2] = sum_i J_i
 * out_dev[3 .. 3+m) = sum_i Ucurv_i                    (conserved totals)
 * prim: padded; the other arrays interior; out_dev: device, 3 + m doubles. */
es_status es_diagnostics(es_ctx* ctx, const double* prim, const double* Ucurv, const double* J,
                         const double* dUcurv, const double* dJ, double* out_dev,
                         hipStream_t stream);

/* Synchronise the stream and report the failures recorded by con2prim since the
 * last call (then clear them): ES_EMESH if some node's Jacobian J was not
 * positive (a tangled mesh: every con2prim of a step, i.e. of every stage
 * state, checks the evolved J of eq. RMHDSemiJ_O2p_ES before recovering the
 * state; the node's primitive output is NaN), else ES_EADMISSIBLE (a state
 * outside the admissible set), else ES_ENOCONV, else ES_OK.  n_fail (all
 * failing interior nodes) and first_fail (the smallest failing interior node
 * index) may be NULL. */
es_status es_ctx_status(es_ctx* ctx, hipStream_t stream, long long* n_fail, long long* first_fail);

const char* es_status_string(es_status s);

#ifdef __cplusplus
}
#endif
#endif /* ES_H */
