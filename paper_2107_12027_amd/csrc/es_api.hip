// C ABI of libes.so: context, argument validation and the SSP-RK3 step.
#include <limits.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "es_internal.h"

using es::GridDev;

namespace {

es_status hip_status(hipError_t e) { return e == hipSuccess ? ES_OK : ES_EHIP; }

#define ES_TRY(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return ES_EHIP;          \
    } while (0)

bool valid_grid(const es_grid* g) {
    if (g == nullptr || (g->dim != 2 && g->dim != 3)) return false;
    for (int k = 0; k < 3; ++k) {
        if (k >= g->dim) {
            if (g->n[k] != 1) return false;
            continue;
        }
        if (g->bc[k] != ES_BC_PERIODIC && g->bc[k] != ES_BC_OUTFLOW) return false;
        if (!(g->dxi[k] > 0.0)) return false;
        // the mesh extension by reflection reaches 2 ng nodes past an edge (6 for
        // p <= 3; es_create asks for 9 when p = 4)
        if (g->bc[k] == ES_BC_OUTFLOW && g->n[k] < 7) return false;
        if (g->bc[k] == ES_BC_PERIODIC && (g->n[k] < 1 || !(g->period[k] > 0.0))) return false;
        if (g->n[k] > (1 << 24)) return false;
    }
    return true;
}

template <typename T>
hipError_t alloc(T** p, size_t n) {
    return hipMalloc((void**)p, (n > 0 ? n : 1) * sizeof(T));
}

// The host part of a context: options and the device grid description (no
// device memory).
void describe(es_ctx* c, const es_grid* grid, const es_scheme* scheme, const es_monitor* monitor) {
    memset(c, 0, sizeof(*c));
    c->grid = *grid;
    c->scheme = *scheme;
    if (monitor != nullptr) c->monitor = *monitor;
    GridDev& g = c->g;
    g.dim = grid->dim;
    g.ng = es::ghost_layers(scheme->order_p);
    for (int k = 0; k < 3; ++k) {
        g.n[k] = grid->n[k];
        g.bc[k] = grid->bc[k];
        g.dxi[k] = grid->dxi[k];
        g.period[k] = grid->period[k];
        g.P[k] = (k < grid->dim) ? grid->n[k] + 2 * g.ng : 1;
    }
    g.g2 = grid->dim == 3 ? g.ng : 0;
    for (int k = 0; k < 3; ++k) g.E[k] = (k < grid->dim) ? grid->n[k] + 4 * g.ng : 1;
    g.g6 = grid->dim == 3 ? 2 * g.ng : 0;
    g.nodes = (long long)g.n[0] * g.n[1] * g.n[2];
    g.pnodes = (long long)g.P[0] * g.P[1] * g.P[2];
    g.enodes = (long long)g.E[0] * g.E[1] * g.E[2];
    g.p = scheme->order_p;
    c->m = scheme->phys == ES_RMHD ? 8 : grid->dim + 2;
    c->nprim = c->m + 2;
    c->nmet = grid->dim * (grid->dim + 1);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free CFL step: the per-block maxima of the CFL
// kernels (dim slabs of one double per block) in a static device array.  Every
// GPU the library runs on holds its own copy until the process ends; host code
// never passes the array's name to a kernel (in host code it is a stand-in, not
// a device address) but the address hipGetSymbolAddress returns for the
// current device, resolved once per device and kept.
// ---------------------------------------------------------------------------
constexpr long long kCflScratchDoubles = 3LL * ES_CFL_STATIC_MAX_BLOCKS;
static __device__ __align__(256) double scratch[kCflScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double* scratch_dev[kMaxDevices];   // device address of `scratch` per device (null: not resolved yet)

hipError_t scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (scratch_dev[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char* es_status_string(es_status s) {
    switch (s) {
        case ES_OK: return "ok";
        case ES_EINVAL: return "invalid argument";
        case ES_EADMISSIBLE: return "inadmissible state in con2prim";
        case ES_ENOCONV: return "con2prim did not converge";
        case ES_EMESH: return "non-positive Jacobian";
        case ES_EHIP: return "HIP runtime error";
        case ES_EUNSUPPORTED: return "option not supported by this build";
        case ES_ETOOLARGE: return "grid exceeds the static scratch of an allocation-free entry point";
    }
    return "unknown status";
}

es_status es_create(const es_grid* grid, const es_scheme* scheme, const es_monitor* monitor,
                    es_ctx** out) {
    if (out == nullptr) return ES_EINVAL;
    *out = nullptr;
    if (!valid_grid(grid) || scheme == nullptr || monitor == nullptr) return ES_EINVAL;
    if (scheme->phys != ES_RHD && scheme->phys != ES_RMHD) return ES_EINVAL;
    if (!(scheme->gamma > 1.0 && scheme->gamma <= 2.0)) return ES_EINVAL;
    if (!(scheme->weno_eps > 0.0) || !(scheme->cfl > 0.0)) return ES_EINVAL;
    if (scheme->dissipation != 0 && scheme->dissipation != 1) return ES_EINVAL;
    if (scheme->mixed != 0 && scheme->mixed != 1) return ES_EINVAL;
    if (monitor->enabled) {
        if (monitor->sigma != ES_SIGMA_RHO && monitor->sigma != ES_SIGMA_LNRHO) return ES_EINVAL;
        if (monitor->form != ES_MON_PAPER && monitor->form != ES_MON_SQGRAD &&
            monitor->form != ES_MON_GRADLAP)
            return ES_EINVAL;
        if (monitor->filter_passes < 0 || monitor->sweeps < 0 || !(monitor->alpha >= 0.0) ||
            !(monitor->alpha2 >= 0.0))
            return ES_EINVAL;
    }
    // kernels of this build: p = 2, 3 and 4 (RHD and RMHD, FP64 or FP32-mixed)
    if (scheme->order_p != 3 && scheme->order_p != 2 && scheme->order_p != 4) return ES_EUNSUPPORTED;
    for (int k = 0; k < grid->dim; ++k)
        if (grid->bc[k] == ES_BC_OUTFLOW && grid->n[k] < 2 * es::ghost_layers(scheme->order_p) + 1) return ES_EINVAL;

    es_ctx* c = new (std::nothrow) es_ctx();
    if (c == nullptr) return ES_EHIP;
    describe(c, grid, scheme, monitor);
    const GridDev& g = c->g;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return ES_EHIP; }
    c->red_blocks = es::reduction_blocks(g);
    const size_t N = (size_t)g.nodes, P = (size_t)g.pnodes, d = (size_t)grid->dim;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = alloc(&c->prim, P * c->nprim);
    if (e == hipSuccess) e = alloc(&c->met, P * c->nmet);
    if (e == hipSuccess && grid->dim == 2) e = alloc(&c->met1, P * c->nmet);
    if (e == hipSuccess) e = alloc(&c->met2, P * c->nmet);
    if (e == hipSuccess) e = alloc(&c->L, N * (c->m + 1) * d);
    if (e == hipSuccess) e = alloc(&c->Us, N * c->m);
    if (e == hipSuccess) e = alloc(&c->Js, N);
    if (e == hipSuccess) e = alloc(&c->Us2, N * c->m);
    if (e == hipSuccess) e = alloc(&c->Js2, N);
    if (e == hipSuccess) e = alloc(&c->xnew, N * d);
    if (e == hipSuccess) e = alloc(&c->xa, N * d);
    if (e == hipSuccess) e = alloc(&c->xb, N * d);
    if (e == hipSuccess) e = alloc(&c->wa, N);
    if (e == hipSuccess) e = alloc(&c->wb, N);
    if (e == hipSuccess) e = alloc(&c->xe, (size_t)g.enodes * d);
    if (e == hipSuccess) e = alloc(&c->ve, (size_t)g.enodes * d);
    if (e == hipSuccess && grid->dim == 3) e = alloc(&c->pi, (size_t)g.enodes * 9);
    if (e == hipSuccess) e = alloc(&c->red, (size_t)c->red_blocks * (3 + 8));
    if (e == hipSuccess) e = alloc(&c->scal, (size_t)es::NSCAL);
    if (e == hipSuccess) e = alloc(&c->fail, (size_t)4);
    if (e == hipSuccess) {
        (void)es::launch_fill_u64(c->fail, 0ull, 2, nullptr);
        (void)es::launch_fill_u64(c->fail + 3, 0ull, 1, nullptr);
        e = es::launch_fill_u64(c->fail + 2, ULLONG_MAX, 1, nullptr);
    }
    // the primitive workspace seeds the pressure iteration of the next step: start
    // from zeros (an invalid seed, so the first step uses the bracket midpoint)
    if (e == hipSuccess) e = es::launch_zero(c->prim, (long long)(P * c->nprim), nullptr);
    c->use_graph = 1;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        es_destroy(c);
        return ES_EHIP;
    }
    *out = c;
    return ES_OK;
}

es_status es_destroy(es_ctx* c) {
    if (c == nullptr) return ES_EINVAL;
    void* bufs[] = {c->prim, c->met, c->met1, c->met2, c->L, c->Us, c->Js, c->Us2, c->Js2, c->xnew, c->xa, c->xb,
                    c->wa, c->wb, c->xe, c->ve, c->pi, c->red, c->scal, c->fail,
                    c->adj_lamU, c->adj_lamJ, c->adj_lamL, c->adj_accU, c->adj_accJ,
                    c->adj_gU, c->adj_gJ, c->gdir, c->adj_eig};
    if (c->gexec != nullptr) (void)hipGraphExecDestroy(c->gexec);
    if (c->cap != nullptr) (void)hipStreamDestroy(c->cap);
    for (void* b : bufs)
        if (b != nullptr) (void)hipFree(b);
    delete c;
    return ES_OK;
}

size_t es_nvars(const es_ctx* c) { return c ? (size_t)c->m : 0; }
size_t es_nprim(const es_ctx* c) { return c ? (size_t)c->nprim : 0; }
size_t es_nmet(const es_ctx* c) { return c ? (size_t)c->nmet : 0; }
size_t es_nodes(const es_ctx* c) { return c ? (size_t)c->g.nodes : 0; }
size_t es_padded_nodes(const es_ctx* c) { return c ? (size_t)c->g.pnodes : 0; }
size_t es_ghost_layers(const es_ctx* c) { return c ? (size_t)c->g.ng : 0; }

es_status es_prim2con(es_ctx* c, const double* prim, const double* J, double* U, hipStream_t s) {
    if (c == nullptr || prim == nullptr || J == nullptr || U == nullptr) return ES_EINVAL;
    return hip_status(es::launch_prim2con(c, prim, J, U, s));
}

es_status es_metrics(es_ctx* c, const double* x, const double* xdot, double* met, double* J0,
                     hipStream_t s) {
    if (c == nullptr || x == nullptr || met == nullptr) return ES_EINVAL;
    return hip_status(es::launch_metrics(c, x, xdot, nullptr, 0.0, met, J0, s));
}

es_status es_con2prim(es_ctx* c, const double* U, const double* J, double* prim, hipStream_t s) {
    if (c == nullptr || U == nullptr || J == nullptr || prim == nullptr) return ES_EINVAL;
    return hip_status(es::launch_con2prim(c, U, J, prim, 0, s));
}

es_status es_residual(es_ctx* c, const double* prim, const double* met, double* dU, double* dJ,
                      hipStream_t s) {
    if (c == nullptr || prim == nullptr || met == nullptr || dU == nullptr || dJ == nullptr)
        return ES_EINVAL;
    return hip_status(es::launch_residual(c, prim, met, dU, dJ, s));
}

es_status es_cfl(es_ctx* c, const double* prim, const double* met, const double* J, double* dt_dev,
                 hipStream_t s) {
    if (c == nullptr || prim == nullptr || met == nullptr || J == nullptr || dt_dev == nullptr)
        return ES_EINVAL;
    return hip_status(es::launch_cfl(c, prim, met, J, dt_dev, nullptr, s));
}

size_t es_cfl_static_blocks(const es_grid* grid) {
    if (!valid_grid(grid)) return 0;
    return (size_t)((grid->n[0] + 63) / 64) * (size_t)((grid->n[1] + 3) / 4) * (size_t)grid->n[2];
}

es_status es_cfl_noalloc(const es_grid* grid, const es_scheme* scheme, const double* prim, const double* met,
                         const double* J, double* dt_dev, hipStream_t s) {
    if (grid == nullptr || scheme == nullptr || prim == nullptr || met == nullptr || J == nullptr ||
        dt_dev == nullptr)
        return ES_EINVAL;
    if (!valid_grid(grid)) return ES_EINVAL;
    if (scheme->phys != ES_RHD && scheme->phys != ES_RMHD) return ES_EINVAL;
    if (!(scheme->gamma > 1.0 && scheme->gamma <= 2.0) || !(scheme->cfl > 0.0)) return ES_EINVAL;
    if (scheme->order_p != 2 && scheme->order_p != 3 && scheme->order_p != 4) return ES_EINVAL;
    if (es_cfl_static_blocks(grid) > (size_t)ES_CFL_STATIC_MAX_BLOCKS) return ES_ETOOLARGE;
    double* red = nullptr;
    ES_TRY(scratch_address(&red));
    // a context on the stack that owns no device memory: the CFL kernels read its
    // grid, scheme and reduction buffer only
    es_ctx tmp;
    describe(&tmp, grid, scheme, nullptr);
    tmp.red = red;
    tmp.red_blocks = es::reduction_blocks(tmp.g);
    if ((size_t)tmp.red_blocks != es_cfl_static_blocks(grid)) return ES_EINVAL;
    return hip_status(es::launch_cfl(&tmp, prim, met, J, dt_dev, nullptr, s));
}

es_status es_mesh_redistribute(es_ctx* c, const double* prim, const double* x, const double* dt_dev,
                               double* x_new, double* xdot, double* dtau_dev, hipStream_t s) {
    if (c == nullptr || prim == nullptr || x == nullptr || dt_dev == nullptr || x_new == nullptr ||
        xdot == nullptr || x_new == x)
        return ES_EINVAL;
    if (!c->monitor.enabled) return hip_status(es::launch_zero_mesh_velocity(c, x, x_new, xdot, s));
    return hip_status(es::launch_mesh(c, prim, x, dt_dev, x_new, xdot, dtau_dev, s));
}

// xdot_in: NULL for the scheme's own mesh (adaptive redistribution, or a static
// mesh), else the caller's mesh velocity, held over the step (xdot unused then)
static es_status enqueue_step(es_ctx* c, double* U, double* J, double* x, double* xdot,
                              double* dt_dev, const double* fixed_dt_dev, hipStream_t s,
                              double* ckpt = nullptr, const double* xdot_in = nullptr) {
    const long long N = c->g.nodes, nU = N * c->m, nX = N * c->g.dim;
    const es::Checkpoint k = ckpt ? es::checkpoint_layout(c, ckpt) : es::Checkpoint{};
    auto w = [](const double* p) { return const_cast<double*>(p); };
    if (ckpt) {
        ES_TRY(es::launch_copy(w(k.U[0]), U, nU, s));
        ES_TRY(es::launch_copy(w(k.J[0]), J, N, s));
        ES_TRY(es::launch_copy(w(k.x), x, nX, s));
    }
    // con2prim (the primitive workspace holds the previous stage and seeds the
    // pressure iteration), metrics on x^n (spatial part), CFL step
    // (with the adaptive mesh, dt is finalised inside the mesh launches)
    ES_TRY(es::launch_con2prim(c, U, J, c->prim, 1, s));
    const bool adaptive = c->monitor.enabled != 0 && xdot_in == nullptr;
    bool grad_done = false;
    ES_TRY(es::launch_cfl_mesh(c, c->prim, x, J, dt_dev, fixed_dt_dev, s, adaptive, adaptive, &grad_done));
    // mesh redistribution: x^{n+1} into c->xnew, mesh velocity into xdot
    if (xdot_in != nullptr) {
        xdot = const_cast<double*>(xdot_in);
        ES_TRY(es::launch_mesh_advance(c, x, xdot_in, dt_dev, c->xnew, s));
    } else if (adaptive) {
        ES_TRY(es::launch_mesh(c, c->prim, x, dt_dev, c->xnew, xdot, nullptr, s, true, fixed_dt_dev, grad_done));
    } else {
        ES_TRY(es::launch_zero_mesh_velocity(c, x, c->xnew, xdot, s));
    }
    if (ckpt) {
        ES_TRY(es::launch_copy(w(k.dt), dt_dev, 1, s));
        ES_TRY(es::launch_copy(w(k.xdot), xdot, nX, s));
    }
    // stages: the combinations of stages 0 and 1 are formed inside the next
    // con2prim (stage states in Us, then Us2); the last one also copies x^{n+1}
    static const double coef[3] = {0.0, 1.0, 0.5};
    const bool batched = es::metrics_stages_batched(c);
    if (batched) ES_TRY(es::launch_metrics_stages(c, x, xdot, dt_dev, c->met, c->met1, c->met2, s));
    // 3D: the CFL launch left the spatial metrics of x^n in c->met (unless dt was
    // prescribed), so stage 0, on the same mesh, adds only its temporal part
    const bool met0_spatial = !batched && fixed_dt_dev == nullptr;
    // 3D: the stage-2 metrics (into met2) right after the stage-1 ones, while the
    // extended mesh velocity that both read is still in cache
    for (int st = 0; st < 3; ++st) {
        const double* met = c->met;
        if (batched) {
            met = st == 0 ? c->met : (st == 1 ? c->met1 : c->met2);
        } else if (st == 0 && met0_spatial) {
            ES_TRY(es::launch_temporal_metrics3d(c, xdot, c->met, s));
        } else if (st == 2) {
            met = c->met2;
        } else {
            ES_TRY(es::launch_metrics(c, x, xdot, dt_dev, coef[st], c->met, nullptr, s, false));
            if (st == 1) ES_TRY(es::launch_metrics(c, x, xdot, dt_dev, coef[2], c->met2, nullptr, s, true));
        }
        ES_TRY(es::launch_residual_dirs(c, c->prim, met, c->L, s));
        if (st == 0) {
            ES_TRY(es::launch_combine_con2prim(c, 0, U, J, nullptr, nullptr, c->L, dt_dev, c->Us, c->Js,
                                               c->prim, s));
        } else if (st == 1) {
            ES_TRY(es::launch_combine_con2prim(c, 1, U, J, c->Us, c->Js, c->L, dt_dev, c->Us2, c->Js2,
                                               c->prim, s));
        } else {
            ES_TRY(es::launch_rk_combine(c, 2, U, J, c->Us2, c->Js2, c->L, dt_dev, s, c->xnew, x));
        }
        if (ckpt && st < 2) {
            ES_TRY(es::launch_copy(w(k.U[st + 1]), st == 0 ? c->Us : c->Us2, nU, s));
            ES_TRY(es::launch_copy(w(k.J[st + 1]), st == 0 ? c->Js : c->Js2, N, s));
        }
    }
    return ES_OK;
}

// one step through the context's HIP graph, captured again when the arguments change
static es_status graph_step(es_ctx* c, double* U, double* J, double* x, double* xdot, double* dt_dev,
                            const double* fixed_dt_dev, const double* xdot_in, hipStream_t s) {
    if (!c->use_graph) return enqueue_step(c, U, J, x, xdot, dt_dev, fixed_dt_dev, s, nullptr, xdot_in);
    const void* key[7] = {U, J, x, xdot, dt_dev, fixed_dt_dev, xdot_in};
    if (c->gexec == nullptr || memcmp(key, c->gkey, sizeof(key)) != 0) {
        if (c->gexec != nullptr) {
            ES_TRY(hipGraphExecDestroy(c->gexec));
            c->gexec = nullptr;
        }
        // the capture stream must not depend on earlier work while capturing
        ES_TRY(hipStreamSynchronize(c->cap));
        ES_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        const es_status st = enqueue_step(c, U, J, x, xdot, dt_dev, fixed_dt_dev, c->cap, nullptr, xdot_in);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap, &graph);
        if (st != ES_OK || e != hipSuccess || graph == nullptr) {
            if (graph != nullptr) (void)hipGraphDestroy(graph);
            return st != ES_OK ? st : ES_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            c->gexec = nullptr;
            return ES_EHIP;
        }
        memcpy(c->gkey, key, sizeof(key));
    }
    // the replay goes into the caller's stream (ordered with its other work)
    ES_TRY(hipGraphLaunch(c->gexec, s));
    return ES_OK;
}

es_status es_rk3_step(es_ctx* c, double* U, double* J, double* x, double* xdot, double* dt_dev,
                      const double* fixed_dt_dev, hipStream_t s) {
    if (c == nullptr || U == nullptr || J == nullptr || x == nullptr || xdot == nullptr ||
        dt_dev == nullptr)
        return ES_EINVAL;
    return graph_step(c, U, J, x, xdot, dt_dev, fixed_dt_dev, nullptr, s);
}

es_status es_rk3_step_moving(es_ctx* c, double* U, double* J, double* x, const double* xdot,
                             double* dt_dev, const double* fixed_dt_dev, hipStream_t s) {
    if (c == nullptr || U == nullptr || J == nullptr || x == nullptr || xdot == nullptr ||
        dt_dev == nullptr)
        return ES_EINVAL;
    return graph_step(c, U, J, x, nullptr, dt_dev, fixed_dt_dev, xdot, s);
}

// the adjoint covers the FP64 form, p = 2 and p = 3 (the ghost width of p <= 3)
static bool adjoint_supported(const es_ctx* c) {
    return c->scheme.mixed == 0 && (c->scheme.order_p == 3 || c->scheme.order_p == 2);
}

size_t es_ckpt_doubles(const es_ctx* c) { return c ? (size_t)es::checkpoint_doubles(c) : 0; }

es_status es_rk3_step_save(es_ctx* c, double* U, double* J, double* x, double* xdot, double* dt_dev,
                           const double* fixed_dt_dev, double* ckpt, hipStream_t s) {
    if (c == nullptr || U == nullptr || J == nullptr || x == nullptr || xdot == nullptr ||
        dt_dev == nullptr || ckpt == nullptr)
        return ES_EINVAL;
    if (!adjoint_supported(c)) return ES_EUNSUPPORTED;
    return enqueue_step(c, U, J, x, xdot, dt_dev, fixed_dt_dev, s, ckpt);
}

static es_status ensure_adjoint(es_ctx* c) {
    if (c->adj_lamU != nullptr) return ES_OK;
    const size_t N = (size_t)c->g.nodes, m = (size_t)c->m;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = alloc(&c->adj_lamU, N * m);
    if (e == hipSuccess) e = alloc(&c->adj_lamJ, N);
    if (e == hipSuccess) e = alloc(&c->adj_lamL, N * m);
    if (e == hipSuccess) e = alloc(&c->adj_accU, N * m);
    if (e == hipSuccess) e = alloc(&c->adj_accJ, N);
    if (e == hipSuccess) e = alloc(&c->adj_gU, N * m);
    if (e == hipSuccess) e = alloc(&c->adj_gJ, N);
    if (e == hipSuccess) e = alloc(&c->gdir, (size_t)c->g.pnodes * m * (size_t)c->g.dim);
    if (e == hipSuccess && c->scheme.phys == ES_RMHD && c->scheme.dissipation != 0)
        e = alloc(&c->adj_eig, es::face_eig_doubles_rmhd(c));
    if (e != hipSuccess) return ES_EHIP;
    // positions the residual VJP does not write (ghost corners) are never read;
    // clear once so the buffer holds no stale values
    ES_TRY(es::launch_zero(c->gdir, c->g.pnodes * c->m * c->g.dim, nullptr));
    ES_TRY(hipDeviceSynchronize());
    return ES_OK;
}

es_status es_residual_vjp(es_ctx* c, const double* U, const double* J, const double* met,
                          const double* lamU, double* gU, double* gJ, hipStream_t s) {
    if (c == nullptr || U == nullptr || J == nullptr || met == nullptr || lamU == nullptr ||
        gU == nullptr || gJ == nullptr)
        return ES_EINVAL;
    if (!adjoint_supported(c)) return ES_EUNSUPPORTED;
    const es_status st = ensure_adjoint(c);
    if (st != ES_OK) return st;
    return hip_status(es::launch_state_residual_vjp(c, U, J, met, lamU, gU, gJ, s));
}

es_status es_rk3_step_vjp(es_ctx* c, const double* ckpt, const double* lamU, const double* lamJ,
                          double* gU, double* gJ, hipStream_t s) {
    if (c == nullptr || ckpt == nullptr || lamU == nullptr || lamJ == nullptr || gU == nullptr ||
        gJ == nullptr)
        return ES_EINVAL;
    if (!adjoint_supported(c)) return ES_EUNSUPPORTED;
    const es_status st = ensure_adjoint(c);
    if (st != ES_OK) return st;
    return hip_status(es::launch_rk3_vjp(c, ckpt, lamU, lamJ, gU, gJ, s));
}

es_status es_con2prim_vjp(es_ctx* c, const double* U, const double* J, const double* gprim, double* gU,
                          double* gJ, hipStream_t s) {
    if (c == nullptr || U == nullptr || J == nullptr || gprim == nullptr || gU == nullptr || gJ == nullptr)
        return ES_EINVAL;
    return hip_status(es::launch_con2prim_vjp(c, U, J, gprim, gU, gJ, s));
}

es_status es_prim2con_vjp(es_ctx* c, const double* prim, const double* J, const double* gU, double* gprim,
                          double* gJ, hipStream_t s) {
    if (c == nullptr || prim == nullptr || J == nullptr || gU == nullptr || gprim == nullptr)
        return ES_EINVAL;
    return hip_status(es::launch_prim2con_vjp(c, prim, J, gU, gprim, gJ, s));
}

es_status es_set_graph(es_ctx* c, int enable) {
    if (c == nullptr || (enable != 0 && enable != 1)) return ES_EINVAL;
    c->use_graph = enable;
    return ES_OK;
}

es_status es_diagnostics(es_ctx* c, const double* prim, const double* U, const double* J,
                         const double* dU, const double* dJ, double* out, hipStream_t s) {
    if (c == nullptr || prim == nullptr || U == nullptr || J == nullptr || dU == nullptr ||
        dJ == nullptr || out == nullptr)
        return ES_EINVAL;
    return hip_status(es::launch_diagnostics(c, prim, U, J, dU, dJ, out, s));
}

es_status es_ctx_status(es_ctx* c, hipStream_t s, long long* n_fail, long long* first_fail) {
    if (c == nullptr) return ES_EINVAL;
    if (hipStreamSynchronize(s) != hipSuccess) return ES_EHIP;
    unsigned long long h[4];
    if (hipMemcpy(h, c->fail, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return ES_EHIP;
    if (n_fail) *n_fail = (long long)(h[0] + h[1] + h[3]);
    if (first_fail) *first_fail = h[2] == ULLONG_MAX ? -1 : (long long)h[2];
    (void)es::launch_fill_u64(c->fail, 0ull, 2, s);
    (void)es::launch_fill_u64(c->fail + 2, ULLONG_MAX, 1, s);
    (void)es::launch_fill_u64(c->fail + 3, 0ull, 1, s);
    if (hipStreamSynchronize(s) != hipSuccess) return ES_EHIP;
    if (h[3] > 0) return ES_EMESH;
    if (h[0] > 0) return ES_EADMISSIBLE;
    if (h[1] > 0) return ES_ENOCONV;
    return ES_OK;
}

}  // extern "C"
