#!/usr/bin/env python3
"""Benchmark: cell-updates/s of one SSP-RK3 step of the entropy-stable adaptive
moving-mesh scheme (2D RHD quadrant Riemann problem, 400 x 400 nodes, adaptive
mesh with 10 Jacobi sweeps, FP64) on one MI355X.

One step = the whole hot path: con2prim, CFL step, mesh redistribution
(monitor, filter, Jacobi sweeps, Delta_tau, new mesh and mesh velocity) and
three Runge-Kutta stages of metrics + con2prim + residual + combination.
Inputs are resident in HBM before the timed region; the time step stays on the
device (no host synchronisation inside the timed steps).

The headline value is the FP64 path.  The same workload is then timed in the
FP32-mixed form (scheme.mixed = 1) and reported under "mixed", with the relative
L1 error of one step from the initial data against the oracle's step for both
forms (the oracle step is the cpu_baseline run).

Prints one JSON line (see the repository contract).  ``--gpus N`` with N > 1
exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK3 step, FP64 vs FP32-mixed at stated L1 err; adjoint/fwd"
PEAK_FP64_VECTOR = 78.6e12       # FLOP/s, MI355X FP64 vector (FMA = 2 flops)
PEAK_HBM = 8.0e12                # B/s

# Algorithmic FP64 operations of one es_residual call per interior node (both
# directions of the 2D RHD ES scheme, p = 3): counted by executing the device
# arithmetic of the two-point flux and of the face dissipation with an
# op-counting scalar (paper_2107_12027_amd/csrc/opcount.cpp, run by
# `python -m paper_2107_12027_amd.build --opcount`): + - * / sqrt log exp fabs
# fmax count 1, fma counts 2.  Per node and direction: 3 two-point fluxes
# (102.3 each), 1 face dissipation (1494.7), state preparation (6) and the
# flux-difference accumulation (66): 1873.7; two directions: 3747.5.
RESIDUAL_FLOPS_PER_NODE_2D_RHD = 3747.5

# HBM bytes of one es_residual call on the 400 x 400 quadrant workload, from the
# FETCH_SIZE and WRITE_SIZE counters (rocprofv3 --pmc, one counter per run) of
# k_residual_rhd and k_sum_dirs, scaled by what the same counters read for a
# 1 GiB device copy (FETCH x 2.000, WRITE x 1.000); the summary with its commands
# is profiles/es_residual_hbm_counters_rhd2d_quadrant_400.txt.  Valid for the
# kernels as they were measured; None for other workloads.
RESIDUAL_TRAFFIC_BYTES_QUADRANT_400 = 57.73e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=400)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--residual-reps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--workload", default="quadrant",
                    choices=["quadrant", "sine", "rotor", "blast3d", "fourier"],
                    help="quadrant: the headline 2D RHD problem; the others time the remaining "
                         "workloads (FP64 step and residual only)")
    ap.add_argument("--paper-case", default=None,
                    choices=["rp1", "rp2", "rp3", "rmhd_blast", "shock_cloud", "vortex2d", "vortex3d"],
                    help="run one of the paper's 2D examples to its end time as MM-O5 (adaptive) and "
                         "UM-O5 (uniform, finer) and report the GPU time-to-solution ratio beside the "
                         "paper's CPU ratio; vortex2d / vortex3d: errors and orders of MM-O6 and MM-O5 "
                         "on the RMHD vortex (not headline lines)")
    ap.add_argument("--vortex-n", default=None,
                    help="mesh sizes N of the vortex study (2D: N x N, default 20,40,80,160; "
                         "3D: N x N x 5N, default 16,24,32,48,64)")
    ap.add_argument("--no-fourier-gradient", action="store_true",
                    help="skip the gradient study of the adjoint configuration (objects adjoint_fourier*)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed work, copy one buffer of this size once (a plain copy "
                         "kernel of known traffic, for scaling HBM counters)")
    return ap.parse_args()


def cpu_baseline(n, seed):
    """The oracle as it stands, timed on the host for one RK3 step of the same
    workload; also returns the oracle's state after that step."""
    from oracle import physics as ph, stepper as st
    from paper_2107_12027_amd import workloads as wl
    w = wl.quadrant_riemann(n=n, seed=seed)
    P = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
    U, J = st.initial_state(w.grid, w.scheme, P, w.x)
    t0 = time.perf_counter()
    out = st.rk3_step(w.grid, w.scheme, w.monitor, U, J, w.x)
    t = time.perf_counter() - t0
    if not out["ok"].all():
        return None, None
    return ({"value": w.grid.nnodes / t, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
             "sample": "one SSP-RK3 step of the full %dx%d workload from its initial state "
                       "(numpy oracle, %.1f s)" % (n, n, t)}, out["U"])


def l1_rel(a, b):
    import numpy as np
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return [float(v) for v in np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)]


class Run:
    """One context and its device state for the workload, from the initial data."""

    def __init__(self, w, mixed):
        import dataclasses
        import numpy as np
        import torch
        from paper_2107_12027_amd import es
        self.w = w
        scheme = dataclasses.replace(w.scheme, mixed=mixed)
        self.ctx = ctx = es.Context(w.grid, scheme, w.monitor)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
        P = np.concatenate([w.prim["rho"][None], w.prim["u"], w.prim["p"][None], w.prim["B"]])
        if w.scheme.phys == 1:
            sel = list(range(8))
        else:
            sel = [0, 1, 2, 4] if w.grid.dim == 2 else [0, 1, 2, 3, 4]
        self.met = torch.empty((ctx.nmet,) + ctx.padded_shape(), dtype=torch.float64, device="cuda")
        self.prim = torch.empty((ctx.nprim,) + ctx.padded_shape(), dtype=torch.float64, device="cuda")
        self.J = torch.empty(ctx.shape(), dtype=torch.float64, device="cuda")
        self.x = dev(w.x)
        ctx.metrics(self.x, None, self.met, self.J)
        self.U = torch.empty((ctx.m,) + ctx.shape(), dtype=torch.float64, device="cuda")
        ctx.prim2con(dev(P[sel]), self.J, self.U)
        self.xdot = torch.empty_like(self.x)
        self.dt = torch.empty(1, dtype=torch.float64, device="cuda")

    def step(self):
        self.ctx.rk3_step(self.U, self.J, self.x, self.xdot, self.dt)

    def timed(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        st0 = self.ctx.status()[0]
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            self.step()
        e1.record(stream)
        torch.cuda.synchronize()
        status, nfail, first = self.ctx.status()
        if st0 != 0 or status != 0:
            print("bench.py: con2prim failure during the run (status %d, %d nodes, first %d)"
                  % (status, nfail, first), file=sys.stderr)
            sys.exit(3)
        return e0.elapsed_time(e1)

    def residual_ms(self, reps):
        """Average es_residual time on the current state (HIP events on the launch stream)."""
        import torch
        ctx = self.ctx
        dU = torch.empty_like(self.U)
        dJ = torch.empty_like(self.J)
        ctx.con2prim(self.U, self.J, self.prim)
        ctx.metrics(self.x, self.xdot, self.met)
        ctx.residual(self.prim, self.met, dU, dJ)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        r0 = torch.cuda.Event(enable_timing=True)
        r1 = torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for _ in range(reps):
            ctx.residual(self.prim, self.met, dU, dJ)
        r1.record(stream)
        torch.cuda.synchronize()
        return r0.elapsed_time(r1) / reps


def adjoint_timing(w, steps, fwd_ms):
    """Forward steps with checkpoints, then their vector-Jacobian products in
    reverse order (es_rk3_step_save / es_rk3_step_vjp), timed with HIP events."""
    import torch
    if steps <= 0:
        return None
    run = Run(w, 0)
    ctx = run.ctx
    ck = [torch.empty(ctx.ckpt_doubles(), dtype=torch.float64, device="cuda") for _ in range(steps)]
    lamU = torch.ones_like(run.U)
    lamJ = torch.zeros_like(run.J)
    gU = torch.empty_like(run.U)
    gJ = torch.empty_like(run.J)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        ctx.rk3_step_save(run.U, run.J, run.x, run.xdot, run.dt, ck[k])
    ev[1].record(stream)
    for k in reversed(range(steps)):
        ctx.rk3_step_vjp(ck[k], lamU, lamJ, gU, gJ)
        lamU, gU = gU, lamU
        lamJ, gJ = gJ, lamJ
    ev[2].record(stream)
    torch.cuda.synchronize()
    if ctx.status()[0] != 0 or not bool(torch.isfinite(lamU).all()):
        return None
    save_ms = ev[0].elapsed_time(ev[1]) / steps
    vjp_ms = ev[1].elapsed_time(ev[2]) / steps
    return {"steps": steps, "forward_ms_per_step": fwd_ms, "forward_with_checkpoint_ms_per_step": save_ms,
            "vjp_ms_per_step": vjp_ms, "adjoint_over_forward": vjp_ms / fwd_ms,
            "note": "VJP of es_rk3_step with the mesh trajectory and dt held fixed; FP64"}


def fourier_gradient(n=256, steps=100, h=1e-6, eps=0.05, rmhd=True):
    """Gradient of L = integral of rho^2 over [0.4,0.6]^2 after `steps` steps with
    respect to the 8 density-mode coefficients of the Fourier-mode workload (the
    adjoint configuration: 2D RMHD; rmhd=False: its RHD counterpart; static
    periodic mesh, the time step fixed at the CFL step of the initial state):
    forward with per-step checkpoints, the adjoint chain in reverse, and central
    differences of the forward (h) for every coefficient.  Timed with HIP events
    (forward with checkpoints, reverse)."""
    import numpy as np
    import torch
    from paper_2107_12027_amd import es, losses, workloads as wl
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    _, _, c0 = wl.fourier_modes(0)
    make = wl.rmhd_fourier if rmhd else wl.rhd_fourier

    def start(c):
        w = make(n=n, coeffs=c)
        run = Run(w, 0)
        xs = w.x
        inside = (xs[0] >= 0.4) & (xs[0] <= 0.6) & (xs[1] >= 0.4) & (xs[1] <= 0.6)
        return w, run, dev(inside * (1.0 / (n * n)))

    w, run, weight = start(c0)
    ctx = run.ctx
    ctx.cfl(*_cfl_inputs(run), run.dt)
    fixed = run.dt.clone()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ck = [torch.empty(ctx.ckpt_doubles(), dtype=torch.float64, device="cuda") for _ in range(steps)]
    J0 = run.J.clone()
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        ctx.rk3_step_save(run.U, run.J, run.x, run.xdot, run.dt, ck[k], fixed)
    ev[1].record(stream)
    L, gU, gJ = losses.density_squared(ctx, run.U, run.J, weight)
    ev[2].record(stream)
    oU, oJ = torch.empty_like(gU), torch.empty_like(gJ)
    for k in reversed(range(steps)):
        ctx.rk3_step_vjp(ck[k], gU, gJ, oU, oJ)
        gU, oU = oU, gU
        gJ, oJ = oJ, gJ
    ev[3].record(stream)
    torch.cuda.synchronize()
    if rmhd:
        P0 = dev(np.concatenate([w.prim["rho"][None], w.prim["u"], w.prim["p"][None], w.prim["B"]]))
    else:
        P0 = dev(np.stack([w.prim["rho"], w.prim["u"][0], w.prim["u"][1], w.prim["p"]]))
    tang = losses.density_mode_tangents(ctx, P0, J0, dev(wl.fourier_basis(w.x)), eps)
    grad = (tang * gU[None]).sum(dim=(1, 2, 3)).cpu().numpy()
    del ck

    def loss(c):
        _, r, wt = start(c)
        for _ in range(steps):
            r.ctx.rk3_step(r.U, r.J, r.x, r.xdot, r.dt, fixed)
        return float(losses.density_squared(r.ctx, r.U, r.J, wt)[0])

    fd = np.array([(loss(c0 + h * e) - loss(c0 - h * e)) / (2 * h) for e in np.eye(8)])
    fwd_ms = ev[0].elapsed_time(ev[1]) / steps
    rev_ms = ev[2].elapsed_time(ev[3]) / steps
    return {"workload": w.name + ("" if rmhd else " (RHD counterpart of the RMHD configuration)"),
            "steps": steps, "loss": float(L), "grad": grad.tolist(), "fd_grad": fd.tolist(), "fd_h": h,
            "max_rel_diff_vs_fd": float(np.max(np.abs(grad - fd)) / np.max(np.abs(fd))),
            "forward_with_checkpoint_ms_per_step": fwd_ms, "vjp_ms_per_step": rev_ms,
            "adjoint_over_forward": rev_ms / fwd_ms,
            "note": "static mesh, dt fixed at the CFL step of the initial state; FP64" +
                    ("; the adjoint holds the face eigen-structure of the ES dissipation" if rmhd else "")}


def _cfl_inputs(run):
    """prim, met, J of the run's current state for es_cfl."""
    run.ctx.con2prim(run.U, run.J, run.prim)
    run.ctx.metrics(run.x, None, run.met)
    return run.prim, run.met, run.J


RESIDUAL_FLOPS_PER_NODE_3D_RHD = 8313.0   # same count, 3 directions (2771.0 each)


def other_workload(args):
    """Time one of the other workloads: RK3 steps and es_residual, FP64 and
    FP32-mixed."""
    import numpy as np
    from paper_2107_12027_amd import workloads as wl
    make = {"sine": lambda: wl.advected_sine(n=64),
            "rotor": lambda: wl.rmhd_rotor(n=512),
            "blast3d": lambda: wl.blast3d(n=128, seed=0),
            "fourier": lambda: wl.rmhd_fourier(n=256, seed=0)}[args.workload]
    w = make()
    run = Run(w, 0)
    t_ms = run.timed(args.steps, args.warmup)
    res_ms = run.residual_ms(args.residual_reps)
    # the FP32-mixed form over the same steps from the same initial data, and the
    # relative L1 difference of the final states (per conserved component)
    mrun = Run(w, 1)
    t_mixed_ms = mrun.timed(args.steps, args.warmup)
    res_mixed_ms = mrun.residual_ms(args.residual_reps)
    a, b = mrun.U.cpu().numpy(), run.U.cpu().numpy()
    a, b = a.reshape(a.shape[0], -1), b.reshape(b.shape[0], -1)
    den = np.maximum(np.abs(b).sum(axis=1), 1e-300)
    mixed = {"ms_per_step": t_mixed_ms / args.steps, "es_residual_ms": res_mixed_ms,
             "speedup_vs_fp64": t_ms / t_mixed_ms,
             "l1_rel_diff_vs_fp64": (np.abs(a - b).sum(axis=1) / den).tolist(),
             "diff_sample": "final states after the %d warm-up and %d timed steps of both forms"
                            % (args.warmup, args.steps)}
    nodes = w.grid.nnodes
    flops = None
    if w.scheme.phys == 0:
        flops = RESIDUAL_FLOPS_PER_NODE_2D_RHD if w.grid.dim == 2 else RESIDUAL_FLOPS_PER_NODE_3D_RHD
    roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": None, "traffic": None, "kernel": "es_residual", "avg_launch_ms": res_ms}
    if flops is not None:
        ach = flops * nodes / (res_ms * 1e-3)
        roof["achieved"] = ach / 1e12
        roof["frac"] = ach / PEAK_FP64_VECTOR
    line = {"metric": METRIC, "value": nodes * args.steps / (t_ms * 1e-3), "unit": "cell-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_ms / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": w.name, "system": ("RMHD" if w.scheme.phys else "RHD") + " %dD" % w.grid.dim,
                       "grid": list(w.grid.shape[::-1]), "nodes": nodes,
                       "mesh": "adaptive" if w.monitor.enabled else "static", "precision": "FP64"},
            "roofline": roof, "cpu_baseline": None, "mixed": mixed}
    print(json.dumps(line))


def run_to_end(w, check_every=32, max_wall_s=240.0):
    """Advance ``w`` with es_rk3_step until t >= t_end (the last step is not
    clipped); dt is summed on the device and read back every ``check_every``
    steps, then every step once t_end is within reach.  Returns a dict with the
    wall time (host clock, from initial data resident in HBM to the final
    synchronisation), the GPU time between HIP events, the step count and t
    (a run that exceeds max_wall_s stops early and reports t < t_end)."""
    import torch
    run = Run(w, 0)
    tsum = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx = run.ctx
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    steps, t, dt_last, every = 0, 0.0, None, check_every
    status, nfail = 0, 0
    while t < w.t_end:
        for _ in range(every):
            run.step()
            tsum.add_(run.dt)
        steps += every
        t_new = float(tsum.item())
        dt_last = (t_new - t) / every
        t = t_new
        # (es_ctx_status reports and clears the failures since its last call)
        status, nfail, _ = ctx.status()
        if status != 0 or time.perf_counter() - t_wall > max_wall_s:
            break
        if t + check_every * dt_last >= w.t_end:
            every = 1
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    return {"workload": w.name, "grid": list(w.grid.shape[::-1]), "steps": steps, "t": t,
            "wall_s": wall, "gpu_s": e0.elapsed_time(e1) * 1e-3, "status": int(status),
            "failed_nodes": int(nfail), "ms_per_step": e0.elapsed_time(e1) / max(steps, 1)}


def paper_case(args):
    """MM-O5 vs UM-O5 time to solution for one of the paper's 2D examples."""
    from paper_2107_12027_amd import workloads as wl
    make, n_mm, n_um, paper_ratio = wl.PAPER_COMPARISONS[args.paper_case]
    mm = run_to_end(make(n_mm, True))
    um = run_to_end(make(n_um, False))
    um_same = run_to_end(make(n_mm, False))     # the moving-mesh overhead at equal resolution
    ok = mm["status"] == 0 and um["status"] == 0
    line = {"paper_case": args.paper_case, "t_end": make(n_mm, True).t_end, "mm_o5": mm, "um_o5": um,
            "um_o5_same_grid": um_same,
            "gpu_time_ratio_mm_over_um": mm["gpu_s"] / um["gpu_s"] if ok else None,
            "wall_time_ratio_mm_over_um": mm["wall_s"] / um["wall_s"] if ok else None,
            "paper_cpu_time_ratio": paper_ratio, "dtype": "f64", "data": "synthetic (the paper's initial data)"}
    print(json.dumps(line))


def vortex_run(dim, n, adaptive, max_wall_s=150.0):
    """The RMHD vortex of Section 6 (2D: N x N nodes to t = 4; 3D: N x N x 5N
    nodes to t = 0.1): MM-O6 (EC scheme, prescribed mesh, dt = CFL dxi^2) or MM-O5
    (ES scheme, adaptive mesh with the gradient + Laplacian monitor, dt = CFL
    dxi^(5/3)), dxi = 1/N the computational spacing, the step count rounded up so
    that the run ends at the end time.  Returns the L1 and max errors of rho
    against the closed form and the GPU time (HIP events)."""
    import math
    import numpy as np
    import torch
    from paper_2107_12027_amd import workloads as wl
    w = wl.rmhd_vortex(dim, n, 0.0, dissipation=int(adaptive), adaptive=adaptive)
    t_end = w.t_end
    run = Run(w, 0)
    ctx = run.ctx
    power = 5.0 / 3.0 if adaptive else 2.0
    steps = int(math.ceil(t_end / (w.scheme.cfl * (1.0 / n) ** power) - 1e-9))
    dt = t_end / steps
    fixed = torch.tensor([dt], dtype=torch.float64, device="cuda")
    shape = torch.from_numpy(wl.vortex_mesh_shape(w.grid)[1]).cuda()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    done = 0
    t_print = t_wall
    while done < steps:
        for k in range(done, min(steps, done + 256)):
            if adaptive:
                ctx.rk3_step(run.U, run.J, run.x, run.xdot, run.dt, fixed)
            else:
                da = wl.vortex_mesh_amplitude((k + 1) * dt) - wl.vortex_mesh_amplitude(k * dt)
                torch.mul(shape, da / dt, out=run.xdot)
                ctx.rk3_step_moving(run.U, run.J, run.x, run.xdot, run.dt, fixed)
        done = min(steps, done + 256)
        torch.cuda.synchronize()
        now = time.perf_counter()
        if now - t_print > 30.0:
            print("vortex%dd N=%d: %d of %d steps" % (dim, n, done, steps), file=sys.stderr, flush=True)
            t_print = now
        if now - t_wall > max_wall_s:
            break
    e1.record(stream)
    torch.cuda.synchronize()
    status, nfail, _ = ctx.status()
    out = {"n": n, "nodes": w.grid.nnodes, "steps": done, "dt": dt, "t": done * dt,
           "gpu_s": e0.elapsed_time(e1) * 1e-3, "wall_s": time.perf_counter() - t_wall, "status": int(status)}
    if status == 0 and done == steps:
        ctx.con2prim(run.U, run.J, run.prim)
        x = run.x.cpu().numpy()
        if dim == 2:
            rho = run.prim[0, 3:-3, 3:-3].cpu().numpy()
            exact = wl.vortex2d_state(x[0], x[1], t_end)[0]
        else:
            rho = run.prim[0, 3:-3, 3:-3, 3:-3].cpu().numpy()
            exact = wl.vortex3d_state(x[0], x[1], x[2], t_end)[0]
        out["l1_rho"] = float(np.mean(np.abs(rho - exact)))
        out["linf_rho"] = float(np.max(np.abs(rho - exact)))
    return out


def vortex_study(args, dim):
    """Errors and orders of MM-O6 and MM-O5 on the 2D or 3D RMHD vortex (Section 6)."""
    import math
    spec = args.vortex_n or ("20,40,80,160" if dim == 2 else "16,24,32,48,64")
    ns = [int(v) for v in spec.split(",")]
    name_case = "vortex%dd" % dim
    line = {"paper_case": name_case, "t_end": 4.0 if dim == 2 else 0.1, "dtype": "f64",
            "data": "synthetic (the paper's closed-form initial data)"}
    for name, adaptive in (("mm_o6", False), ("mm_o5", True)):
        runs = []
        for n in ns:
            r = vortex_run(dim, n, adaptive)
            runs.append(r)
            print("%s %s N=%d: %s" % (name_case, name, n, json.dumps(r)), file=sys.stderr, flush=True)
        rates = []
        for a, b in zip(runs[:-1], runs[1:]):
            ok = "l1_rho" in a and "l1_rho" in b
            rates.append(math.log(a["l1_rho"] / b["l1_rho"]) / math.log(b["n"] / a["n"]) if ok else None)
        line[name] = {"runs": runs, "rates_l1_rho": rates}
    print(json.dumps(line))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2107_12027_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.paper_case in ("vortex2d", "vortex3d"):
        return vortex_study(args, 2 if args.paper_case == "vortex2d" else 3)
    if args.paper_case is not None:
        return paper_case(args)
    if args.workload != "quadrant":
        return other_workload(args)
    w = wl.quadrant_riemann(n=args.n, seed=args.seed)
    g = w.grid

    # accuracy sample: one step from the initial data on both forms (compared with
    # the oracle's step below, outside every timed region)
    one_step = {}
    for mixed in (0, 1):
        r = Run(w, mixed)
        r.step()
        torch.cuda.synchronize()
        if r.ctx.status()[0] != 0:
            print("bench.py: con2prim failure in the first step", file=sys.stderr)
            sys.exit(3)
        one_step[mixed] = r.U.cpu().numpy()
        del r

    run = Run(w, 0)
    t_ms = run.timed(args.steps, args.warmup)
    res_ms = run.residual_ms(args.residual_reps)
    mrun = Run(w, 1)
    t_mixed_ms = mrun.timed(args.steps, args.warmup)
    res_mixed_ms = mrun.residual_ms(args.residual_reps)
    adjoint = adjoint_timing(w, args.adjoint_steps, t_ms / args.steps)
    study = args.adjoint_steps > 0 and not args.no_fourier_gradient
    adjoint_fourier = fourier_gradient(rmhd=True) if study else None
    adjoint_fourier_rhd = fourier_gradient(rmhd=False) if study else None

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    nodes = g.nnodes
    value = nodes * args.steps / (t_ms * 1e-3)
    flops = RESIDUAL_FLOPS_PER_NODE_2D_RHD
    traffic = RESIDUAL_TRAFFIC_BYTES_QUADRANT_400 if (args.n, args.seed) == (400, 2) else None
    roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": None, "traffic": traffic, "traffic_unit": "HBM bytes per es_residual call",
            "kernel": "es_residual (k_residual_rhd, both sweeps in one launch, + k_sum_dirs)",
            "avg_launch_ms": res_ms}
    if flops is not None:
        ach = flops * nodes / (res_ms * 1e-3)
        roof["achieved"] = ach / 1e12
        roof["frac"] = ach / PEAK_FP64_VECTOR
    if traffic is not None:
        # the HBM side of the same call: counter bytes over the measured duration
        roof["hbm_achieved_gbs"] = traffic / (res_ms * 1e-3) / 1e9
        roof["hbm_frac"] = traffic / (res_ms * 1e-3) / PEAK_HBM
    cpu = None
    mixed = {"value": nodes * args.steps / (t_mixed_ms * 1e-3), "unit": "cell-updates/s",
             "ms_per_step": t_mixed_ms / args.steps, "dtype": "f32 pair/dissipation, f64 elsewhere",
             "es_residual_ms": res_mixed_ms, "speedup_vs_fp64": t_ms / t_mixed_ms,
             "l1_rel_err_vs_oracle": None, "fp64_l1_rel_err_vs_oracle": None,
             "err_sample": "one SSP-RK3 step of the %dx%d workload from its initial state, "
                           "relative L1 per conserved component" % (args.n, args.n)}
    if not args.no_cpu_baseline:
        cpu, Uo = cpu_baseline(args.n, args.seed)
        if Uo is not None:
            mixed["l1_rel_err_vs_oracle"] = l1_rel(one_step[1], Uo)
            mixed["fp64_l1_rel_err_vs_oracle"] = l1_rel(one_step[0], Uo)
    line = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "system": "2D RHD, Gamma 5/3", "grid": [args.n, args.n],
                   "nodes": nodes, "scheme": "ES: 6th-order EC flux + WENO5 dissipation, SSP-RK3, CFL 0.4",
                   "mesh": "adaptive, monitor alpha 1200 on ln rho, 3 filter passes, 10 Jacobi sweeps",
                   "boundary": "outflow", "precision": "FP64"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "adjoint": adjoint,
        "adjoint_fourier": adjoint_fourier,
        "adjoint_fourier_rhd": adjoint_fourier_rhd,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
