#!/usr/bin/env python3
"""Benchmark: cell-updates/s of one SSP-RK3 step of the entropy-stable adaptive
moving-mesh scheme on one MI355X.

Headline workload (default): 3D RHD blast wave, 128^3 nodes on [0,1]^3,
outflow, adaptive mesh (paper monitor on rho, alpha 800, 3 filter passes, 5
Jacobi sweeps), CFL 0.3, seed 0, 100 RK3 steps, FP64 -- the largest
single-GPU workload of the set.  One step = the whole hot path: con2prim, CFL
step, mesh redistribution (monitor, filter, Jacobi sweeps, Delta_tau, new mesh
and mesh velocity) and three Runge-Kutta stages of metrics + con2prim +
residual + combination.  Inputs are resident in HBM before the timed region;
the time step stays on the device (no host synchronisation inside the timed
steps).  The W warm-up steps run first; the state is then reset to the initial
data and exactly K steps are timed, so with the default K = 100 the timed run
is the workload's 100 steps.

The same K steps are timed in the FP32-mixed form (scheme.mixed = 1) and the
relative L1 difference of the final states (mixed vs FP64) is reported per
conserved component under "mixed".  "cpu_baseline" is the oracle (numpy,
limited to one thread) timed on one step of the same blast recipe at a small
size (40^3 by default); the GPU FP64 and mixed steps of that sample are compared
with the oracle's step.  The other workloads (advected sine, quadrant seeds 0-3,
RMHD rotor, the RMHD adjoint configuration) are reported as extra objects.

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

# Algorithmic FP64 operations of one es_residual call per interior node: counted
# by executing the device arithmetic of the two-point flux and of the face
# dissipation with an op-counting scalar (paper_2107_12027_amd/csrc/opcount.cpp,
# run by `python -m paper_2107_12027_amd.build --opcount`): + - * / sqrt log exp
# fabs fmax count 1, fma counts 2.  2D RHD ES, p = 3, per node and direction: 3
# two-point fluxes (102.3 each), 1 face dissipation (1494.7), state preparation
# (6) and the flux-difference accumulation (66): 1873.7; two directions: 3747.5.
# 3D RHD ES: 2771.0 per direction, 8313.0 for the three.  RMHD ES, p = 3 (the
# numeric face eigen-structure dominates: about 35,400 per face; averaged over
# smooth states with well-separated eigenvalues): 73914.1 per node in 2D, 111738.6
# in 3D.
RESIDUAL_FLOPS_PER_NODE_2D_RHD = 3747.5
RESIDUAL_FLOPS_PER_NODE_3D_RHD = 8313.0
RESIDUAL_FLOPS_PER_NODE_2D_RMHD = 73914.1
RESIDUAL_FLOPS_PER_NODE_3D_RMHD = 111738.6

# HBM bytes of one es_residual call, from the FETCH_SIZE and WRITE_SIZE counters
# (rocprofv3 --pmc, one counter per run) of the residual kernel and k_sum_dirs,
# scaled by what the same counters read for a 1 GiB device copy (FETCH x 2.000,
# WRITE x 1.000).  Valid for the kernels as they were measured; the summaries
# with their commands are the es_residual_hbm_counters_* files under profiles/.
RESIDUAL_TRAFFIC_BYTES = {
    "rhd2d_quadrant_riemann_400_seed2": 57.85e6,
    "rhd3d_blast_128": 1329.3e6,
    "rmhd2d_rotor_512": 1483.2e6,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None,
                    help="grid size of the workload (default: 128 for the 3D blast, 400 for the quadrant)")
    ap.add_argument("--seed", type=int, default=None,
                    help="seed of the workload (default: 0 for the 3D blast, 2 for the quadrant)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=40,
                    help="size n^3 of the blast sample the oracle is timed on (cpu_baseline)")
    ap.add_argument("--residual-reps", type=int, default=20)
    ap.add_argument("--adjoint-steps", type=int, default=10)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra objects (advected sine, quadrant seeds, rotor, adjoint configuration)")
    ap.add_argument("--workload", default="blast3d",
                    choices=["blast3d", "quadrant", "sine", "rotor", "fourier"],
                    help="blast3d: the headline 3D RHD blast; the others time one of the remaining "
                         "workloads alone (FP64 and mixed step, residual)")
    ap.add_argument("--paper-case", default=None,
                    choices=["rp1", "rp2", "rp3", "rmhd_blast", "shock_cloud", "vortex2d", "vortex3d"],
                    help="run one of the paper's 2D examples to its end time as MM-O5 (adaptive) and "
                         "UM-O5 (uniform, finer) and report the GPU time-to-solution ratio beside the "
                         "paper's CPU ratio; vortex2d / vortex3d: errors and orders of MM-O6 and MM-O5 "
                         "on the RMHD vortex (not headline lines)")
    ap.add_argument("--vortex-n", default=None,
                    help="mesh sizes N of the vortex study (2D: N x N, default 20,40,80,160; "
                         "3D: N x N x 5N, default 16,24,32,48,64)")
    ap.add_argument("--vortex-sweeps", type=int, default=None,
                    help="Jacobi sweeps mu of the MM-O5 mesh redistribution in the vortex study "
                         "(default: the example's 10)")
    ap.add_argument("--vortex-schemes", default="mm_o6,mm_o5",
                    help="schemes of the vortex study, from mm_o6 and mm_o5")
    ap.add_argument("--no-fourier-gradient", action="store_true",
                    help="skip the gradient study of the adjoint configuration (object c5_adjoint)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed work, copy one buffer of this size once (a plain copy "
                         "kernel of known traffic, for scaling HBM counters)")
    return ap.parse_args()


def oracle_step(w):
    """One RK3 step of workload ``w`` by the oracle as it stands (numpy, BLAS and
    OpenMP pools limited to one thread), timed on the host.  Returns (seconds,
    Ucurv after the step or None if con2prim failed)."""
    from threadpoolctl import threadpool_limits
    from oracle import physics as ph, stepper as st
    P = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
    with threadpool_limits(limits=1):
        U, J = st.initial_state(w.grid, w.scheme, P, w.x)
        t0 = time.perf_counter()
        out = st.rk3_step(w.grid, w.scheme, w.monitor, U, J, w.x)
        t = time.perf_counter() - t0
    return t, (out["U"] if out["ok"].all() else None)


def cpu_baseline(w):
    """cpu_baseline object: the oracle timed on one step of the sample workload."""
    t, Uo = oracle_step(w)
    shape = "x".join(str(s) for s in w.grid.shape[::-1])
    cpu = {"value": w.grid.nnodes / t, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
           "host_cpus": os.cpu_count(),
           "sample": "one SSP-RK3 step of %s (%s nodes, the headline recipe at a smaller size) from its "
                     "initial state: numpy oracle limited to one thread, %.1f s" % (w.name, shape, t)}
    return cpu, Uo


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
        self.init = (self.U.clone(), self.J.clone(), self.x.clone())

    def reset(self):
        """Back to the initial data (same tensors, so a captured step graph stays valid)."""
        U0, J0, x0 = self.init
        self.U.copy_(U0)
        self.J.copy_(J0)
        self.x.copy_(x0)

    def step(self):
        self.ctx.rk3_step(self.U, self.J, self.x, self.xdot, self.dt)

    def timed(self, steps, warmup, reset=True):
        """W warm-up steps, then (reset=True) back to the initial data, then K timed
        steps between HIP events on the current stream.  Returns (GPU ms for the K
        steps, host wall seconds of the same region)."""
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        st0, nf0, ff0 = self.ctx.status()
        if st0 != 0:
            print("bench.py: failure in the warm-up steps (status %d, %d nodes, first %d)" % (st0, nf0, ff0),
                  file=sys.stderr)
            sys.exit(3)
        if reset:
            self.reset()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            self.step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        status, nfail, first = self.ctx.status()
        if status != 0:
            print("bench.py: failure during the timed steps (status %d, %d nodes, first %d)"
                  % (status, nfail, first), file=sys.stderr)
            sys.exit(3)
        return e0.elapsed_time(e1), wall

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
    grad = losses.density_mode_gradient(ctx, P0, J0, gU, dev(wl.fourier_basis(w.x)), eps).cpu().numpy()
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


def residual_flops(w):
    """Algorithmic FP64 ops of one es_residual call per interior node (ES, p = 3)."""
    if w.scheme.order_p != 3 or w.scheme.dissipation != 1:
        return None
    if w.scheme.phys == 1:
        return RESIDUAL_FLOPS_PER_NODE_2D_RMHD if w.grid.dim == 2 else RESIDUAL_FLOPS_PER_NODE_3D_RMHD
    return RESIDUAL_FLOPS_PER_NODE_2D_RHD if w.grid.dim == 2 else RESIDUAL_FLOPS_PER_NODE_3D_RHD


def l1_rel_diff(a, b):
    """Relative L1 difference per component of two (comps, ...) arrays: sum|a - b| / sum|b|
    (components with sum|b| = 0 report the absolute mean difference)."""
    import numpy as np
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    den = np.abs(b).sum(axis=1)
    num = np.abs(a - b).sum(axis=1)
    return [float(n / d) if d > 0 else float(n / a.shape[1]) for n, d in zip(num, den)]


def fp64_and_mixed(w, steps, warmup, reps):
    """K timed steps of workload ``w`` in the FP64 and the FP32-mixed forms from the
    same initial data, es_residual timing on the FP64 run's final state, and the
    relative L1 difference of the two final states per conserved component."""
    run = Run(w, 0)
    t_ms, wall = run.timed(steps, warmup)
    res_ms = run.residual_ms(reps)
    mrun = Run(w, 1)
    t_mixed_ms, _ = mrun.timed(steps, warmup)
    res_mixed_ms = mrun.residual_ms(reps)
    diff = l1_rel_diff(mrun.U.cpu().numpy(), run.U.cpu().numpy())
    nodes = w.grid.nnodes
    mixed = {"value": nodes * steps / (t_mixed_ms * 1e-3), "unit": "cell-updates/s",
             "ms_per_step": t_mixed_ms / steps, "es_residual_ms": res_mixed_ms,
             "speedup_vs_fp64": t_ms / t_mixed_ms,
             "dtype": "f32 pair algebra and dissipation, f64 elsewhere",
             "l1_rel_diff_vs_fp64": diff,
             "diff_sample": "final conserved states (Ucurv components in order) after the same %d steps "
                            "from the initial data in both forms" % steps}
    flops = residual_flops(w)
    roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": None, "traffic": RESIDUAL_TRAFFIC_BYTES.get(w.name),
            "traffic_unit": "HBM bytes per es_residual call",
            "kernel": "es_residual (the residual kernel, all directions in one launch, + k_sum_dirs)",
            "avg_launch_ms": res_ms, "flops_per_node": flops}
    if flops is not None:
        ach = flops * nodes / (res_ms * 1e-3)
        roof["achieved"] = ach / 1e12
        roof["frac"] = ach / PEAK_FP64_VECTOR
    if roof["traffic"] is not None:
        roof["hbm_achieved_gbs"] = roof["traffic"] / (res_ms * 1e-3) / 1e9
        roof["hbm_frac"] = roof["traffic"] / (res_ms * 1e-3) / PEAK_HBM
    return {"t_ms": t_ms, "wall_s": wall, "res_ms": res_ms, "mixed": mixed, "roofline": roof, "run": run}


def describe(w):
    g, s, m = w.grid, w.scheme, w.monitor
    cfg = {"workload": w.name, "system": "%dD %s, Gamma %.4g" % (g.dim, "RMHD" if s.phys else "RHD", s.gamma),
           "grid": list(g.shape[::-1]), "nodes": g.nnodes,
           "scheme": "%s: %d-th order EC flux%s, SSP-RK3, CFL %.2g" % (
               "ES" if s.dissipation else "EC", 2 * s.order_p,
               " + WENO%d dissipation" % (2 * s.order_p - 1) if s.dissipation else "", s.cfl),
           "boundary": "periodic" if g.bc[0] == 0 else "outflow", "precision": "FP64"}
    if m.enabled:
        cfg["mesh"] = "adaptive: monitor form %d, alpha %g on %s, %d filter passes, %d Jacobi sweeps" % (
            m.form, m.alpha, "ln rho" if m.sigma == 1 else "rho", m.filter_passes, m.sweeps)
    else:
        cfg["mesh"] = "static"
    return cfg


def other_workload(args):
    """Time one workload alone: RK3 steps and es_residual, FP64 and FP32-mixed."""
    from paper_2107_12027_amd import workloads as wl
    make = {"sine": lambda: wl.advected_sine(n=args.n or 64),
            "quadrant": lambda: wl.quadrant_riemann(n=args.n or 400, seed=2 if args.seed is None else args.seed),
            "rotor": lambda: wl.rmhd_rotor(n=args.n or 512),
            "fourier": lambda: wl.rmhd_fourier(n=args.n or 256, seed=0)}[args.workload]
    w = make()
    r = fp64_and_mixed(w, args.steps, args.warmup, args.residual_reps)
    nodes = w.grid.nnodes
    line = {"metric": METRIC, "value": nodes * args.steps / (r["t_ms"] * 1e-3), "unit": "cell-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["t_ms"] / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": describe(w), "roofline": r["roofline"], "cpu_baseline": None,
            "mixed": r["mixed"]}
    print(json.dumps(line))


def c1_sine(n=64):
    """Advected sine (64^2, adaptive mesh) run to t = 0.2, the last step shortened
    to end there; L1 error of rho against the exact advected profile
    rho = 1 + 0.2 sin 2pi(x + y - 0.4 t) at the final mesh nodes."""
    import numpy as np
    import torch
    from paper_2107_12027_amd import workloads as wl
    w = wl.advected_sine(n=n)
    run = Run(w, 0)
    ctx = run.ctx
    t_sum = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    steps, t = 0, 0.0
    while True:
        # steps of the scheme's own dt while at least 2 more fit, checked every 8 steps
        for _ in range(8):
            run.step()
            t_sum.add_(run.dt)
        steps += 8
        t = float(t_sum.item())
        if t + 16 * float(run.dt.item()) >= w.t_end:
            break
    while True:
        ctx.cfl(*_cfl_inputs(run), run.dt)
        dt = float(run.dt.item())
        last = t + dt >= w.t_end
        fixed = torch.tensor([w.t_end - t if last else dt], dtype=torch.float64, device="cuda")
        run.ctx.rk3_step(run.U, run.J, run.x, run.xdot, run.dt, fixed)
        t += float(fixed.item())
        steps += 1
        if last:
            break
    e1.record(stream)
    torch.cuda.synchronize()
    status = ctx.status()[0]
    ctx.con2prim(run.U, run.J, run.prim)
    x = run.x.cpu().numpy()
    rho = run.prim[0, 3:-3, 3:-3].cpu().numpy()
    exact = 1.0 + 0.2 * np.sin(2 * np.pi * (x[0] + x[1] - 0.4 * t))
    return {"workload": w.name, "t": t, "steps": steps, "status": int(status),
            "ms_per_step": e0.elapsed_time(e1) / steps,
            "value": w.grid.nnodes * steps / (e0.elapsed_time(e1) * 1e-3), "unit": "cell-updates/s",
            "l1_err_rho_vs_exact": float(np.mean(np.abs(rho - exact))),
            "linf_err_rho_vs_exact": float(np.max(np.abs(rho - exact))),
            "note": "FP64; the last step is shortened to end at t = 0.2 (its dt from es_cfl)"}


def c2_quadrant_seeds(n=400, steps=300, seeds=(0, 1, 2, 3), chunk=10):
    """The quadrant Riemann problem for seeds 0-3 (400^2, adaptive, 300 steps):
    per seed the outcome (con2prim status, checked every ``chunk`` steps) and the
    GPU time per step."""
    import torch
    from paper_2107_12027_amd import workloads as wl
    out = []
    for seed in seeds:
        w = wl.quadrant_riemann(n=n, seed=seed, steps=steps)
        run = Run(w, 0)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        done, status, first = 0, 0, -1
        while done < steps:
            k = min(chunk, steps - done)
            for _ in range(k):
                run.step()
            status, _, first = run.ctx.status()
            if status != 0:
                break
            done += k
        e1.record(stream)
        torch.cuda.synchronize()
        rec = {"seed": seed, "status": int(status), "steps_completed": done,
               "ms_per_step": e0.elapsed_time(e1) / max(done + (chunk if status else 0), 1)}
        if status == 0:
            rec["value"] = w.grid.nnodes * done / (e0.elapsed_time(e1) * 1e-3)
        else:
            rec["failed_between_steps"] = [done + 1, done + chunk]
            rec["first_failed_node"] = int(first)
        out.append(rec)
        del run
    return {"workload": "rhd2d_quadrant_riemann_%d" % n, "steps": steps, "seeds": out,
            "note": "FP64, status checked every %d steps (es_ctx_status synchronises); 0 = ok, "
                    "2 = inadmissible state reached con2prim" % chunk}


def c3_rotor(n=512, steps=200, warmup=2, reps=10):
    """RMHD rotor 512^2, 200 steps, FP64 and FP32-mixed."""
    from paper_2107_12027_amd import workloads as wl
    w = wl.rmhd_rotor(n=n, steps=steps)
    r = fp64_and_mixed(w, steps, warmup, reps)
    return {"workload": w.name, "steps": steps, "value": w.grid.nnodes * steps / (r["t_ms"] * 1e-3),
            "unit": "cell-updates/s", "ms_per_step": r["t_ms"] / steps, "es_residual_ms": r["res_ms"],
            "roofline": r["roofline"], "mixed": r["mixed"], "config": describe(w)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2107_12027_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        # a plain device copy of known size: the scale of the HBM counters
        m = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(m, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if args.paper_case in ("vortex2d", "vortex3d"):
        return vortex_study(args, 2 if args.paper_case == "vortex2d" else 3)
    if args.paper_case is not None:
        return paper_case(args)
    if args.workload != "blast3d":
        return other_workload(args)

    n = args.n or 128
    seed = 0 if args.seed is None else args.seed
    w = wl.blast3d(n=n, seed=seed)
    print("bench.py: %s, %d warm-up + %d timed steps, FP64 and mixed" % (w.name, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    r = fp64_and_mixed(w, args.steps, args.warmup, args.residual_reps)
    t_ms = r["t_ms"]
    nodes = w.grid.nnodes
    fwd_ms = t_ms / args.steps
    del r["run"]
    torch.cuda.empty_cache()
    print("bench.py: headline done (%.3f ms per step)" % fwd_ms, file=sys.stderr, flush=True)
    adjoint = adjoint_timing(w, args.adjoint_steps, fwd_ms)
    torch.cuda.empty_cache()

    extras = {}
    if not args.no_extras:
        for name, fn in (("c1_advected_sine", c1_sine), ("c2_quadrant_seeds", c2_quadrant_seeds),
                         ("c3_rotor", c3_rotor)):
            extras[name] = fn()
            torch.cuda.empty_cache()
            print("bench.py: %s done" % name, file=sys.stderr, flush=True)
        if args.adjoint_steps > 0 and not args.no_fourier_gradient:
            extras["c5_adjoint"] = fourier_gradient(rmhd=True)
            print("bench.py: c5_adjoint done", file=sys.stderr, flush=True)

    cpu = None
    mixed = r["mixed"]
    if not args.no_cpu_baseline:
        # the oracle on a sample of the same recipe, and the GPU forms' first step on it
        ws = wl.blast3d(n=args.cpu_n, seed=seed)
        one = {}
        for mx in (0, 1):
            rs_ = Run(ws, mx)
            rs_.step()
            torch.cuda.synchronize()
            one[mx] = rs_.U.cpu().numpy() if rs_.ctx.status()[0] == 0 else None
            del rs_
        cpu, Uo = cpu_baseline(ws)
        if Uo is not None and one[0] is not None and one[1] is not None:
            mixed["sample_l1_rel_err_vs_oracle"] = l1_rel_diff(one[1], Uo)
            mixed["sample_fp64_l1_rel_err_vs_oracle"] = l1_rel_diff(one[0], Uo)
            mixed["sample"] = "one step of %s from its initial data, GPU forms vs the oracle" % ws.name

    cfg = describe(w)
    cfg["seed"] = seed
    line = {
        "metric": METRIC, "value": nodes * args.steps / (t_ms * 1e-3), "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": fwd_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": cfg,
        "timed_wall_s": r["wall_s"],
        "roofline": r["roofline"],
        "cpu_baseline": cpu,
        "mixed": mixed,
        "adjoint": adjoint,
    }
    line.update(extras)
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


def vortex_run(dim, n, adaptive, max_wall_s=150.0, sweeps=None):
    """The RMHD vortex of Section 6 (2D: N x N nodes to t = 4; 3D: N x N x 5N
    nodes to t = 0.1): MM-O6 (EC scheme, prescribed mesh, dt = CFL dxi^2) or MM-O5
    (ES scheme, adaptive mesh with the gradient + Laplacian monitor, dt = CFL
    dxi^(5/3)), dxi = 1/N the computational spacing, the step count rounded up so
    that the run ends at the end time.  Returns the L1 and max errors of rho
    against the closed form and the GPU time (HIP events).  sweeps: the Jacobi
    sweep count of the adaptive redistribution instead of the example's."""
    import math
    import numpy as np
    import torch
    from paper_2107_12027_amd import workloads as wl
    w = wl.rmhd_vortex(dim, n, 0.0, dissipation=int(adaptive), adaptive=adaptive)
    if adaptive and sweeps is not None:
        w.monitor.sweeps = int(sweeps)
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
    if args.vortex_sweeps is not None:
        line["mm_o5_sweeps"] = args.vortex_sweeps
    for name, adaptive in (("mm_o6", False), ("mm_o5", True)):
        if name not in args.vortex_schemes.split(","):
            continue
        runs = []
        for n in ns:
            r = vortex_run(dim, n, adaptive, sweeps=args.vortex_sweeps)
            runs.append(r)
            print("%s %s N=%d: %s" % (name_case, name, n, json.dumps(r)), file=sys.stderr, flush=True)
        rates = []
        for a, b in zip(runs[:-1], runs[1:]):
            ok = "l1_rho" in a and "l1_rho" in b
            rates.append(math.log(a["l1_rho"] / b["l1_rho"]) / math.log(b["n"] / a["n"]) if ok else None)
        line[name] = {"runs": runs, "rates_l1_rho": rates}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
