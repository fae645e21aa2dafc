"""Helpers for the GPU parity tests: build seeded inputs, move them to the GPU,
call the C ABI through the binding, and compare with the oracle."""
import numpy as np
import torch

from oracle import physics as ph, metrics as mt, residual as rs, stepper as st
from paper_2107_12027_amd import es, workloads as wl


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty(*shape):
    return torch.empty(shape, dtype=torch.float64, device="cuda")


def rel_inf(a, b):
    """max |a - b| / max |b| per leading component."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    out = []
    for c in range(a.shape[0]):
        sc = np.max(np.abs(b[c]))
        out.append(np.max(np.abs(a[c] - b[c])) / (sc if sc > 0 else 1.0))
    return np.array(out)


def full_P(prim):
    return ph.full_prim(prim["rho"], prim["u"], prim["p"], prim["B"])


def prim_interior(P, phys, dim):
    return P[ph.comps(phys, dim)]


class Case:
    """A grid with a curvilinear (optionally moving) mesh and a primitive state."""

    def __init__(self, dim, n, bc, phys=ph.RHD, seed=0, smooth=False, amp=0.03, vmax=0.9,
                 moving=True, dissipation=1, monitor=None, rho_rng=(0.1, 1.0), p_rng=(0.1, 1.0),
                 mixed=0, uniform=False, p=3):
        rng = np.random.default_rng(seed)
        self.grid = wl.make_grid(dim, n, bc)
        self.x = wl.perturbed_mesh(self.grid, rng, amp=amp)
        self.xdot = (wl.perturbed_mesh(self.grid, rng, amp=0.05) - wl.uniform_mesh(self.grid)) if moving \
            else np.zeros_like(self.x)
        if uniform:
            pr = wl.random_prim((1,) * dim, rng, phys=phys, dim=dim, vmax=vmax)
            pr = {k: np.broadcast_to(v.reshape(v.shape[:v.ndim - dim] + (1,) * dim),
                                     v.shape[:v.ndim - dim] + self.grid.shape).copy()
                  for k, v in pr.items()}
        elif smooth:
            pr = wl.smooth_prim(self.x, rng, phys)
        else:
            pr = wl.random_prim(self.grid.shape, rng, phys=phys, dim=dim, vmax=vmax,
                                rho_rng=rho_rng, p_rng=p_rng)
        self.P = full_P(pr)
        self.scheme = wl.Scheme(phys=phys, dissipation=dissipation, mixed=mixed, order_p=p)
        self.monitor = monitor if monitor is not None else wl.Monitor(enabled=0)
        self.ctx = es.Context(self.grid, self.scheme, self.monitor)
        self.dim, self.phys = dim, phys
        self.m = self.ctx.m

    def oracle_state(self):
        J = mt.jacobian(self.grid, self.x, self.scheme.order_p)
        U = st.cons_from_prim(self.grid, self.scheme, self.P, J)
        return U, J

    def residual(self):
        """es_con2prim, es_metrics (with the mesh velocity) and es_residual on the GPU."""
        c = self.ctx
        U, J = self.gpu_state()
        prim = empty(c.nprim, *c.padded_shape())
        met = empty(c.nmet, *c.padded_shape())
        c.con2prim(U, J, prim)
        c.metrics(dev(self.x), dev(self.xdot), met)
        dU = empty(c.m, *c.shape())
        dJ = empty(*c.shape())
        c.residual(prim, met, dU, dJ)
        return U, J, prim, met, dU, dJ

    def oracle_residual(self):
        Uo, Jo = self.oracle_state()
        Po, _ = st.prim_from_cons(self.grid, self.scheme, Uo, Jo)
        meto = mt.metrics(self.grid, self.x, self.xdot, self.scheme.order_p)
        return rs.residual(self.grid, self.scheme, st.pad_solution(self.grid, Po, self.scheme.order_p), meto)

    def gpu_state(self):
        """J^0 by es_metrics and Ucurv by es_prim2con from the same primitive input."""
        c = self.ctx
        met = empty(c.nmet, *c.padded_shape())
        J = empty(*c.shape())
        c.metrics(dev(self.x), None, met, J)
        U = empty(c.m, *c.shape())
        c.prim2con(dev(prim_interior(self.P, self.phys, self.dim)), J, U)
        return U, J


def run_steps(w, nsteps, x0=None):
    """Run nsteps of es_rk3_step and of the oracle from the same workload."""
    g = w.grid
    ctx = es.Context(g, w.scheme, w.monitor)
    P = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
    x = w.x if x0 is None else x0
    met = empty(ctx.nmet, *ctx.padded_shape())
    J = empty(*ctx.shape())
    xg = dev(x)
    ctx.metrics(xg, None, met, J)
    U = empty(ctx.m, *ctx.shape())
    ctx.prim2con(dev(P[ph.comps(w.scheme.phys, g.dim)]), J, U)
    xdot = empty(g.dim, *ctx.shape())
    dt = empty(1)
    Uo, Jo = st.initial_state(g, w.scheme, P, x)
    xo = x.copy()
    for _ in range(nsteps):
        ctx.rk3_step(U, J, xg, xdot, dt)
        out = st.rk3_step(g, w.scheme, w.monitor, Uo, Jo, xo)
        Uo, Jo, xo = out["U"], out["J"], out["x"]
        assert abs(host(dt)[0] - out["dt"]) <= 1e-12 * out["dt"]
    assert ctx.status()[0] == es.ES_OK
    return (host(U), host(J), host(xg), host(xdot)), (Uo, Jo, xo, out["xdot"])
