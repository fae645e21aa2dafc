"""Parity at the configurations' full sizes through the C ABI.

The 2D configurations (quadrant Riemann problem 400^2 seed 2, RMHD rotor 512^2,
RMHD Fourier modes 256^2): es_metrics, es_prim2con, es_con2prim and the FP64 ES
es_residual on the initial data at full size, against the oracle on 4 x 4
windows sampled from the box (its corners, nodes along the discontinuities or the
disk edge, random ones), each window evaluated by the oracle from its own
full-size primitive and metric fields.

The 3D RHD blast workload (sphere r < 0.1 with p = 1000 in p = 1, rho = 1 with
1 % seeded noise, outflow, CFL 0.3):

* At its full size, 128^3 nodes, in the launch configuration the benchmark
  times: es_metrics, es_prim2con, es_con2prim and es_residual (FP64 ES, p = 3)
  on the initial data, against the oracle at sampled nodes.  A residual value
  depends only on its stencil, so the oracle evaluates it on small padded
  windows cut from its own full-size primitive and metric fields (computed from
  the workload's initial data, never from the GPU's).
* At 48^3, one whole adaptive RK3 step (con2prim, CFL, monitor, filter, Jacobi
  sweeps, limiter, three stages) element by element against the oracle's step.
"""
import numpy as np
import pytest

from gpu_util import dev, empty, host, rel_inf, run_steps
from oracle import metrics as mt
from oracle import physics as ph
from oracle import residual as rs
from oracle import stepper as st
from paper_2107_12027_amd import es, workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _sample_windows(n, rng, w=2, count=48):
    """Window origins (interior index of the first node along each axis): the eight
    corners of the box, nodes on the shell r ~ 0.1 where the pressure jumps, and
    random ones."""
    out = [(a, b, c) for a in (0, n - w) for b in (0, n - w) for c in (0, n - w)]
    centre = (n - 1) / 2.0
    r = 0.1 * (n - 1)
    while len(out) < count // 2:
        d = rng.normal(size=3)
        p = centre + r * d / np.linalg.norm(d)
        out.append(tuple(int(np.clip(round(v) - w // 2, 0, n - w)) for v in p))
    while len(out) < count:
        out.append(tuple(int(v) for v in rng.integers(0, n - w + 1, size=3)))
    return out


def test_blast3d_128_residual_at_sampled_nodes():
    wk = wl.blast3d(n=128, seed=0)
    g = wk.grid
    ctx = es.Context(g, wk.scheme, wk.monitor)
    P = ph.full_prim(wk.prim["rho"], wk.prim["u"], wk.prim["p"], wk.prim["B"])
    sel = ph.comps(wk.scheme.phys, g.dim)
    met = empty(ctx.nmet, *ctx.padded_shape())
    J = empty(*ctx.shape())
    ctx.metrics(dev(wk.x), None, met, J)
    U = empty(ctx.m, *ctx.shape())
    ctx.prim2con(dev(P[sel]), J, U)
    prim = empty(ctx.nprim, *ctx.padded_shape())
    ctx.con2prim(U, J, prim)
    dU = empty(ctx.m, *ctx.shape())
    dJ = empty(*ctx.shape())
    ctx.residual(prim, met, dU, dJ)
    assert ctx.status()[0] == es.ES_OK
    dUg, dJg = host(dU), host(dJ)
    del prim, met, U

    # the oracle's full-size fields from the initial data
    Uo, Jo = st.initial_state(g, wk.scheme, P, wk.x)
    Po, ok = st.prim_from_cons(g, wk.scheme, Uo, Jo)
    assert ok.all()
    Ppad = st.pad_solution(g, Po)
    meto = mt.metrics(g, wk.x, None, 3)
    w = 2
    wg = wl.Grid(3, (w, w, w), g.bc, g.dxi, g.period, g.lo, g.length)
    got, want, gotJ, wantJ = [], [], [], []
    for (i, j, k) in _sample_windows(g.n[0], np.random.default_rng(7), w):
        sl = (slice(None), slice(k, k + w + 6), slice(j, j + w + 6), slice(i, i + w + 6))
        dUw, dJw = rs.residual(wg, wk.scheme, Ppad[sl], meto[sl])
        isl = (slice(None), slice(k, k + w), slice(j, j + w), slice(i, i + w))
        got.append(dUg[isl].reshape(ctx.m, -1))
        want.append(dUw.reshape(ctx.m, -1))
        gotJ.append(dJg[isl[1:]].ravel())
        wantJ.append(dJw.ravel())
    got, want = np.concatenate(got, axis=1), np.concatenate(want, axis=1)
    # the shell samples carry the blast's residual; every component is nonzero there
    assert np.all(np.max(np.abs(want), axis=1) > 0)
    r = rel_inf(got, want)
    assert np.all(r <= TOL), r
    # static uniform mesh: the VCL gives dJ = 0 up to rounding on both sides
    assert np.max(np.abs(np.concatenate(gotJ))) <= 1e-12 * np.max(np.abs(Jo))
    assert np.max(np.abs(np.concatenate(wantJ))) <= 1e-12 * np.max(np.abs(Jo))


def _windows2d(n, rng, w, extra, count=64):
    """Window origins (i, j): the four corners, the origins in `extra`, random ones."""
    out = [(a, b) for a in (0, n[0] - w) for b in (0, n[1] - w)]
    out += [(int(np.clip(i, 0, n[0] - w)), int(np.clip(j, 0, n[1] - w))) for i, j in extra]
    while len(out) < count:
        out.append((int(rng.integers(0, n[0] - w + 1)), int(rng.integers(0, n[1] - w + 1))))
    return out


def _sampled_residual_2d(wk, extra, tol, w=4, floor=None):
    """floor: compare each component against max(its own max, floor x the largest
    component's max) instead of its own max (components that are rounding noise)."""
    g = wk.grid
    ctx = es.Context(g, wk.scheme, wk.monitor)
    ng = ctx.ng
    P = ph.full_prim(wk.prim["rho"], wk.prim["u"], wk.prim["p"], wk.prim["B"])
    sel = ph.comps(wk.scheme.phys, g.dim)
    met = empty(ctx.nmet, *ctx.padded_shape())
    J = empty(*ctx.shape())
    ctx.metrics(dev(wk.x), None, met, J)
    U = empty(ctx.m, *ctx.shape())
    ctx.prim2con(dev(P[sel]), J, U)
    prim = empty(ctx.nprim, *ctx.padded_shape())
    ctx.con2prim(U, J, prim)
    dU = empty(ctx.m, *ctx.shape())
    dJ = empty(*ctx.shape())
    ctx.residual(prim, met, dU, dJ)
    assert ctx.status()[0] == es.ES_OK
    dUg, dJg = host(dU), host(dJ)
    Uo, Jo = st.initial_state(g, wk.scheme, P, wk.x)
    Po, ok = st.prim_from_cons(g, wk.scheme, Uo, Jo)
    assert ok.all()
    Ppad = st.pad_solution(g, Po, wk.scheme.order_p)
    meto = mt.metrics(g, wk.x, None, wk.scheme.order_p)
    wg = wl.Grid(2, (w, w, 1), g.bc, g.dxi, g.period, g.lo, g.length)
    got, want, gotJ = [], [], []
    for (i, j) in _windows2d(g.n, np.random.default_rng(11), w, extra):
        sl = (slice(None), slice(j, j + w + 2 * ng), slice(i, i + w + 2 * ng))
        dUw, _ = rs.residual(wg, wk.scheme, Ppad[sl], meto[sl])
        isl = (slice(None), slice(j, j + w), slice(i, i + w))
        got.append(dUg[isl].reshape(ctx.m, -1))
        want.append(dUw.reshape(ctx.m, -1))
        gotJ.append(dJg[isl[1:]].ravel())
    got, want = np.concatenate(got, axis=1), np.concatenate(want, axis=1)
    if floor is not None:
        big = np.max(np.abs(want))
        r = np.array([np.max(np.abs(got[c] - want[c])) / max(np.max(np.abs(want[c])), floor * big)
                      for c in range(ctx.m)])
        assert np.all(r <= tol), r
    else:
        live = np.max(np.abs(want), axis=1) > 0
        r = rel_inf(got[live], want[live])
        assert np.all(r <= tol), r
        # zero components (m_3 of 2D data without it) stay zero on the GPU
        assert np.max(np.abs(got[~live]), initial=0.0) == 0.0
    # static uniform mesh: the VCL gives dJ = 0 up to rounding
    assert np.max(np.abs(np.concatenate(gotJ))) <= 1e-12 * np.max(np.abs(Jo))
    return r


def test_quadrant_400_residual_at_sampled_nodes():
    wk = wl.quadrant_riemann(n=400, seed=2)
    # the two discontinuities x = 0.5 and y = 0.5 and their crossing
    extra = [(198, 198), (199, 60), (60, 199), (199, 330), (330, 199), (197, 197)]
    _sampled_residual_2d(wk, extra, TOL)


def test_rotor_512_residual_at_sampled_nodes():
    # B along x: exactly repeated eigenvalues at every face outside the disk, and in
    # the taper faces whose Alfven and slow speeds lie just outside the grouping
    # tolerance (smallest ungrouped gap 1.003e-6 in these windows), where the scaled
    # eigenvectors are ill-conditioned: perturbing the oracle's own input by 1e-15
    # moves its residual here by up to 2.8e-7 (B_1) of the component scale
    # max(own max, 1e-3 x largest; m_3 and B_3 are rounding noise).  The bar is ten
    # times that.
    wk = wl.rmhd_rotor(n=512)
    c, r0 = 255.5, 0.1 * 511
    extra = [(int(c + r0 * np.cos(t)) - 2, int(c + r0 * np.sin(t)) - 2) for t in np.linspace(0, 2 * np.pi, 12, endpoint=False)]
    _sampled_residual_2d(wk, extra, 3e-6, floor=1e-3)


def test_fourier_256_residual_at_sampled_nodes():
    # smooth state, face eigenvalues well separated (smallest gap 7e-3), but the
    # residual (about 1e-2) is a small difference of O(1) fluxes at this resolution:
    # perturbing the oracle's own input by 1e-15 moves it by up to 4.8e-11 of a
    # component's max; the uniform field's components are rounding noise (1e-14) and
    # are measured against 1e-2 of the largest component.  The bar is 1e-9.
    wk = wl.rmhd_fourier(n=256, seed=0)
    _sampled_residual_2d(wk, [(100, 100), (128, 128)], 1e-9, floor=1e-2)


def test_rk3_step_blast3d_48_adaptive():
    wk = wl.blast3d(n=48, seed=0)
    (U, J, x, xd), (Uo, Jo, xo, xdo) = run_steps(wk, 1)
    assert np.all(rel_inf(U, Uo) <= TOL), rel_inf(U, Uo)
    assert rel_inf(J[None], Jo[None])[0] <= TOL
    assert np.max(np.abs(x - xo)) <= 1e-13
    assert np.max(np.abs(xd - xdo)) <= 1e-12 * max(np.max(np.abs(xdo)), 1e-300)
