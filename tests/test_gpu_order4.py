"""The p = 4 scheme on the GPU (8th-order EC flux and metrics with alpha_{4,n} of
eq. HOCoeff, WENO7 dissipation, w = 2p - 1; a padded layout of four ghost layers)
against the oracle on identical seeded inputs: metrics and Jacobian, con2prim on
the padded box, the EC and ES residuals of both systems on random curvilinear
moving meshes (2D and 3D), the FP32-mixed residual within its bound, adaptive
RK3 steps, and the refusal of the adjoint.  Same bars as the p = 3 path (RMHD ES:
the well-separated states of the p = 3 tests at 1e-12)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import physics as ph, metrics as mt, stepper as st, residual as rs  # noqa: E402
from paper_2107_12027_amd import es, workloads as wl  # noqa: E402
from gpu_util import Case, dev, host, empty, rel_inf, run_steps  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12
GRIDS = [(2, (130, 70, 1), (0, 0, 0)), (2, (64, 123, 1), (1, 1, 0)),
         (3, (70, 9, 10), (0, 0, 0)), (3, (10, 66, 9), (1, 1, 1))]


def test_p4_layout_has_four_ghost_layers():
    case = Case(2, (20, 18, 1), (0, 0, 0), seed=0, p=4)
    assert case.ctx.ng == 4 and case.ctx.padded_shape() == (26, 28)
    # outflow axes need 2 ng + 1 = 9 nodes
    g = wl.make_grid(2, (8, 12, 1), (wl.OUTFLOW, wl.OUTFLOW, wl.PERIODIC))
    with pytest.raises(es.EsError) as err:
        es.Context(g, wl.Scheme(order_p=4), wl.Monitor(enabled=0))
    assert err.value.status == es.ES_EINVAL


@pytest.mark.parametrize("dim,n,bc", GRIDS)
def test_p4_metrics_and_jacobian(dim, n, bc):
    case = Case(dim, n, bc, seed=1, p=4)
    c = case.ctx
    met = empty(c.nmet, *c.padded_shape())
    J = empty(*c.shape())
    c.metrics(dev(case.x), dev(case.xdot), met, J)
    want = mt.metrics(case.grid, case.x, case.xdot, 4)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(host(met) - want)) <= 1e-13 * scale
    Jw = mt.jacobian(case.grid, case.x, 4)
    assert np.max(np.abs(host(J) - Jw)) <= 1e-13 * np.max(np.abs(Jw))
    # the metrics without the initial Jacobian take the marching 3D kernel
    met2 = empty(c.nmet, *c.padded_shape())
    c.metrics(dev(case.x), dev(case.xdot), met2)
    assert np.max(np.abs(host(met2) - want)) <= 1e-13 * scale


@pytest.mark.parametrize("dim,n,bc", GRIDS[1:3])
@pytest.mark.parametrize("phys", [ph.RHD, ph.RMHD])
def test_p4_con2prim_padded(dim, n, bc, phys):
    case = Case(dim, n, bc, phys=phys, seed=2, vmax=0.95, p=4)
    c = case.ctx
    U, J = case.gpu_state()
    prim = empty(c.nprim, *c.padded_shape())
    c.con2prim(U, J, prim)
    assert c.status()[0] == es.ES_OK
    Uo, Jo = case.oracle_state()
    Po, ok = st.prim_from_cons(case.grid, case.scheme, Uo, Jo)
    assert ok.all()
    sel = ph.comps(phys, dim)                      # the primitive slots, pressure in the U slot of E
    Ppad = st.pad_solution(case.grid, Po, 4)[sel]
    p = Ppad[sel.index(4)]
    want = np.concatenate([Ppad, np.log(Ppad[0])[None], np.log(Ppad[0] / p)[None]])
    assert np.all(rel_inf(host(prim), want) <= 1e-12), rel_inf(host(prim), want)


@pytest.mark.parametrize("dim,n,bc", GRIDS)
@pytest.mark.parametrize("diss", [0, 1])
def test_p4_residual(dim, n, bc, diss):
    case = Case(dim, n, bc, seed=4 + diss, dissipation=diss, p=4)
    _, _, _, _, dU, dJ = case.residual()
    dUo, dJo = case.oracle_residual()
    r = rel_inf(host(dU), dUo)
    assert np.all(r <= TOL), r
    assert rel_inf(host(dJ)[None], dJo[None])[0] <= TOL


SEP_B0 = np.array([0.6, 0.45, 0.35])


@pytest.mark.parametrize("dim,n,bc", [(2, (40, 36, 1), (0, 0, 0)), (2, (33, 30, 1), (1, 1, 0)),
                                      (3, (10, 9, 11), (0, 1, 0))])
@pytest.mark.parametrize("diss", [0, 1])
def test_p4_rmhd_residual(dim, n, bc, diss):
    # EC at random states; ES at smooth states with well-separated eigenvalues (the
    # p = 3 construction: field B0 + 0.1 (smooth))
    if diss:
        case = Case(dim, n, bc, phys=ph.RMHD, seed=31 + dim, smooth=True, dissipation=1, p=4)
        case.P[5:8] = SEP_B0.reshape((3,) + (1,) * dim) + 0.1 * case.P[5:8]
    else:
        case = Case(dim, n, bc, phys=ph.RMHD, seed=7, dissipation=0, p=4)
    _, _, _, _, dU, dJ = case.residual()
    dUo, dJo = case.oracle_residual()
    r = rel_inf(host(dU), dUo)
    assert np.all(r <= TOL), r
    assert rel_inf(host(dJ)[None], dJo[None])[0] <= TOL


@pytest.mark.parametrize("dim,n,bc", GRIDS[:3])
def test_p4_mixed_residual_within_bound(dim, n, bc):
    # FP32 pair algebra and dissipation: relative L1 within the p = 3 bound on
    # random states (tests/test_gpu_mixed.py)
    case = Case(dim, n, bc, seed=9, dissipation=1, mixed=1, p=4)
    _, _, _, _, dU, _ = case.residual()
    dUo, _ = case.oracle_residual()
    a, b = host(dU).reshape(case.m, -1), dUo.reshape(case.m, -1)
    l1 = np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)
    assert np.all(l1 <= 1e-4), l1


@pytest.mark.parametrize("name", ["sine", "quadrant", "blast3d"])
def test_p4_rk3_step_adaptive(name):
    w = {"sine": lambda: wl.advected_sine(n=72), "quadrant": lambda: wl.quadrant_riemann(n=70, seed=2),
         "blast3d": lambda: wl.blast3d(n=24, seed=0)}[name]()
    w.scheme.order_p = 4
    (U, J, x, xd), (Uo, Jo, xo, xdo) = run_steps(w, 1)
    assert np.all(rel_inf(U, Uo) <= TOL), rel_inf(U, Uo)
    assert rel_inf(J[None], Jo[None])[0] <= TOL
    assert np.max(np.abs(x - xo)) <= 1e-13


def test_p4_adjoint_unsupported():
    w = wl.quadrant_riemann(n=20, seed=2)
    w.scheme.order_p = 4
    ctx = es.Context(w.grid, w.scheme, w.monitor)
    U, J, x, xd = empty(ctx.m, *ctx.shape()), empty(*ctx.shape()), empty(2, *ctx.shape()), empty(2, *ctx.shape())
    dt, ck = empty(1), empty(ctx.ckpt_doubles())
    with pytest.raises(es.EsError) as err:
        ctx.rk3_step_save(U, J, x, xd, dt, ck)
    assert err.value.status == es.ES_EUNSUPPORTED
