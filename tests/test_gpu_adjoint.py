"""Hand-written adjoint (es_residual_vjp, es_rk3_step_save / es_rk3_step_vjp and
the torch.autograd.Function around them) against directional difference
quotients.

A VJP g = (dF)^T lam is checked through <g, v> = d/dh <lam, F(u + h v)> at h = 0
for random lam and v.  The reference difference quotients come from the oracle
(central differences of the numpy residual or RK3 step); for the ES scheme the
oracle holds its sign switch Y at the values of the unperturbed state (Y is
piecewise constant: its derivative is zero wherever it is defined, and a
difference quotient across a switch flip measures the flip, not the derivative).
The adjoint holds the mesh trajectory and the time step fixed; the oracle step is
given the same time step and mesh velocity.  Central differences at h = 1e-7
(residual) or 1e-8 (step) of quantities computed to ~1e-16 agree with the exact
derivative to ~1e-8 relative (measured 4e-10 to 4e-8 on these cases)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import physics as ph, stepper as st, metrics as mt, residual as rs  # noqa: E402
from paper_2107_12027_amd import es, workloads as wl  # noqa: E402
from paper_2107_12027_amd.autograd import rk3_step as rk3_step_ad  # noqa: E402
from gpu_util import Case, dev, host, empty  # noqa: E402

pytestmark = pytest.mark.gpu

# lines of 100 nodes take the VJP's aligned segment layout (two segments per line),
# the others the flat one (lines laid end to end)
CASES = [(2, (40, 36, 1), (0, 0, 0), True), (2, (40, 36, 1), (0, 0, 0), False),
         (2, (70, 66, 1), (1, 0, 0), True), (2, (30, 33, 1), (1, 1, 0), False),
         (3, (12, 10, 9), (0, 0, 0), True), (3, (12, 10, 9), (1, 1, 1), False),
         (2, (100, 36, 1), (0, 1, 0), True)]


def _oracle_L(case, U, J, met, Y=None, details=False):
    P, ok = st.prim_from_cons(case.grid, case.scheme, U, J)
    assert ok.all()
    return rs.residual(case.grid, case.scheme, st.pad_solution(case.grid, P), met, details=details, Y_fixed=Y)


@pytest.mark.parametrize("dim,n,bc,smooth", CASES)
@pytest.mark.parametrize("diss", [0, 1])
def test_residual_vjp_against_oracle_differences(dim, n, bc, smooth, diss):
    case = Case(dim, n, bc, seed=21, dissipation=diss, smooth=smooth, moving=True)
    c = case.ctx
    U, J = case.gpu_state()
    met = empty(c.nmet, *c.padded_shape())
    c.metrics(dev(case.x), dev(case.xdot), met)
    rng = np.random.default_rng(5)
    Uo, Jo = host(U), host(J)
    meto = mt.metrics(case.grid, case.x, case.xdot)
    Y = None
    if diss:
        _, _, info = _oracle_L(case, Uo, Jo, meto, details=True)
        Y = {k: info[k]["Y"] for k in range(dim)}
    h = 1e-7
    # three (lambda, v) pairs: v along U and J, along U only, along J only
    for pair in range(3):
        lam = rng.normal(size=(c.m,) + c.shape())
        gU = empty(c.m, *c.shape())
        gJ = empty(*c.shape())
        c.residual_vjp(U, J, met, dev(lam), gU, gJ)
        vU = Uo * rng.normal(size=Uo.shape) * (pair != 2)
        vJ = Jo * rng.normal(size=Jo.shape) * (pair != 1)
        adj = float(np.sum(host(gU) * vU) + np.sum(host(gJ) * vJ))
        Lp, _ = _oracle_L(case, Uo + h * vU, Jo + h * vJ, meto, Y)
        Lm, _ = _oracle_L(case, Uo - h * vU, Jo - h * vJ, meto, Y)
        fd = float(np.sum(lam * (Lp - Lm))) / (2 * h)
        assert abs(adj - fd) <= 5e-7 * abs(fd), (pair, adj, fd)


def _gpu_state(w, ctx):
    P = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
    met = empty(ctx.nmet, *ctx.padded_shape())
    J = empty(*ctx.shape())
    x = dev(w.x)
    ctx.metrics(x, None, met, J)
    U = empty(ctx.m, *ctx.shape())
    ctx.prim2con(dev(P[ph.comps(w.scheme.phys, w.grid.dim)]), J, U)
    return U, J, x


@pytest.mark.parametrize("name", ["sine", "quadrant", "blast3d"])
def test_rk3_step_vjp_against_oracle_differences(name):
    # adaptive workloads: the adjoint holds the recorded mesh velocity and time
    # step; the oracle step is run with the same prescribed mesh velocity and dt
    w = {"sine": lambda: wl.advected_sine(n=40), "quadrant": lambda: wl.quadrant_riemann(n=40, seed=2),
         "blast3d": lambda: wl.blast3d(n=12, seed=0, p_in=10.0)}[name]()
    g = w.grid
    ctx = es.Context(g, w.scheme, w.monitor)
    U, J, x = _gpu_state(w, ctx)
    Uo, Jo = host(U).copy(), host(J).copy()
    xo = host(x).copy()
    ck = empty(ctx.ckpt_doubles())
    xd = empty(g.dim, *ctx.shape())
    dt = empty(1)
    ctx.rk3_step_save(U, J, x, xd, dt, ck)
    assert ctx.status()[0] == es.ES_OK
    rng = np.random.default_rng(8)
    lamU = rng.normal(size=Uo.shape)
    lamJ = rng.normal(size=Jo.shape)
    gU = empty(ctx.m, *ctx.shape())
    gJ = empty(*ctx.shape())
    ctx.rk3_step_vjp(ck, dev(lamU), dev(lamJ), gU, gJ)
    dt0, xdot0 = float(host(dt)[0]), host(xd)
    base = st.rk3_step(g, w.scheme, None, Uo, Jo, xo, dt=dt0, xdot=xdot0, details=True)
    # directions in U and in J separately (their contributions can nearly cancel);
    # h = 1e-8: on the discontinuous quadrant data the O(h^2) term of the central
    # difference is 3e-7 relative at h = 1e-7 and 7e-9 at h = 1e-8
    h = 1e-8
    for vU, vJ in ((Uo * rng.normal(size=Uo.shape), 0.0 * Jo), (0.0 * Uo, Jo * rng.normal(size=Jo.shape))):
        adj = float(np.sum(host(gU) * vU) + np.sum(host(gJ) * vJ))
        op = st.rk3_step(g, w.scheme, None, Uo + h * vU, Jo + h * vJ, xo, dt=dt0, xdot=xdot0, Y_fixed=base["Y"])
        om = st.rk3_step(g, w.scheme, None, Uo - h * vU, Jo - h * vJ, xo, dt=dt0, xdot=xdot0, Y_fixed=base["Y"])
        assert op["ok"].all() and om["ok"].all()
        fd = float(np.sum(lamU * (op["U"] - om["U"])) + np.sum(lamJ * (op["J"] - om["J"]))) / (2 * h)
        assert abs(adj - fd) <= 1e-6 * abs(fd), (adj, fd)


def test_step_with_checkpoint_equals_step():
    w = wl.quadrant_riemann(n=70, seed=2)
    out = []
    for save in (False, True):
        ctx = es.Context(w.grid, w.scheme, w.monitor)
        ctx.set_graph(False)
        U, J, x = _gpu_state(w, ctx)
        xd = empty(w.grid.dim, *ctx.shape())
        dt = empty(1)
        for _ in range(2):
            if save:
                ctx.rk3_step_save(U, J, x, xd, dt, empty(ctx.ckpt_doubles()))
            else:
                ctx.rk3_step(U, J, x, xd, dt)
        out.append((host(U), host(J), host(x), host(dt)))
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_autograd_function_two_steps():
    # loss after two steps of the torch.autograd.Function; the gradient equals the
    # chained es_rk3_step_vjp calls and passes a GPU difference check (EC scheme:
    # no switch, static curvilinear mesh, fixed dt)
    case = Case(2, (48, 40, 1), (0, 0, 0), seed=30, dissipation=0, smooth=True, moving=False)
    c = case.ctx
    U0, J0 = case.gpu_state()
    x0 = dev(case.x)
    fixed = dev(np.array([2e-3]))
    rng = np.random.default_rng(9)
    wU = dev(rng.normal(size=(c.m,) + c.shape()))
    wJ = dev(rng.normal(size=c.shape()))

    def loss_of(U, J):
        x = x0
        for _ in range(2):
            U, J, x, _ = rk3_step_ad(U, J, c, x, fixed)
        return (wU * U).sum() + (wJ * J).sum()

    Ua = U0.clone().requires_grad_(True)
    Ja = J0.clone().requires_grad_(True)
    loss = loss_of(Ua, Ja)
    gU, gJ = torch.autograd.grad(loss, (Ua, Ja))
    v = U0 * dev(rng.normal(size=(c.m,) + c.shape()))
    h = 1e-6
    with torch.no_grad():
        fd = (loss_of(U0 + h * v, J0) - loss_of(U0 - h * v, J0)) / (2 * h)
    adj = float((gU * v).sum())
    assert abs(adj - float(fd)) <= 1e-7 * abs(float(fd)), (adj, float(fd))
    assert torch.isfinite(gJ).all()


def _fourier_forward(n, steps, coeffs, dt, ckpts=None, phys=ph.RHD, p=3):
    """GPU forward of the Fourier-mode workload (RHD, or RMHD as in the adjoint
    configuration) with a fixed time step and order parameter p; returns (ctx, U, J,
    prim0 interior, mask weight) after `steps` steps."""
    from paper_2107_12027_amd import losses
    w = (wl.rhd_fourier if phys == ph.RHD else wl.rmhd_fourier)(n=n, coeffs=coeffs)
    w.scheme.order_p = p
    ctx = es.Context(w.grid, w.scheme, w.monitor)
    U, J, x = _gpu_state(w, ctx)
    Pfull = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
    P0 = dev(Pfull[ph.comps(w.scheme.phys, 2)] if phys == ph.RHD else Pfull)
    xd = empty(2, *ctx.shape())
    dtv = empty(1)
    fixed = dev(np.array([dt]))
    for k in range(steps):
        if ckpts is not None:
            ck = empty(ctx.ckpt_doubles())
            ctx.rk3_step_save(U, J, x, xd, dtv, ck, fixed)
            ckpts.append(ck)
        else:
            ctx.rk3_step(U, J, x, xd, dtv, fixed)
    xs = w.x
    inside = (xs[0] >= 0.4) & (xs[0] <= 0.6) & (xs[1] >= 0.4) & (xs[1] <= 0.6)
    weight = dev(inside * (1.0 / (n * n)))
    return ctx, U, J, P0, weight, losses


@pytest.mark.parametrize("phys,K,tol,p", [(ph.RHD, 4, 1e-6, 3), (ph.RMHD, 3, 1e-5, 3), (ph.RMHD, 2, 5e-5, 2)])
def test_fourier_mode_gradient_against_differences(phys, K, tol, p):
    # the gradient of L = integral of rho^2 over [0.4,0.6]^2 after K steps with
    # respect to the 8 density-mode coefficients (the adjoint configuration's loss on
    # its RMHD workload, and on the RHD counterpart; static mesh, fixed dt): adjoint
    # chain (es_rk3_step_save / es_rk3_step_vjp, con2prim by the implicit-function
    # rule at both ends) against central differences h = 1e-6 of the GPU forward and,
    # for two coefficients, of the oracle's forward.  RMHD: the adjoint holds the face
    # eigen-structure, whose variation multiplies the WENO jumps of this smooth flow.
    # p = 2 (RMHD): the same chain through the 4th-order flux and WENO3 dissipation;
    # the held eigen-structure's terms multiply the WENO3 jumps, larger on this 32^2
    # state than WENO5's (measured 2.4e-5 of the largest component against 4e-6 at
    # p = 3), while the residual VJP itself matches the oracle with the structure
    # held to 1e-6 (test_p2_rmhd_residual_vjp_against_oracle_differences)
    n, dt, h = 32, 6.25e-3, 1e-6
    make = wl.rhd_fourier if phys == ph.RHD else wl.rmhd_fourier
    _, _, c0 = wl.fourier_modes(0)
    ck = []
    ctx, U, J, P0, weight, losses = _fourier_forward(n, K, c0, dt, ck, phys, p)
    L, gU, gJ = losses.density_squared(ctx, U, J, weight)
    for k in reversed(range(K)):
        oU, oJ = empty(*gU.shape), empty(*gJ.shape)
        ctx.rk3_step_vjp(ck[k], gU, gJ, oU, oJ)
        gU, gJ = oU, oJ
    w0 = make(n=n, coeffs=c0)
    J0 = dev(mt.jacobian(w0.grid, w0.x, p))
    phi = dev(wl.fourier_basis(w0.x))
    grad = losses.density_mode_gradient(ctx, P0, J0, gU, phi, 0.05).cpu().numpy()

    def loss_gpu(c):
        cx, Ux, Jx, _, wx, _ = _fourier_forward(n, K, c, dt, None, phys, p)
        return float(losses.density_squared(cx, Ux, Jx, wx)[0])

    fd = np.array([(loss_gpu(c0 + h * e) - loss_gpu(c0 - h * e)) / (2 * h) for e in np.eye(8)])
    scale = np.max(np.abs(fd))
    assert np.max(np.abs(grad - fd)) <= tol * scale, (grad, fd)

    # the oracle's forward (same inputs, prescribed zero mesh velocity and the same dt)
    def loss_oracle(c):
        wx = make(n=n, coeffs=c)
        wx.scheme.order_p = p
        Px = ph.full_prim(wx.prim["rho"], wx.prim["u"], wx.prim["p"], wx.prim["B"])
        Uo, Jo = st.initial_state(wx.grid, wx.scheme, Px, wx.x)
        xo = wx.x
        for _ in range(K):
            out = st.rk3_step(wx.grid, wx.scheme, None, Uo, Jo, xo, dt=dt, xdot=np.zeros_like(xo))
            Uo, Jo, xo = out["U"], out["J"], out["x"]
        Po, ok = st.prim_from_cons(wx.grid, wx.scheme, Uo, Jo)
        assert ok.all()
        return float(np.sum(host(weight) * Po[0] ** 2))

    for m in (0, 5):
        e = np.eye(8)[m]
        fo = (loss_oracle(c0 + h * e) - loss_oracle(c0 - h * e)) / (2 * h)
        assert abs(grad[m] - fo) <= tol * scale, (m, grad[m], fo)


# ---------------------------------------------------------------------------
# RMHD: the pair fluxes, the Godunov-Powell source and the face dissipation with
# its eigen-structure held (as well as Y); the oracle's difference quotients hold
# both through Y_fixed and eig_fixed
# ---------------------------------------------------------------------------
RCASES = [(2, (40, 36, 1), (0, 0, 0), True), (2, (30, 33, 1), (1, 1, 0), False),
          (3, (10, 9, 8), (0, 0, 0), True)]


@pytest.mark.parametrize("dim,n,bc,smooth", RCASES)
@pytest.mark.parametrize("diss", [0, 1])
def test_rmhd_residual_vjp_against_oracle_differences(dim, n, bc, smooth, diss, p=3):
    case = Case(dim, n, bc, phys=ph.RMHD, seed=23, dissipation=diss, smooth=smooth, moving=True, p=p)
    c = case.ctx
    U, J = case.gpu_state()
    met = empty(c.nmet, *c.padded_shape())
    c.metrics(dev(case.x), dev(case.xdot), met)
    rng = np.random.default_rng(6)
    lam = rng.normal(size=(c.m,) + c.shape())
    gU = empty(c.m, *c.shape())
    gJ = empty(*c.shape())
    c.residual_vjp(U, J, met, dev(lam), gU, gJ)
    Uo, Jo = host(U), host(J)
    vU = Uo * rng.normal(size=Uo.shape) * 1e-2
    vJ = Jo * rng.normal(size=Jo.shape) * 1e-2
    adj = float(np.sum(host(gU) * vU) + np.sum(host(gJ) * vJ))
    meto = mt.metrics(case.grid, case.x, case.xdot, p)
    Y = eig = None
    if diss:
        _, _, info = _oracle_L(case, Uo, Jo, meto, details=True)
        Y = {k: info[k]["Y"] for k in range(dim)}
        eig = {k: info[k]["eig"] for k in range(dim)}

    def Lo(Ux, Jx):
        P, ok = st.prim_from_cons(case.grid, case.scheme, Ux, Jx)
        assert ok.all()
        return rs.residual(case.grid, case.scheme, st.pad_solution(case.grid, P), meto, Y_fixed=Y, eig_fixed=eig)

    h = 1e-6
    Lp, _ = Lo(Uo + h * vU, Jo + h * vJ)
    Lm, _ = Lo(Uo - h * vU, Jo - h * vJ)
    fd = float(np.sum(lam * (Lp - Lm))) / (2 * h)
    assert abs(adj - fd) <= 1e-6 * abs(fd), (adj, fd)
