"""Pins for the semi-discrete scheme (Section 3.2, Theorem 4.1, Proposition 4.2,
Theorem 5.1) on random curvilinear moving meshes."""
import numpy as np
import pytest

from oracle import physics as ph, metrics as mt, residual as rs, stepper as st, ecflux as ec
from paper_2107_12027_amd import workloads as wl

G = 5.0 / 3.0
CASES = [(ph.RHD, 2, (12, 10, 1)), (ph.RHD, 3, (7, 6, 8)), (ph.RMHD, 2, (10, 12, 1))]


def setup(phys, dim, n, bc=(0, 0, 0), seed=0, smooth=False):
    rng = np.random.default_rng(seed)
    g = wl.make_grid(dim, n, bc)
    x = wl.perturbed_mesh(g, rng, amp=0.03)
    xdot = wl.perturbed_mesh(g, rng, amp=0.05) - wl.uniform_mesh(g)
    met = mt.metrics(g, x, xdot)
    if smooth:
        pr = wl.smooth_prim(x, rng, phys)
    else:
        pr = wl.random_prim(g.shape, rng, phys=phys, dim=dim, vmax=0.9)
    P = ph.full_prim(pr["rho"], pr["u"], pr["p"], pr["B"])
    return g, x, xdot, met, P


@pytest.mark.parametrize("phys,dim,n", CASES)
def test_ec_scheme_conserves_entropy(phys, dim, n):
    # Theorem 4.1: sum_i (V_i . dU_i/dt - phi_i dJ_i/dt) = 0 on a periodic mesh
    g, x, xdot, met, P = setup(phys, dim, n)
    sc = wl.Scheme(phys=phys, dissipation=0)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P), met)
    sel = ph.comps(phys, dim)
    V = ph.entropy_vars(P, G)[sel]
    phi, _, _ = ph.potentials(P, G)
    ep = rs.entropy_production(g, sc, P, dU, dJ)
    scale = np.sum(np.abs(V * dU)) + np.sum(np.abs(phi * dJ))
    assert abs(ep) < 1e-14 * scale


@pytest.mark.parametrize("phys,dim,n", CASES)
def test_es_scheme_produces_entropy_with_right_sign(phys, dim, n):
    # Theorem 5.1: the ES scheme can only decrease the total entropy
    for seed in range(3):
        g, x, xdot, met, P = setup(phys, dim, n, seed=seed)
        sc = wl.Scheme(phys=phys, dissipation=1)
        dU, dJ = rs.residual(g, sc, st.pad_solution(g, P), met)
        assert rs.entropy_production(g, sc, P, dU, dJ) < 0


@pytest.mark.parametrize("phys,dim,n", CASES)
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_free_stream_preservation(phys, dim, n, bc):
    # Proposition 4.2 / remark after Theorem 5.1: for a constant state dU/dt = U_0 dJ/dt
    g, x, xdot, met, P = setup(phys, dim, n, bc=bc)
    Pc = np.broadcast_to(P.reshape(8, -1)[:, :1].reshape((8,) + (1,) * dim), P.shape).copy()
    U0 = ph.cons(Pc, G)[ph.comps(phys, dim)]
    for diss in (0, 1):
        sc = wl.Scheme(phys=phys, dissipation=diss)
        dU, dJ = rs.residual(g, sc, st.pad_solution(g, Pc), met)
        assert np.max(np.abs(dU - U0 * dJ)) < 1e-13 * np.max(np.abs(U0)) * np.max(np.abs(met)) / min(g.dxi[:dim])


@pytest.mark.parametrize("phys,dim,n", CASES)
def test_conservation_on_periodic_mesh(phys, dim, n):
    # telescoping form: sum_i dD_i/dt = 0, sum_i dJ_i/dt = 0 and, for RHD, every component
    g, x, xdot, met, P = setup(phys, dim, n)
    sc = wl.Scheme(phys=phys, dissipation=1)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P), met)
    comps = range(dU.shape[0]) if phys == ph.RHD else [0]
    for c in comps:
        assert abs(np.sum(dU[c])) < 1e-13 * np.sum(np.abs(dU[c]))
    assert abs(np.sum(dJ)) < 1e-12 * (np.sum(np.abs(dJ)) + 1)


@pytest.mark.parametrize("phys,dim,n", CASES)
def test_literal_fluxes_equal_telescoped_pairs(phys, dim, n):
    # eq. ECFlux_O2p summed over s telescopes to sum_n alpha_n [F~(i,i+n) - F~(i-n,i)]:
    # an independent assembly of the EC part from the pair flux alone
    g, x, xdot, met, P = setup(phys, dim, n, seed=4)
    sc = wl.Scheme(phys=phys, dissipation=0)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P), met)
    Ppad = st.pad_solution(g, P)
    al = mt.alpha(3)
    want = np.zeros((8,) + g.shape)
    wantJ = np.zeros(g.shape)
    src = np.zeros(g.shape)
    for k in range(dim):
        ax = dim - 1 - k
        Pk = rs._line_view(Ppad, g, k, 1)
        ak = rs._line_view(met[k * (dim + 1):(k + 1) * (dim + 1)], g, k, 1)
        i = np.arange(3, 3 + g.n[k])
        for m in range(1, 4):
            T = lambda a, idx: np.take(a, idx, axis=1 + ax)
            fp = ec.curvilinear_pair(T(Pk, i), T(Pk, i + m), T(ak, i), T(ak, i + m), G, phys, dim)
            fm = ec.curvilinear_pair(T(Pk, i - m), T(Pk, i), T(ak, i - m), T(ak, i), G, phys, dim)
            want -= al[m - 1] * (fp - fm) / g.dxi[k]
            wantJ -= al[m - 1] * 0.5 * (T(ak, i + m)[0] - T(ak, i - m)[0]) / g.dxi[k]
            if phys == ph.RMHD:
                src += al[m - 1] * (ec.curvilinear_pair_B(T(Pk, i), T(Pk, i + m), T(ak, i), T(ak, i + m), dim)
                                    - ec.curvilinear_pair_B(T(Pk, i - m), T(Pk, i), T(ak, i - m), T(ak, i), dim)) / g.dxi[k]
    if phys == ph.RMHD:
        want -= ph.phi_prime(P, G) * src
    sel = ph.comps(phys, dim)
    np.testing.assert_allclose(dU, want[sel], rtol=1e-11, atol=1e-11 * np.max(np.abs(dU)))
    np.testing.assert_allclose(dJ, wantJ, rtol=1e-11, atol=1e-12 * (1 + np.max(np.abs(dJ))))


def _order_errors(diss, moving, Ns, p=3):
    errs = []
    for n in Ns:
        g = wl.make_grid(2, (n, n, 1), (0, 0, 0))
        x = wl.perturbed_mesh(g, np.random.default_rng(5), amp=0.02)
        xdot = (wl.perturbed_mesh(g, np.random.default_rng(9), amp=0.05) - wl.uniform_mesh(g)) if moving else np.zeros_like(x)
        s = x[0] + x[1]
        rho = 1 + 0.2 * np.sin(2 * np.pi * s)
        drho = 0.4 * np.pi * np.cos(2 * np.pi * s)
        vx = vy = 0.2
        W = 1 / np.sqrt(1 - vx * vx - vy * vy)
        u = np.zeros((3,) + g.shape)
        u[0], u[1] = W * vx, W * vy
        P = ph.full_prim(rho, u, np.ones(g.shape), np.zeros((3,) + g.shape))
        met = mt.metrics(g, x, xdot, p)
        J = mt.jacobian(g, x, p)
        dU, dJ = rs.residual(g, wl.Scheme(dissipation=diss, order_p=p), st.pad_solution(g, P, p), met)
        U = ph.cons(P, G)[[0, 1, 2, 4]]
        # exact rate of change following a mesh node of the advected-density solution
        dUdrho = np.array([W, W * W * vx, W * W * vy, W * W])[:, None, None]
        exact = dUdrho * ((xdot[0] + xdot[1]) - (vx + vy)) * drho
        errs.append(np.mean(np.abs((dU - U * dJ) / J - exact)))     # discrete L1 norm
    return np.array(errs)


@pytest.mark.parametrize("moving", [0, 1])
def test_ec_residual_sixth_order(moving):
    e = _order_errors(0, moving, (16, 32, 64))
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 5.7, (e, rates)


@pytest.mark.parametrize("moving", [0, 1])
def test_es_residual_fifth_order(moving):
    e = _order_errors(1, moving, (32, 64, 128))
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 4.8, (e, rates)


# p = 2: the 4th-order EC flux (alpha_{2,n} = 4/3, -1/6) with WENO3 dissipation (w = 2p - 1)
@pytest.mark.parametrize("moving", [0, 1])
def test_ec_residual_fourth_order_p2(moving):
    e = _order_errors(0, moving, (16, 32, 64), p=2)
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 3.9, (e, rates)


def test_es_residual_third_order_p2():
    # WENO3-JS with eps = 1e-6 loses accuracy near the extrema of the profile on
    # coarse meshes (rates 2.0, 2.6 from 32 to 128); from 128 to 256 the rate is 3.7
    e = _order_errors(1, 0, (64, 128, 256), p=2)
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 2.9, (e, rates)


# p = 4: the 8th-order EC flux and metrics (alpha_{4,n} = 8/5, -2/5, 8/105, -1/140) with
# WENO7 dissipation (w = 2p - 1) on a box padded by four ghost layers
@pytest.mark.parametrize("moving", [0, 1])
def test_ec_residual_eighth_order_p4(moving):
    e = _order_errors(0, moving, (16, 32, 64), p=4)
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 7.7, (e, rates)


def test_es_residual_seventh_order_p4():
    e = _order_errors(1, 0, (32, 64, 128), p=4)
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 6.5, (e, rates)


@pytest.mark.parametrize("phys,dim,n", CASES)
def test_p4_entropy_and_free_stream(phys, dim, n):
    # Theorems 4.1 and 5.1 and Proposition 4.2 with p = 4 (four ghost layers)
    g, x, xdot, _, P = setup(phys, dim, n, seed=5)
    met = mt.metrics(g, x, xdot, 4)
    sel = ph.comps(phys, dim)
    sc = wl.Scheme(phys=phys, dissipation=0, order_p=4)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P, 4), met)
    V = ph.entropy_vars(P, G)[sel]
    phi, _, _ = ph.potentials(P, G)
    scale = np.sum(np.abs(V * dU)) + np.sum(np.abs(phi * dJ))
    assert abs(rs.entropy_production(g, sc, P, dU, dJ)) < 1e-14 * scale
    sc = wl.Scheme(phys=phys, dissipation=1, order_p=4)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P, 4), met)
    assert rs.entropy_production(g, sc, P, dU, dJ) < 0
    Pc = np.broadcast_to(P.reshape(8, -1)[:, :1].reshape((8,) + (1,) * dim), P.shape).copy()
    U0 = ph.cons(Pc, G)[sel]
    for diss in (0, 1):
        sc = wl.Scheme(phys=phys, dissipation=diss, order_p=4)
        dU, dJ = rs.residual(g, sc, st.pad_solution(g, Pc, 4), met)
        assert np.max(np.abs(dU - U0 * dJ)) < 1e-13 * np.max(np.abs(U0)) * np.max(np.abs(met)) / min(g.dxi[:dim])


def test_p4_metrics_discrete_scl_and_affine_exactness():
    # the 8th-order CMM metrics satisfy the discrete SCL on a random periodic mesh and
    # are exact (constant cofactors) on an affine one
    for dim, n in ((2, (14, 13, 1)), (3, (9, 10, 11))):
        rng = np.random.default_rng(8 + dim)
        g = wl.make_grid(dim, n, (0, 0, 0))
        x = wl.perturbed_mesh(g, rng, amp=0.03)
        met = mt.metrics(g, x, None, 4)
        al = mt.alpha(4)
        ng = mt.ghost(4)
        for j in range(dim):
            scl = 0.0
            for k in range(dim):
                a = met[k * (dim + 1) + 1 + j]
                ax = a.ndim - 1 - k
                dk = mt.delta(a, ax, 4)
                for kk in range(dim):
                    if kk != k:
                        dk = mt.crop(dk, a.ndim - 1 - kk, ng)
                    else:
                        dk = mt.crop(dk, ax, ng - 4)
                scl = scl + dk / g.dxi[k]
            assert np.max(np.abs(scl)) < 1e-11 * np.max(np.abs(met))
        A = rng.normal(size=(dim, dim)) * 0.2 + np.eye(dim)
        xa = np.einsum("ab,b...->a...", A, wl.uniform_mesh(wl.make_grid(dim, n, (1, 1, 1))))
        ga = wl.make_grid(dim, n, (1, 1, 1))
        meta = mt.metrics(ga, xa, None, 4)
        for c in range(meta.shape[0]):
            assert np.ptp(meta[c]) < 1e-11 * (1 + np.max(np.abs(meta[c])))


def test_rmhd_vortex_ec_high_order_p4():
    # p = 4 on the vortex: rate 6.4 from 24 to 48 nodes per side, then the error meets
    # a floor of about 5e-8 that p = 3 meets too (the field decays only like
    # e^{-r^2/2} and is about 3e-5 at the periodic boundary of [-5, 5]^2), so the
    # clean eighth-order pin is the advected profile above
    e = _vortex_errors(0, (24, 48), order=4)
    rate = np.log2(e[0] / e[1])
    assert rate > 6.2, (e, rate)
    assert e[1] < 0.5 * _vortex_errors(0, (48,), order=3)[0]


@pytest.mark.parametrize("phys,dim,n", CASES[:2])
def test_p2_entropy_and_free_stream(phys, dim, n):
    # Theorems 4.1 and 5.1 and Proposition 4.2 hold for any p: with p = 2 the EC
    # residual produces no entropy, the ES residual only decreases it, and a
    # uniform state on the moving curvilinear mesh keeps dU/dt = U_0 dJ/dt
    g, x, xdot, _, P = setup(phys, dim, n, seed=3)
    met = mt.metrics(g, x, xdot, 2)
    sel = ph.comps(phys, dim)
    sc = wl.Scheme(phys=phys, dissipation=0, order_p=2)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P), met)
    V = ph.entropy_vars(P, G)[sel]
    phi, _, _ = ph.potentials(P, G)
    scale = np.sum(np.abs(V * dU)) + np.sum(np.abs(phi * dJ))
    assert abs(rs.entropy_production(g, sc, P, dU, dJ)) < 1e-14 * scale
    sc = wl.Scheme(phys=phys, dissipation=1, order_p=2)
    dU, dJ = rs.residual(g, sc, st.pad_solution(g, P), met)
    assert rs.entropy_production(g, sc, P, dU, dJ) < 0
    Pc = np.broadcast_to(P.reshape(8, -1)[:, :1].reshape((8,) + (1,) * dim), P.shape).copy()
    U0 = ph.cons(Pc, G)[sel]
    for diss in (0, 1):
        sc = wl.Scheme(phys=phys, dissipation=diss, order_p=2)
        dU, dJ = rs.residual(g, sc, st.pad_solution(g, Pc), met)
        assert np.max(np.abs(dU - U0 * dJ)) < 1e-13 * np.max(np.abs(U0)) * np.max(np.abs(met)) / min(g.dxi[:dim])


def _vortex_errors(diss, Ns, order=3):
    # the semi-discrete residual against the exact d(J U)/dt of the RMHD vortex at
    # t = 0 (complex-step derivative of the closed form in t) on static uniform
    # periodic meshes of [-5, 5]^2
    errs = []
    for n in Ns:
        g = wl.make_grid(2, (n, n, 1), (0, 0, 0), lo=(-5.0, -5.0, 0.0), length=(10.0, 10.0, 1.0))
        x = wl.uniform_mesh(g)
        rho, v, p, B = wl.vortex2d_state(x[0], x[1], 0.0)
        W = 1.0 / np.sqrt(1.0 - np.sum(v * v, axis=0))
        P = ph.full_prim(rho, W * v, p, B)
        met = mt.metrics(g, x, None, order)
        J = mt.jacobian(g, x, order)
        dU, dJ = rs.residual(g, wl.Scheme(phys=ph.RMHD, dissipation=diss, order_p=order),
                             st.pad_solution(g, P, order), met)
        hc = 1e-30
        rc, vc, pc, Bc = wl.vortex2d_state(x[0].astype(complex), x[1].astype(complex), 1j * hc)
        Wc = 1.0 / np.sqrt(1.0 - np.sum(vc * vc, axis=0))
        Uc = ph.cons(ph.full_prim(rc, Wc * vc, pc, Bc), wl.VORTEX_GAMMA)
        exact = np.imag(Uc) / hc
        errs.append(np.mean(np.abs(dU / J - exact[:8])))
    return np.array(errs)


def test_rmhd_vortex_ec_sixth_order():
    # the RMHD vortex is an exact solution (the closed form of Section 6): the EC
    # residual converges to its time derivative at the design order 2p = 6
    e = _vortex_errors(0, (24, 48, 96))
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 5.5, (e, rates)


def test_rmhd_vortex_es_order():
    # the ES residual (EC flux plus WENO5 dissipation on the scaled entropy
    # variable jumps) tends to the design order 5 from below: the WENO weights
    # lose accuracy near the vortex's critical points on coarse meshes, so the
    # observed rate climbs (3.1, 3.8, 4.2 over 24 -> 192 nodes per side)
    e = _vortex_errors(1, (96, 192))
    rate = np.log2(e[0] / e[1])
    assert rate > 4.0, (e, rate)


def _vortex3d_errors(Ns, t=1.0):
    # the EC residual on the paper's prescribed 3D moving mesh (Section 6, example
    # RMHD_3DVortex, nodes on the periodic N x N x 5N box, taken at t = 1 so that
    # the mesh velocity is not zero) against the exact semi-discrete rate: along a
    # node path d(J U)/dt = J (dU/dt + xdot . grad U) + U dJ/dt, with the discrete
    # dJ/dt of the VCL and the material derivative by a complex step along (xdot, 1)
    errs = []
    for n in Ns:
        w = wl.rmhd_vortex(3, n, t=t, dissipation=0)
        g, x = w.grid, w.x
        _, xd = wl.vortex_mesh(g, t)
        met = mt.metrics(g, x, xd)
        J = mt.jacobian(g, x)
        P = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
        dU, dJ = rs.residual(g, w.scheme, st.pad_solution(g, P), met)
        hc = 1e-30
        xc = x + 1j * hc * xd
        rc, vc, pc, Bc = wl.vortex3d_state(xc[0], xc[1], xc[2], t + 1j * hc)
        Wc = 1.0 / np.sqrt(1.0 - np.sum(vc * vc, axis=0))
        Uc = ph.cons(ph.full_prim(rc, Wc * vc, pc, Bc), wl.VORTEX_GAMMA)
        errs.append(np.mean(np.abs((dU - np.real(Uc) * dJ) / J - np.imag(Uc) / hc)))
    return np.array(errs)


def test_rmhd_vortex3d_ec_on_prescribed_moving_mesh():
    # the 3D vortex (a Lorentz boost of the 2D rest-frame vortex along (1, 1, 1)) is an
    # exact solution: the EC residual with the nested 3D metrics and the temporal
    # metrics of the moving mesh tends to it at the design order 6 (observed 4.5 from
    # 24 to 32, 5.1 from 32 to 48 nodes per unit side, rising)
    e = _vortex3d_errors((32, 48))
    rate = np.log(e[0] / e[1]) / np.log(1.5)
    assert rate > 4.8, (e, rate)


def test_rmhd_vortex_ec_fourth_order_p2():
    # p = 2: the 4th-order EC residual (pair coefficients 4/3, -1/6, metrics of the
    # same order) converges to the vortex's time derivative at order 4
    e = _vortex_errors(0, (24, 48, 96), order=2)
    rates = np.log2(e[:-1] / e[1:])
    assert rates[-1] > 3.7, (e, rates)
