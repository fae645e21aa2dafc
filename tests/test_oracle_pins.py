"""Pins for the oracle parts that the face dissipation and the CFL step rest on,
each checked against something other than the oracle itself:

* the explicit inverse of the entropy-variable map (the face state of eq.
  ESFlux_HO is the state whose entropy variables are the mean of the two nodes')
  against the forward map V(P) of Section 2, which test_oracle_physics pins by
  complex-step differentiation of the entropy;
* lambda^ = max_m |J dxi_k/dt + L_k lambda_m(T U)| of eq. ESFlux_HO against the
  textbook closed-form RHD speeds and, for RMHD, the fast magnetosonic roots of
  the textbook characteristic quartic, found here by plain bisection;
* the scale of the whole dissipation term (the factor 1/2 of eq. ESFlux_HO,
  D = lambda^ T^{-1} R(TU), and R R^T = dU/dV): in its first-order limit (WENO
  values equal to the two face nodes, Y = I) the flux difference between the ES
  and the EC residual at a single jump is lambda^ [U] / 2 up to O(|[V]|^3), the
  midpoint rule for [U] = int dU/dV dV along the straight path in V;
* the RMHD spectral radius of eq. cfl (numeric eigenvalues of the
  Godunov-Powell modified Jacobian) against the same quartic.
"""
import numpy as np
import pytest

from oracle import dissipation as ds
from oracle import metrics as mt
from oracle import physics as ph
from oracle import residual as rs
from oracle import stepper as st
from oracle_util import rand_P
from paper_2107_12027_amd import workloads as wl

G = 5.0 / 3.0


# ---------------------------------------------------------------------------
# textbook characteristic speeds (written out here, independent of the oracle)
# ---------------------------------------------------------------------------

def _fast_quartic(P, n):
    """Characteristic quartic of ideal RMHD for waves with normal n (Anile 1989):
        Q(lam) = rho h (1 - cs^2) a^4 - (1 - lam^2) [(|b|^2 + rho h cs^2) a^2 - cs^2 Bt^2],
    a = W (lam - v.n), Bt = b.n - lam b^0, cs^2 = Gamma p / (rho h), with the
    four-vector b^mu = (W v.B, B/W + W (v.B) v).  Its outermost roots are the fast
    magnetosonic speeds; for B = 0 they are the sound speeds.  Returns Q as a
    function of lam for one state (P an 8-vector, n a unit 3-vector)."""
    rho, u, p, B = P[0], P[1:4], P[4], P[5:8]
    W = np.sqrt(1.0 + u @ u)
    v = u / W
    vB = v @ B
    b0 = W * vB
    b = B / W + W * vB * v
    bsq = B @ B / (W * W) + vB * vB
    rh = rho + G / (G - 1.0) * p
    cs2 = G * p / rh
    vn, bn = v @ n, b @ n

    def Q(lam):
        a = W * (lam - vn)
        Bt = bn - lam * b0
        return rh * (1.0 - cs2) * a ** 4 - (1.0 - lam * lam) * ((bsq + rh * cs2) * a * a - cs2 * Bt * Bt)
    return Q


def _outer_roots(Q):
    """Smallest and largest root of Q in (-1, 1) by a sign-change scan on a
    tanh-spaced grid followed by plain bisection."""
    lam = np.tanh(np.linspace(-12.0, 12.0, 40001))
    q = Q(lam)
    idx = np.nonzero(np.sign(q[:-1]) != np.sign(q[1:]))[0]
    assert len(idx) >= 2, "expected the two fast roots"

    def bisect(lo, hi):
        qlo = Q(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid == lo or mid == hi:
                break
            qm = Q(mid)
            if np.sign(qm) == np.sign(qlo):
                lo, qlo = mid, qm
            else:
                hi = mid
        return 0.5 * (lo + hi)
    return bisect(lam[idx[0]], lam[idx[0] + 1]), bisect(lam[idx[-1]], lam[idx[-1] + 1])


def _rhd_speeds(P, n):
    """Closed-form RHD speeds (physics.eigen_speeds_rhd, the textbook formula)."""
    return np.stack(ph.eigen_speeds_rhd(P, G, n))


def _unit(rng, N, dim):
    n = np.zeros((3, N))
    n[:dim] = rng.normal(size=(dim, N))
    return n / np.linalg.norm(n, axis=0)


# ---------------------------------------------------------------------------
# 1. the entropy-variable inverse
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("phys,dim", [(ph.RHD, 2), (ph.RHD, 3), (ph.RMHD, 2)])
def test_prim_from_entropy_vars_round_trip(phys, dim):
    rng = np.random.default_rng(11 + 3 * phys + dim)
    P = rand_P(2000, rng, phys, dim, vmax=0.99, lo=0.01)
    # near-rest states (|u| down to 1e-12) and, for RMHD, fields along and across v
    P[1:4, :200] *= 10.0 ** rng.uniform(-12, -3, size=200)
    if phys == ph.RMHD:
        P[5:8, 200:300] = P[1:4, 200:300] * rng.uniform(-3, 3, size=100)
        P[5:8, 300:400] *= 10.0 ** rng.uniform(-12, -2, size=100)
    Q = ph.prim_from_entropy_vars(ph.entropy_vars(P, G), G)
    sel = [0, 1, 2, 3, 4, 5, 6, 7] if phys == ph.RMHD else [0, 1, 2, 3, 4]
    scale = np.maximum(np.abs(P[sel]), 1.0)
    assert np.max(np.abs(Q[sel] - P[sel]) / scale) < 1e-12
    if phys == ph.RHD:
        assert np.max(np.abs(Q[5:8])) == 0.0


# ---------------------------------------------------------------------------
# 2. lambda^ against the textbook speeds
# ---------------------------------------------------------------------------

def _face_case(rng, phys, dim, N):
    """Stencils of 6 random states (p = 3) and random node metrics with a_t != 0."""
    Pst = np.stack([rand_P(N, rng, phys, dim, vmax=0.95, lo=0.05) for _ in range(6)])
    ast = np.zeros((2, dim + 1, N))
    base = rng.normal(size=(dim + 1, N))
    base[0] = rng.choice([-1.0, 1.0], size=N) * rng.uniform(0.5, 3.0, size=N)   # a_t away from 0
    for s in range(2):
        ast[s] = base + 0.1 * rng.normal(size=(dim + 1, N))
    return Pst, ast


@pytest.mark.parametrize("phys,dim", [(ph.RHD, 2), (ph.RHD, 3), (ph.RMHD, 2)])
def test_lambda_hat_against_textbook_speeds(phys, dim):
    rng = np.random.default_rng(5 + 7 * phys + dim)
    N = 60
    Pst, ast = _face_case(rng, phys, dim, N)
    _, info = ds.face_dissipation(Pst, ast, G, phys, dim, 1e-6, details=True)
    abar = 0.5 * (ast[0] + ast[1])
    ax = np.zeros((3, N))
    ax[:dim] = abar[1:]
    L = np.linalg.norm(ax, axis=0)
    n = ax / L
    # face state: entropy variables averaged, mapped back by the pinned inverse
    Pf = ph.prim_from_entropy_vars(0.5 * (ph.entropy_vars(Pst[2], G) + ph.entropy_vars(Pst[3], G)), G)
    if phys == ph.RHD:
        Pf[5:8] = 0.0
        lam = _rhd_speeds(Pf, n)                                  # (3, N)
        lo, hi = lam[0], lam[2]
    else:
        lo, hi = np.zeros(N), np.zeros(N)
        for f in range(N):
            lo[f], hi[f] = _outer_roots(_fast_quartic(Pf[:, f], n[:, f]))
    want = np.maximum(np.abs(abar[0] + L * lo), np.abs(abar[0] + L * hi))
    assert np.all(np.abs(abar[0]) > 0.1)          # the temporal metric matters here
    np.testing.assert_allclose(info["lhat"], want, rtol=1e-9, atol=0)


# ---------------------------------------------------------------------------
# 3. the scale of the dissipation term through its first-order limit
# ---------------------------------------------------------------------------

def _jump_case(phys, delta, nx=16, ny=8):
    """2D grid with outflow axes, affine skew mesh (metric normals not along the
    axes, |J grad xi| != 1), constant mesh velocity (J dxi/dt != 0); state P_a on
    nodes i < nx/2 and P_b = P_a + delta * (a fixed direction) beyond, constant
    along xi_2."""
    g = wl.make_grid(2, (nx, ny, 1), (wl.OUTFLOW, wl.OUTFLOW, wl.PERIODIC))
    xi1 = np.arange(nx) / (nx - 1)
    xi2 = np.arange(ny) / (ny - 1)
    E2, E1 = np.meshgrid(xi2, xi1, indexing="ij")
    A = np.array([[2.0, 0.5], [0.3, 3.0]])           # x = A xi
    x = np.stack([A[0, 0] * E1 + A[0, 1] * E2, A[1, 0] * E1 + A[1, 1] * E2])
    xdot = np.zeros_like(x)
    xdot[0] = 0.7
    xdot[1] = -0.4
    Pa = np.array([0.8, 0.3, -0.2, 0.1 if phys == ph.RMHD else 0.0, 0.6, 0.0, 0.0, 0.0])
    dP = np.array([0.5, -0.7, 0.4, 0.3 if phys == ph.RMHD else 0.0, 0.9, 0.0, 0.0, 0.0])
    if phys == ph.RMHD:
        Pa[5:8] = [0.4, -0.3, 0.5]
        dP[5:8] = [0.6, 0.2, -0.5]
    Pb = Pa + delta * dP
    P = np.zeros((8,) + g.shape)
    P[:, :, : nx // 2] = Pa[:, None, None]
    P[:, :, nx // 2:] = Pb[:, None, None]
    return g, x, xdot, P, Pa, Pb


@pytest.mark.parametrize("phys", [ph.RHD, ph.RMHD])
def test_dissipation_scale_first_order_limit(phys):
    errs = []
    for delta in (4e-3, 2e-3):
        g, x, xdot, P, Pa, Pb = _jump_case(phys, delta)
        # weno_eps tiny: a constant sub-stencil gets all the weight, so the WENO values at
        # the jump face are the two face nodes' and vanish elsewhere
        base = wl.Scheme(phys=phys, order_p=3, weno_eps=1e-40)
        met = mt.metrics(g, x, xdot, 3)
        Ppad = st.pad_solution(g, P)
        dU_ec, _ = rs.residual(g, wl.Scheme(phys=phys, order_p=3, dissipation=0), Ppad, met)
        _, _, info = rs.residual(g, base, Ppad, met, details=True)
        ones = {k: np.ones_like(info[k]["Y"]) for k in info}
        dU_es, _ = rs.residual(g, base, Ppad, met, Y_fixed=ones)
        diff = dU_es - dU_ec                            # (m, ny, nx)
        i = g.n[0] // 2 - 1                             # the node left of the jump
        # lambda^ at the jump face from the textbook speeds (metrics: constant, affine mesh)
        a = mt.metrics(g, x, xdot, 3)[:, 3, 3 + i]      # direction-1 metrics of a node
        at, ax = a[0], np.array([a[1], a[2], 0.0])
        L = np.linalg.norm(ax)
        n = ax / L
        Pf = ph.prim_from_entropy_vars(0.5 * (ph.entropy_vars(Pa, G) + ph.entropy_vars(Pb, G)), G)
        if phys == ph.RHD:
            lo, _, hi = ph.eigen_speeds_rhd(Pf[:, None], G, n[:, None])
            lo, hi = float(lo[0]), float(hi[0])
        else:
            lo, hi = _outer_roots(_fast_quartic(Pf, n))
        lhat = max(abs(at + L * lo), abs(at + L * hi))
        sel = ph.comps(phys, 2)
        jumpU = (ph.cons(Pb[:, None], G) - ph.cons(Pa[:, None], G))[sel, 0]
        want = lhat * jumpU / (2.0 * g.dxi[0])
        # no dissipation away from the jump face; node i and i+1 get +-lambda^ [U] / (2 dxi)
        assert np.max(np.abs(np.delete(diff, [i, i + 1], axis=2))) < 1e-9 * np.max(np.abs(want))
        got_l = diff[:, :, i]
        got_r = diff[:, :, i + 1]
        assert np.max(np.abs(got_l - got_l[:, :1])) < 1e-12 * np.max(np.abs(want))
        err = max(np.max(np.abs(got_l[:, 0] - want)), np.max(np.abs(got_r[:, 0] + want)))
        errs.append(err / np.max(np.abs(want)))
    # second order in the jump (midpoint-rule error of O(|[V]|^3) against [U] = O(|[V]|))
    assert errs[0] < 5e-5, errs
    assert errs[0] / errs[1] > 3.0, errs


# ---------------------------------------------------------------------------
# 4. the RMHD spectral radius of the CFL step
# ---------------------------------------------------------------------------

def test_rmhd_numeric_speeds_fast_magnetosonic():
    rng = np.random.default_rng(23)
    N = 80
    P = rand_P(N, rng, ph.RMHD, 2, vmax=0.95, lo=0.05)
    lam = st.speeds(P, G, ph.RMHD, 2)                    # normal frame, direction x
    ex = np.array([1.0, 0.0, 0.0])
    for f in range(N):
        lo, hi = _outer_roots(_fast_quartic(P[:, f], ex))
        assert abs(np.max(lam[f]) - hi) < 1e-9 and abs(np.min(lam[f]) - lo) < 1e-9, (f, lam[f], lo, hi)


def test_rmhd_spectral_radius_curvilinear():
    # rho_{k,i} = L_k max_m |lambda_m(n_k)| / J_i on a smoothly perturbed mesh
    rng = np.random.default_rng(29)
    g = wl.make_grid(2, (12, 10, 1), (wl.PERIODIC, wl.PERIODIC, wl.PERIODIC))
    x = wl.perturbed_mesh(g, rng, amp=0.03)
    pr = wl.random_prim(g.shape, rng, phys=wl.RMHD, dim=2, vmax=0.9)
    P = ph.full_prim(pr["rho"], pr["u"], pr["p"], pr["B"])
    met = mt.metrics(g, x, None, 3)
    J = mt.jacobian(g, x, 3)
    scheme = wl.Scheme(phys=wl.RMHD)
    rho = st.spectral_radius(g, scheme, P, met, J)
    Pf = P.reshape(8, -1)
    for k in range(2):
        a = rs.interior(met[k * 3:(k + 1) * 3], g).reshape(3, -1)
        for node in range(0, Pf.shape[1], 7):
            ax = np.array([a[1, node], a[2, node], 0.0])
            L = np.linalg.norm(ax)
            lo, hi = _outer_roots(_fast_quartic(Pf[:, node], ax / L))
            want = L * max(abs(lo), abs(hi)) / J.reshape(-1)[node]
            assert abs(rho[k].reshape(-1)[node] - want) < 1e-9 * want
