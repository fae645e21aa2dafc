"""Pins for the ES dissipation ingredients (Section 4): rotation, scaled
eigenvectors, WENO and the sign switch."""
import numpy as np
import pytest

from oracle import physics as ph, dissipation as ds
from oracle_util import rand_P

G = 5.0 / 3.0
CASES = [(ph.RHD, 2), (ph.RHD, 3), (ph.RMHD, 2)]


def test_rotation_orthogonal_first_row_normal():
    rng = np.random.default_rng(0)
    n = rng.normal(size=(3, 500))
    n[:, :3] = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0]]).T
    n /= np.linalg.norm(n, axis=0)
    T = ds.rotation(n)
    I = np.einsum("nab,ncb->nac", T, T)
    np.testing.assert_allclose(I, np.broadcast_to(np.eye(3), I.shape), atol=1e-14)
    np.testing.assert_allclose(T[:, 0, :], n.T, atol=0)
    # determinant +1 (a rotation, as the paper's T_0)
    np.testing.assert_allclose(np.linalg.det(T), 1.0, atol=1e-14)


def _A0_and_S(Pr, phys, dim):
    """A0 = dU/dV and S = dF_1/dV (+ Godunov-Powell term) by complex step through the
    explicit inverse V -> P (physics.prim_from_entropy_vars, pinned by its round
    trip in test_oracle_pins), a route independent of the oracle's primitive one."""
    sel = ph.comps(phys, dim)
    V = ph.entropy_vars(Pr, G)
    N = Pr.shape[1]
    m = len(sel)
    A0 = np.zeros((N, m, m))
    S = np.zeros((N, m, m))
    h = 1e-30
    Phip = ph.phi_prime(Pr, G)
    for b, sb in enumerate(sel):
        Vc = V.astype(complex)
        Vc[sb] += 1j * h
        Pc = ph.prim_from_entropy_vars(Vc, G)
        A0[:, :, b] = (ph.cons(Pc, G)[sel].imag / h).T
        S[:, :, b] = (ph.flux(Pc, G, 0)[sel].imag / h).T
    if phys == ph.RMHD:
        # S + Phi' (dB_1/dV): dB_1/dV is row B_1 of A0
        S = S + np.einsum("an,nb->nab", Phip[sel], A0[:, 5, :])
    return A0, S


@pytest.mark.parametrize("phys,dim", CASES)
def test_scaled_eigenvectors_definition(phys, dim):
    # dU/dV = R R^T and dF_1/dU R = R Lambda
    rng = np.random.default_rng(1 + phys + dim)
    Pr = rand_P(400, rng, phys, dim, vmax=0.95, lo=0.05)
    lam, R = ds.eigensystem(Pr, G, phys, dim)
    A0, S = _A0_and_S(Pr, phys, dim)
    RRt = np.einsum("nab,ncb->nac", R, R)
    rel = np.max(np.abs(RRt - A0), axis=(1, 2)) / np.max(np.abs(A0), axis=(1, 2))
    assert np.max(rel) < 1e-10
    A = np.einsum("nab,nbc->nac", S, np.linalg.inv(A0))
    AR = np.einsum("nab,nbc->nac", A, R)
    RL = R * lam[:, None, :]
    rel = np.max(np.abs(AR - RL), axis=(1, 2)) / np.max(np.abs(R), axis=(1, 2))
    assert np.max(rel) < 1e-8


@pytest.mark.parametrize("phys,dim", CASES)
def test_scaled_eigenvectors_near_rest(phys, dim):
    # States at rest up to rounding: velocity components of order 1e-18 (and exact
    # zeros) put entries of order 1e-50 beside entries of order one in dF/dU; the
    # eigen-structure must still satisfy its definition there.
    rng = np.random.default_rng(11 + phys + dim)
    Pr = rand_P(60, rng, phys, dim, vmax=0.5, lo=0.2)
    tiny = rng.normal(size=(3, Pr.shape[1])) * 1e-18
    tiny[:, ::3] = 0.0
    tiny[1:, 1::3] = 0.0
    Pr[1:4] = tiny
    if dim == 2:
        Pr[3] = 0.0
    Pr[3, ::5] = -5.6e-3 if dim == 3 else 0.0
    lam, R = ds.eigensystem(Pr, G, phys, dim)
    A0, S = _A0_and_S(Pr, phys, dim)
    RRt = np.einsum("nab,ncb->nac", R, R)
    rel = np.max(np.abs(RRt - A0), axis=(1, 2)) / np.max(np.abs(A0), axis=(1, 2))
    assert np.max(rel) < 1e-10
    A = np.einsum("nab,nbc->nac", S, np.linalg.inv(A0))
    AR = np.einsum("nab,nbc->nac", A, R)
    rel = np.max(np.abs(AR - R * lam[:, None, :]), axis=(1, 2)) / np.max(np.abs(R), axis=(1, 2))
    assert np.max(rel) < 1e-8


def _degenerate_rmhd_states(rng, n=40):
    """States with exactly coinciding RMHD eigenvalues in the x_1 direction: field
    along the normal (Alfven and slow or fast waves coincide), field across it
    (Alfven and slow speeds equal v_n), no field, and states at rest."""
    Pr = rand_P(4 * n, rng, ph.RMHD, 2, vmax=0.6, lo=0.2)
    Pr[6:8, :n] = 0.0                     # B along the normal
    Pr[5, n:2 * n] = 0.0                  # B across the normal
    Pr[5:8, 2 * n:3 * n] = 0.0            # no field
    Pr[1:4, 3 * n:] = 0.0                 # at rest, B along the normal
    Pr[6:8, 3 * n:] = 0.0
    return Pr


def test_rmhd_eigenstructure_at_degenerate_states():
    rng = np.random.default_rng(17)
    Pr = _degenerate_rmhd_states(rng)
    lam, R = ds.eigensystem(Pr, G, ph.RMHD, 2)
    assert np.all(np.isfinite(R))
    A0, S = _A0_and_S(Pr, ph.RMHD, 2)
    RRt = np.einsum("nab,ncb->nac", R, R)
    rel = np.max(np.abs(RRt - A0), axis=(1, 2)) / np.max(np.abs(A0), axis=(1, 2))
    assert np.max(rel) < 1e-10
    # inside a group the eigenvalues differ by at most 7 GROUP_TOL (chains), and the
    # canonical columns mix their eigenvectors: A R = R Lambda up to that spread
    # (a field along the normal is only nearly degenerate when v has a transverse
    # part: the fluid-frame field b then has one)
    A = np.einsum("nab,nbc->nac", S, np.linalg.inv(A0))
    AR = np.einsum("nab,nbc->nac", A, R)
    rel = np.max(np.abs(AR - R * lam[:, None, :]), axis=(1, 2)) / np.max(np.abs(R), axis=(1, 2))
    assert np.max(rel) < 7 * ds.GROUP_TOL
    spread = np.max(np.abs(lam[:, :, None] - lam[:, None, :]) * (np.abs(lam[:, :, None] - lam[:, None, :])
                                                                  <= ds.GROUP_TOL), axis=(1, 2))
    exact = spread < 1e-13
    assert exact.sum() > 40 and np.max(rel[exact]) < 1e-8


@pytest.mark.parametrize("degenerate", [False, True])
def test_rmhd_group_basis_does_not_depend_on_the_eigensolver_basis(degenerate):
    # rotate the eigenvectors inside every group of equal eigenvalues (and flip
    # signs of single ones): the canonical columns must not change
    rng = np.random.default_rng(23)
    Pr = _degenerate_rmhd_states(rng) if degenerate else rand_P(200, rng, ph.RMHD, 2, vmax=0.9, lo=0.05)
    sel = ph.comps(ph.RMHD, 2)
    JU = ds._jac(lambda P: ph.cons(P, G), Pr, sel, G)
    JF = ds._jac(lambda P: ph.flux(P, G, 0), Pr, sel, G).copy()
    JF[:, :, 5] += ph.phi_prime(Pr, G)[sel].T
    JV = ds._jac(lambda P: ph.entropy_vars(P, G), Pr, sel, G)
    X = np.linalg.inv(JV)
    A0 = JU @ X
    S = JF @ X
    A0 = 0.5 * (A0 + np.transpose(A0, (0, 2, 1)))
    S = 0.5 * (S + np.transpose(S, (0, 2, 1)))
    L = np.linalg.cholesky(A0)
    Li = np.linalg.inv(L)
    Q = Li @ S @ np.transpose(Li, (0, 2, 1))
    lam, Z = np.linalg.eigh(0.5 * (Q + np.transpose(Q, (0, 2, 1))))
    vn = Pr[1] / np.sqrt(1.0 + Pr[1] ** 2 + Pr[2] ** 2 + Pr[3] ** 2)
    R1 = ds.canonical_group_basis(lam, Z, L, Li, vn)
    Z2 = Z.copy()
    for n in range(Z.shape[0]):
        i = 0
        while i < 8:
            j = i
            while j + 1 < 8 and lam[n, j + 1] - lam[n, j] <= ds.GROUP_TOL:
                j += 1
            k = j - i + 1
            Qr, _ = np.linalg.qr(rng.normal(size=(k, k)))
            Z2[n, :, i:j + 1] = Z[n, :, i:j + 1] @ Qr
            i = j + 1
    R2 = ds.canonical_group_basis(lam, Z2, L, Li, vn)
    assert np.max(np.abs(R1 - R2)) <= 1e-10 * np.max(np.abs(R1))


@pytest.mark.parametrize("phys,dim", CASES)
def test_cluster_basis_is_canonical(phys, dim):
    # seeds in order; each later cluster column carries no component of an earlier seed:
    # r_q^T A0^{-1} e_{s_j} = 0 for j < q (so the basis does not depend on how the
    # eigenspace was computed), and the cluster columns have eigenvalue v_n.
    rng = np.random.default_rng(7 + phys + dim)
    Pr = rand_P(300, rng, phys, dim, vmax=0.9, lo=0.05)
    lam, R = ds.eigensystem(Pr, G, phys, dim)
    A0, _ = _A0_and_S(Pr, phys, dim)
    A0i = np.linalg.inv(A0)
    vn = Pr[1] / np.sqrt(1 + Pr[1] ** 2 + Pr[2] ** 2 + Pr[3] ** 2)
    seeds = ds.cluster_seeds(phys, dim)
    for n in range(Pr.shape[1]):
        cl = np.argsort(np.abs(lam[n] - vn[n]))[:len(seeds)]
        np.testing.assert_allclose(lam[n][cl], vn[n], atol=1e-14)
        # M[q, j] = r_q^T A0^{-1} e_{s_j}: r_q is built from seed s_q, so M[q, j] = 0 for j < q
        M = (R[n][:, cl].T @ A0i[n])[:, seeds]
        M = np.abs(M) / np.max(np.abs(M))
        order = np.argsort(-np.sum(M > 1e-7, axis=1), kind="stable")
        assert np.all(np.tril(M[order], -1) < 1e-9), M


def test_weno5_linear_weights_exact_for_quartics():
    # With eps -> infinity the JS weights become the linear ones.  Read as cell averages
    # of H, point data of a quartic H' reconstruct H' at x_{i+1/2} exactly from both sides,
    # so <<v>> = v^+ - v^- vanishes for point samples of any quartic and not of a quintic.
    rng = np.random.default_rng(2)
    x = np.arange(-2, 4) * 1.0
    for deg in range(6):
        c = rng.normal(size=deg + 1)
        Hc = np.polyint(c)
        v = np.polyval(Hc, x + 0.5) - np.polyval(Hc, x - 0.5)      # cell averages of c
        vm = ds.weno5_minus(v[0], v[1], v[2], v[3], v[4], 1e30)
        vp = ds.weno5_minus(v[5], v[4], v[3], v[2], v[1], 1e30)
        exact = np.polyval(c, 0.5)
        if deg <= 4:
            assert abs(vm - exact) < 1e-12 * (1 + abs(exact))
            assert abs(vp - exact) < 1e-12 * (1 + abs(exact))
        w = np.polyval(c, x)                                         # point samples
        jm = ds.weno5_minus(w[0], w[1], w[2], w[3], w[4], 1e30)
        jp = ds.weno5_minus(w[5], w[4], w[3], w[2], w[1], 1e30)
        if deg <= 4:
            assert abs(jp - jm) < 1e-12 * (1 + np.max(np.abs(w)))
        else:
            assert abs(jp - jm) > 1e-6


def test_weno5_jump_fifth_order_on_smooth_data():
    errs = []
    for n in (20, 40, 80, 160):
        h = 1.0 / n
        x = (np.arange(-2, 4) * h)[:, None] + np.linspace(0, 1, 50)[None, :]
        v = np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x)
        vm = ds.weno5_minus(v[0], v[1], v[2], v[3], v[4], 1e-6)
        vp = ds.weno5_minus(v[5], v[4], v[3], v[2], v[1], 1e-6)
        errs.append(np.max(np.abs(vp - vm)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 4.5, (errs, rates)


def test_weno5_odd_symmetry():
    rng = np.random.default_rng(3)
    v = rng.normal(size=(5, 1000))
    a = ds.weno5_minus(*v, 1e-6)
    b = ds.weno5_minus(*(-v), 1e-6)
    np.testing.assert_allclose(a, -b, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("phys,dim", CASES)
def test_sign_property_and_constant_state(phys, dim):
    rng = np.random.default_rng(4 + phys + dim)
    N = 500
    Pst = np.stack([rand_P(N, rng, phys, dim, vmax=0.9, lo=0.05) for _ in range(6)])
    ast = rng.normal(size=(2, dim + 1, N))
    d, info = ds.face_dissipation(Pst, ast, G, phys, dim, 1e-6, details=True)
    prod = info["jump"] * info["Y"] * info["jump_weno"]
    assert np.all(prod >= 0)       # [V~]^T Y <<V~>> >= 0 per component (Theorem 5.1)
    # constant state: no dissipation (Remark after Theorem 5.1)
    Pc = np.repeat(Pst[:1], 6, axis=0)
    dc = ds.face_dissipation(Pc, ast, G, phys, dim, 1e-6)
    assert np.max(np.abs(dc)) == 0.0


def test_weno3_exact_on_linear_data_and_third_order():
    # WENO3-JS (w = 2p - 1 for p = 2) reconstructs the value at x_{i+1/2} from the
    # cell averages of cells i-1, i, i+1 (in the finite-difference form the point
    # values play their role): both candidates reproduce linear data, so the value
    # is exact there; on a smooth monotone profile the error falls at third order
    a, b, c = 0.3, 0.7, 1.1
    assert abs(ds.weno3_minus(a, b, c, 1e-6) - 0.9) < 1e-15
    avg = lambda x, h: (np.exp(x + 0.5 * h) - np.exp(x - 0.5 * h)) / h   # cell averages of exp
    errs = []
    x0 = 0.3
    for h in (0.1, 0.05, 0.025, 0.0125):
        v = ds.weno3_minus(avg(x0 - h, h), avg(x0, h), avg(x0 + h, h), 1e-6)
        errs.append(abs(v - np.exp(x0 + 0.5 * h)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[-1] > 2.7, (errs, rates)


def _decisions(g, scheme, P, x, xdot):
    from oracle import metrics as mt, residual as rs, stepper as st
    met = mt.metrics(g, x, xdot, scheme.order_p)
    return rs.residual(g, scheme, st.pad_solution(g, P), met, details=True)


@pytest.mark.parametrize("case", ["separated", "rotor"])
def test_rmhd_group_decisions_stable_under_rounding(case):
    # The grouping of nearly equal eigenvalues (GROUP_TOL) and the seed acceptance
    # (SEED_TOL) are discontinuous in the state.  Under a 1e-15 relative perturbation
    # of the input no face changes either decision, neither at well-separated states
    # nor at the rotor's exactly degenerate ones; so the oracle's sensitivity at
    # random states comes from eigenvectors of close but ungrouped eigenvalues, and at
    # well-separated states the residual moves by rounding only.
    from paper_2107_12027_amd import workloads as wl
    rng = np.random.default_rng(33)
    if case == "separated":
        g = wl.make_grid(2, (40, 36, 1), (0, 0, 0))
        x = wl.perturbed_mesh(g, rng, amp=0.03)
        xdot = wl.perturbed_mesh(g, rng, amp=0.05) - wl.uniform_mesh(g)
        pr = wl.smooth_prim(x, rng, wl.RMHD)
        B = np.array([0.6, 0.45, 0.35])[:, None, None] + 0.1 * pr["B"]
        P = ph.full_prim(pr["rho"], pr["u"], pr["p"], B)
    else:
        w = wl.rmhd_rotor(n=40)
        g, x, xdot = w.grid, w.x, None
        P = ph.full_prim(w.prim["rho"], w.prim["u"], w.prim["p"], w.prim["B"])
    scheme = wl.Scheme(phys=wl.RMHD)
    dU0, _, i0 = _decisions(g, scheme, P, x, xdot)
    P1 = P * (1 + 1e-15 * rng.uniform(-1, 1, size=P.shape))
    dU1, _, i1 = _decisions(g, scheme, P1, x, xdot)
    gaps = []
    for k in range(g.dim):
        assert np.array_equal(i0[k]["groups"]["labels"], i1[k]["groups"]["labels"])
        assert np.array_equal(i0[k]["groups"]["seeds"], i1[k]["groups"]["seeds"])
        gaps.append(np.sort(np.diff(np.sort(i0[k]["lam"], axis=1), axis=1), axis=1)[:, 1].min())
    if case == "separated":
        assert min(gaps) > 1e-3
        scale = np.abs(dU0).reshape(dU0.shape[0], -1).max(axis=1)
        assert np.max(np.abs(dU1 - dU0).reshape(dU0.shape[0], -1).max(axis=1) / scale) < 1e-12
    else:
        assert min(gaps) == 0.0        # exactly degenerate groups are present


# ---------------------------------------------------------------------------
# WENO7 (w = 2p - 1 for p = 4) from the WENO-JS definition: the generic
# construction must reproduce the published WENO5 and WENO3 closed forms, and
# WENO7 must show its design properties
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r,closed", [(3, "weno5_minus"), (2, "weno3_minus")])
def test_weno_definition_reproduces_published_weno5_and_weno3(r, closed):
    rng = np.random.default_rng(40 + r)
    v = rng.normal(size=(2 * r - 1, 2000)) * rng.uniform(0.01, 10, size=2000)
    for eps in (1e-6, 1e-2, 1e30):
        a = ds.weno_js_minus(list(v), eps)
        b = getattr(ds, closed)(*v, eps)
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13 * np.max(np.abs(v)))


def test_weno7_published_tables():
    # Balsara and Shu (2000): linear weights and candidate coefficients
    from fractions import Fraction as Fr
    c, B, d = ds.weno_js_tables(4)
    assert d == [Fr(1, 35), Fr(12, 35), Fr(18, 35), Fr(4, 35)]
    assert c[0] == [Fr(-3, 12), Fr(13, 12), Fr(-23, 12), Fr(25, 12)]
    assert c[3] == [Fr(3, 12), Fr(13, 12), Fr(-5, 12), Fr(1, 12)]
    # the indicator of the first candidate: 240 beta_0 = v0 (547 v0 - 3882 v1 + 4642 v2 - 1854 v3)
    # + v1 (7043 v1 - 17246 v2 + 7042 v3) + v2 (11003 v2 - 9402 v3) + 2107 v3^2
    Q = [[240 * x for x in row] for row in B[0]]
    assert [Q[0][0], 2 * Q[0][1], 2 * Q[0][2], 2 * Q[0][3]] == [547, -3882, 4642, -1854]
    assert [Q[1][1], 2 * Q[1][2], 2 * Q[1][3], Q[2][2], 2 * Q[2][3], Q[3][3]] == [7043, -17246, 7042, 11003, -9402, 2107]


def test_weno7_linear_weights_exact_for_degree_six():
    rng = np.random.default_rng(5)
    x = np.arange(-3, 5) * 1.0
    for deg in range(8):
        c = rng.normal(size=deg + 1)
        Hc = np.polyint(c)
        v = np.polyval(Hc, x + 0.5) - np.polyval(Hc, x - 0.5)      # cell averages of c
        vm = ds.weno_minus(list(v[0:7]), 1e30)
        vp = ds.weno_minus(list(v[7:0:-1]), 1e30)
        exact = np.polyval(c, 0.5)
        if deg <= 6:
            assert abs(vm - exact) < 1e-11 * (1 + abs(exact))
            assert abs(vp - exact) < 1e-11 * (1 + abs(exact))
        w = np.polyval(c, x)                                         # point samples
        jm = ds.weno_minus(list(w[0:7]), 1e30)
        jp = ds.weno_minus(list(w[7:0:-1]), 1e30)
        if deg <= 6:
            assert abs(jp - jm) < 1e-11 * (1 + np.max(np.abs(w)))
        else:
            assert abs(jp - jm) > 1e-6


def test_weno7_jump_seventh_order_on_smooth_data():
    # (JS weights with eps = 1e-6 cost some accuracy near the extrema on coarse
    # meshes: rates 5.0, 6.1, 6.4, 7.2 from 10 to 160 points per period)
    errs = []
    for n in (40, 80, 160):
        h = 1.0 / n
        x = (np.arange(-3, 5) * h)[:, None] + np.linspace(0, 1, 50)[None, :]
        v = np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x)
        vm = ds.weno_minus(list(v[0:7]), 1e-6)
        vp = ds.weno_minus(list(v[7:0:-1]), 1e-6)
        errs.append(np.max(np.abs(vp - vm)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 6.8, (errs, rates)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_weno_indicators_as_sums_of_squares(r):
    # beta_k evaluated as sum_m D_m (w_km . v)^2 is the definition's quadratic form
    # exactly (rational arithmetic), each square is of differences (w_km annihilates
    # constants), and for r = 3 the factors are the 13/12 and 1/4 of WENO5-JS
    from fractions import Fraction as Fr
    c, B, d = ds.weno_js_tables(r)
    D, W = ds.weno_js_squares(r)
    for k in range(r):
        for a in range(r):
            for b in range(r):
                assert sum(D[m] * W[k][m][a] * W[k][m][b] for m in range(r - 1)) == B[k][a][b]
        for m in range(r - 1):
            assert sum(W[k][m]) == 0
    if r == 3:
        assert D == [Fr(1), Fr(13, 3)]
    if r == 4:
        assert D == [Fr(1), Fr(13, 3), Fr(781, 20)]


def test_weno7_indicators_stable_on_smooth_data():
    # on smooth data of size 1 with variations of 1e-3 (beta ~ 1e-7) the expanded
    # quadratic form loses about eight digits of beta (1e-8 relative); the sum of
    # squares keeps all but about three (1e-12), against 50-digit evaluation of the
    # exact rational form
    import mpmath
    mpmath.mp.dps = 50
    c, B, d = ds.weno_js_tables(4)
    D, W = ds.weno_js_squares(4)
    q = lambda f: mpmath.mpf(f.numerator) / f.denominator
    x = 1.0 + 1e-3 * np.sin(np.arange(-3, 4) * 0.37 + 0.2)
    worst_sq, worst_exp = 0.0, 0.0
    for k in range(4):
        S = x[k:k + 4]
        exact = float(sum(q(D[m]) * mpmath.fsum(q(W[k][m][j]) * mpmath.mpf(S[j]) for j in range(4)) ** 2
                          for m in range(3)))
        sq = sum(float(D[m]) * sum(float(W[k][m][j]) * S[j] for j in range(4)) ** 2 for m in range(3))
        ex = sum(float(B[k][a][b]) * S[a] * S[b] for a in range(4) for b in range(4))
        worst_sq = max(worst_sq, abs(sq - exact) / exact)
        worst_exp = max(worst_exp, abs(ex - exact) / exact)
    assert worst_sq < 1e-11 and worst_exp > 1e-9, (worst_sq, worst_exp)
