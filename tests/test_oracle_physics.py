"""Pins for the oracle physics (Section 1 and Section 2 of the paper)."""
import numpy as np
import pytest

from oracle import physics as ph, stepper as st
from oracle_util import rand_P, cstep

G = 5.0 / 3.0
CASES = [(ph.RHD, 2), (ph.RHD, 3), (ph.RMHD, 2)]


@pytest.mark.parametrize("phys,dim", CASES)
def test_entropy_variables_are_gradient_of_entropy(phys, dim):
    # Definition 2.1: V = eta'(U)^T  <=>  d eta/dP = V^T dU/dP (chain rule)
    rng = np.random.default_rng(1)
    P = rand_P(200, rng, phys, dim, vmax=0.95)
    sel = ph.comps(phys, dim)
    V = ph.entropy_vars(P, G)[sel]
    for s in sel:
        deta = cstep(lambda Q: ph.entropy(Q, G), P, s)
        dU = cstep(lambda Q: ph.cons(Q, G), P, s)[sel]
        lhs = np.sum(V * dU, axis=0)
        np.testing.assert_allclose(lhs, deta, rtol=1e-10, atol=1e-12 * (1 + np.max(np.abs(V * dU))))


@pytest.mark.parametrize("phys,dim", CASES)
def test_entropy_flux_consistency(phys, dim):
    # eq. EntropyConsistentCond for the symmetrizable system (eq. RMHDSymm):
    # dq_k/dP = V^T dF_k/dP + Phi dB_k/dP with q_k = eta v_k.
    rng = np.random.default_rng(2)
    P = rand_P(200, rng, phys, dim, vmax=0.95)
    sel = ph.comps(phys, dim)
    V = ph.entropy_vars(P, G)[sel]
    _, _, Phi = ph.potentials(P, G)

    def q(Q, k):
        s = ph.state(Q, G)
        return ph.entropy(Q, G) * s["v"][k]

    for k in range(dim):
        for s in sel:
            dq = cstep(lambda Q: q(Q, k), P, s)
            dF = cstep(lambda Q: ph.flux(Q, G, k), P, s)[sel]
            dB = 1.0 if s == 5 + k else 0.0
            rhs = np.sum(V * dF, axis=0) + Phi * dB
            np.testing.assert_allclose(rhs, dq, rtol=1e-9, atol=1e-12 * (1 + np.max(np.abs(V * dF))))


@pytest.mark.parametrize("phys,dim", CASES)
def test_potentials_match_definitions(phys, dim):
    # eq. EntropyPotential: phi = V.U - eta, psi_k = V.F_k + Phi B_k - q_k; eq. Phi: Phi = Phi'.V
    rng = np.random.default_rng(3)
    P = rand_P(500, rng, phys, dim)
    sel = ph.comps(phys, dim)
    V = ph.entropy_vars(P, G)
    U = ph.cons(P, G)
    eta = ph.entropy(P, G)
    phi, psi, Phi = ph.potentials(P, G)
    s = ph.state(P, G)
    np.testing.assert_allclose(phi, np.sum(V[sel] * U[sel], axis=0) - eta, rtol=1e-11, atol=1e-11)
    for k in range(3):
        F = ph.flux(P, G, k)
        want = np.sum(V[sel] * F[sel], axis=0) + Phi * P[5 + k] - eta * s["v"][k]
        np.testing.assert_allclose(psi[k], want, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(np.sum(ph.phi_prime(P, G) * V, axis=0), Phi, rtol=1e-12, atol=1e-14)


def test_rhd_flux_matches_textbook_form():
    # B = 0: F_k = (D v_k, m v_k + p e_k, m_k) with m = rho h W^2 v, E = rho h W^2 - p
    rng = np.random.default_rng(4)
    P = rand_P(100, rng, ph.RHD, 3)
    s = ph.state(P, G)
    rho, v, p, W, h = s["rho"], s["v"], s["p"], s["W"], s["h"]
    U = ph.cons(P, G)
    np.testing.assert_allclose(U[0], rho * W)
    np.testing.assert_allclose(U[1:4], rho * h * W * W * v)
    np.testing.assert_allclose(U[4], rho * h * W * W - p)
    F = ph.flux(P, G, 1)
    np.testing.assert_allclose(F[2], rho * h * W * W * v[1] * v[1] + p)
    np.testing.assert_allclose(F[4], rho * h * W * W * v[1])


@pytest.mark.parametrize("dim", [2, 3])
def test_con2prim_rhd_round_trip_and_rest_state(dim):
    rng = np.random.default_rng(5)
    P = rand_P(4000, rng, ph.RHD, dim, vmax=0.99)
    sel = ph.comps(ph.RHD, dim)
    U = ph.cons(P, G)[sel]
    Q, ok = ph.con2prim_rhd(U, G, dim)
    assert ok.all()
    np.testing.assert_allclose(ph.cons(Q, G)[sel], U, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Q[[0, 4]], P[[0, 4]], rtol=1e-10)
    # v = 0: p = (Gamma - 1)(E - D)
    U0 = U.copy()
    U0[1:1 + dim] = 0.0
    Q0, ok0 = ph.con2prim_rhd(U0, G, dim)
    np.testing.assert_allclose(Q0[4], (G - 1) * (U0[-1] - U0[0]), rtol=1e-13)


def test_con2prim_rhd_flags_inadmissible():
    U = np.array([[1.0, 1.0], [0.5, 3.0], [0.0, 0.0], [2.0, 2.0]])   # second: E < sqrt(D^2+m^2)
    Q, ok = ph.con2prim_rhd(U, G, 2)
    assert ok.tolist() == [True, False]
    assert np.isnan(Q[:, 1]).all()


def test_con2prim_rmhd_round_trip():
    rng = np.random.default_rng(6)
    P = rand_P(4000, rng, ph.RMHD, 3, vmax=0.95, lo=0.05)
    U = ph.cons(P, G)
    Q, ok = ph.con2prim_rmhd(U, G)
    assert ok.all()
    np.testing.assert_allclose(ph.cons(Q, G), U, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Q, P, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_numeric_speeds_match_textbook_rhd_eigenvalues(dim):
    # the CFL spectral radius uses numeric eigenvalues; pin them to the closed form
    rng = np.random.default_rng(7)
    P = rand_P(3000, rng, ph.RHD, dim, vmax=0.99)
    lam = np.sort(st.speeds(P, G, ph.RHD, dim), axis=1)
    lm, vn, lp = ph.eigen_speeds_rhd(P, G, np.array([1.0, 0.0, 0.0])[:, None])
    want = np.sort(np.stack([lm, lp] + [vn] * (dim)).T, axis=1)
    np.testing.assert_allclose(lam, want, atol=5e-13)
