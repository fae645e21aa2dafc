"""Pins for the logarithmic mean and the two-point EC fluxes (Section 3.1)."""
import mpmath
import numpy as np
import pytest

from oracle import physics as ph, ecflux as ec
from oracle_util import rand_P

G = 5.0 / 3.0
CASES = [(ph.RHD, 2), (ph.RHD, 3), (ph.RMHD, 2)]


def test_log_mean_against_high_precision():
    mpmath.mp.dps = 50
    rng = np.random.default_rng(0)
    a = rng.uniform(0.01, 10.0, size=400)
    # ratios spanning both branches, including jumps right at the series threshold
    r = np.concatenate([1 + rng.uniform(-1e-9, 1e-9, 100), 1 + rng.uniform(-0.3, 0.3, 100),
                        np.exp(rng.uniform(-5, 5, 100)), 1 + rng.uniform(0.18, 0.25, 100)])
    b = a * r
    got = ec.log_mean(a, b)
    for i in range(len(a)):
        x, y = mpmath.mpf(a[i]), mpmath.mpf(b[i])
        want = (x - y) / (mpmath.log(x) - mpmath.log(y)) if x != y else x
        assert abs(got[i] - float(want)) <= 4e-16 * float(want), (a[i], b[i], got[i], float(want))
    np.testing.assert_allclose(ec.log_mean(a, b), ec.log_mean(b, a), rtol=5e-16)
    np.testing.assert_allclose(ec.log_mean(a, a), a, rtol=2e-16)


def _ec_residuals(Pl, Pr, phys):
    Ut, Ft = ec.pair_UF(Pl, Pr, G, phys)
    dV = ph.entropy_vars(Pr, G) - ph.entropy_vars(Pl, G)
    phl, psl, Phl = ph.potentials(Pl, G)
    phr, psr, Phr = ph.potentials(Pr, G)
    out = []
    r = np.sum(dV * Ut, axis=0) - (phr - phl)
    out.append(np.abs(r) / (np.sum(np.abs(dV * Ut), axis=0) + np.abs(phr - phl)))
    for j in range(3):
        rhs = (psr[j] - psl[j]) - 0.5 * (Pl[5 + j] + Pr[5 + j]) * (Phr - Phl)
        rj = np.sum(dV * Ft[j], axis=0) - rhs
        out.append(np.abs(rj) / (np.sum(np.abs(dV * Ft[j]), axis=0) + np.abs(rhs) + 1e-300))
    return out


@pytest.mark.parametrize("phys,dim", CASES)
def test_ec_condition_holds_to_roundoff(phys, dim):
    # [V].U~ = [phi] and [V].F~_j = [psi_j] - {B_j}[Phi] (conditions under eq. UFcircle)
    rng = np.random.default_rng(10 + phys + dim)
    Pl = rand_P(20000, rng, phys, dim)
    Pr = rand_P(20000, rng, phys, dim)
    for r in _ec_residuals(Pl, Pr, phys):
        assert np.max(r) < 1e-12


@pytest.mark.parametrize("phys,dim", CASES)
def test_ec_condition_small_jumps(phys, dim):
    # nearly equal states exercise the series branch of the logarithmic mean
    rng = np.random.default_rng(20 + phys + dim)
    Pl = rand_P(5000, rng, phys, dim)
    Pr = Pl * (1 + 1e-4 * rng.uniform(-1, 1, size=Pl.shape))
    Ut, Ft = ec.pair_UF(Pl, Pr, G, phys)
    dV = ph.entropy_vars(Pr, G) - ph.entropy_vars(Pl, G)
    phl, psl, Phl = ph.potentials(Pl, G)
    phr, psr, Phr = ph.potentials(Pr, G)
    r = np.sum(dV * Ut, axis=0) - (phr - phl)
    assert np.max(np.abs(r) / np.sum(np.abs(dV * Ut), axis=0)) < 1e-9


@pytest.mark.parametrize("phys,dim", CASES)
def test_pair_flux_consistent_and_symmetric(phys, dim):
    rng = np.random.default_rng(30 + phys + dim)
    Pl = rand_P(3000, rng, phys, dim)
    Pr = rand_P(3000, rng, phys, dim)
    Ut, Ft = ec.pair_UF(Pl, Pl, G, phys)
    U = ph.cons(Pl, G)
    np.testing.assert_allclose(Ut, U, rtol=1e-12, atol=1e-12 * np.max(np.abs(U)))
    for j in range(3):
        F = ph.flux(Pl, G, j)
        np.testing.assert_allclose(Ft[j], F, rtol=1e-12, atol=1e-12 * np.max(np.abs(F)))
    U1, F1 = ec.pair_UF(Pl, Pr, G, phys)
    U2, F2 = ec.pair_UF(Pr, Pl, G, phys)
    np.testing.assert_allclose(U1, U2, rtol=1e-13, atol=1e-14)
    for j in range(3):
        np.testing.assert_allclose(F1[j], F2[j], rtol=1e-13, atol=1e-14)


def test_rmhd_pair_reduces_to_rhd_pair_without_field():
    rng = np.random.default_rng(40)
    Pl = rand_P(3000, rng, ph.RHD, 3)
    Pr = rand_P(3000, rng, ph.RHD, 3)
    m = ec.pair_means(Pl, Pr, G)
    np.testing.assert_allclose(ec.Utilde_rmhd(m, G), ec.Utilde_rhd(m, G), rtol=1e-12, atol=1e-13)
    for j in range(3):
        np.testing.assert_allclose(ec.Ftilde_rmhd(m, G, j), ec.Ftilde_rhd(m, G, j), rtol=1e-12, atol=1e-13)


def test_curvilinear_pair_condition():
    # eq. ECConditionCurv with random metric vectors
    rng = np.random.default_rng(41)
    for phys, dim in CASES:
        Pl = rand_P(2000, rng, phys, dim)
        Pr = rand_P(2000, rng, phys, dim)
        al = rng.normal(size=(dim + 1, 2000))
        ar = rng.normal(size=(dim + 1, 2000))
        F = ec.curvilinear_pair(Pl, Pr, al, ar, G, phys, dim)
        dV = ph.entropy_vars(Pr, G) - ph.entropy_vars(Pl, G)
        phl, psl, Phl = ph.potentials(Pl, G)
        phr, psr, Phr = ph.potentials(Pr, G)
        rhs = 0.5 * (al[0] + ar[0]) * (phr - phl)
        for j in range(dim):
            aj = 0.5 * (al[1 + j] + ar[1 + j])
            rhs = rhs + aj * (psr[j] - psl[j]) - 0.5 * aj * (Pl[5 + j] + Pr[5 + j]) * (Phr - Phl)
        lhs = np.sum(dV * F, axis=0)
        assert np.max(np.abs(lhs - rhs) / (np.sum(np.abs(dV * F), axis=0) + np.abs(rhs))) < 1e-12
