"""Mutation checks of the oracle pins (CPU only).

Each test plants one plausible mistake in the oracle's own source text (a
dropped term, a wrong factor, a wrong line of an inverse), runs the pinned
comparison of tests/test_oracle_pins.py on the mutated oracle, and asserts that
the comparison now fails.  The mutants live only inside the test (the oracle
module's function is swapped by monkeypatch and restored afterwards).

* lambda^ of eq. ESFlux_HO without the temporal metric J dxi_k/dt;
* the factor 1/2 of eq. ESFlux_HO replaced by 1;
* the b^0 line of the explicit entropy-variable inverse (b^0 = u.b/W) with W
  in place of 1/W.
"""
import inspect
import textwrap

import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import dissipation as ds
from oracle import metrics as mt
from oracle import physics as ph
from oracle import residual as rs
from oracle import stepper as st
from oracle_util import rand_P
from paper_2107_12027_amd import workloads as wl

G = pins.G


def _mutant(module, name, old, new):
    """The function module.name recompiled from its source with `old` replaced by
    `new` (exactly one occurrence), in the module's namespace."""
    src = textwrap.dedent(inspect.getsource(getattr(module, name)))
    assert src.count(old) == 1, (name, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), "<mutant %s.%s>" % (module.__name__, name), "exec"), ns)
    return ns[name]


def _lambda_hat_error(phys, dim):
    """max relative difference between the oracle's lambda^ and the textbook value
    (the comparison of test_lambda_hat_against_textbook_speeds)."""
    rng = np.random.default_rng(5 + 7 * phys + dim)
    N = 60
    Pst, ast = pins._face_case(rng, phys, dim, N)
    _, info = ds.face_dissipation(Pst, ast, G, phys, dim, 1e-6, details=True)
    abar = 0.5 * (ast[0] + ast[1])
    ax = np.zeros((3, N))
    ax[:dim] = abar[1:]
    L = np.linalg.norm(ax, axis=0)
    n = ax / L
    Pf = ph.prim_from_entropy_vars(0.5 * (ph.entropy_vars(Pst[2], G) + ph.entropy_vars(Pst[3], G)), G)
    Pf[5:8] = 0.0
    lam = pins._rhd_speeds(Pf, n)
    want = np.maximum(np.abs(abar[0] + L * lam[0]), np.abs(abar[0] + L * lam[2]))
    return float(np.max(np.abs(info["lhat"] - want) / want))


def test_lambda_hat_pin_catches_a_dropped_temporal_metric(monkeypatch):
    assert _lambda_hat_error(ph.RHD, 2) < 1e-9
    bad = _mutant(ds, "face_dissipation", "np.abs(abar[0][:, None] + L[:, None] * lam)",
                  "np.abs(L[:, None] * lam)")
    monkeypatch.setattr(ds, "face_dissipation", bad)
    assert _lambda_hat_error(ph.RHD, 2) > 1e-2


def _first_order_limit_error(phys, delta=4e-3):
    """relative error of the ES - EC flux difference at a single jump against
    lambda^ [U] / (2 dxi) (the comparison of test_dissipation_scale_first_order_limit)."""
    g, x, xdot, P, Pa, Pb = pins._jump_case(phys, delta)
    base = wl.Scheme(phys=phys, order_p=3, weno_eps=1e-40)
    met = mt.metrics(g, x, xdot, 3)
    Ppad = st.pad_solution(g, P)
    dU_ec, _ = rs.residual(g, wl.Scheme(phys=phys, order_p=3, dissipation=0), Ppad, met)
    _, _, info = rs.residual(g, base, Ppad, met, details=True)
    ones = {k: np.ones_like(info[k]["Y"]) for k in info}
    dU_es, _ = rs.residual(g, base, Ppad, met, Y_fixed=ones)
    diff = dU_es - dU_ec
    i = g.n[0] // 2 - 1
    a = mt.metrics(g, x, xdot, 3)[:, 3, 3 + i]
    at, ax = a[0], np.array([a[1], a[2], 0.0])
    L = np.linalg.norm(ax)
    n = ax / L
    Pf = ph.prim_from_entropy_vars(0.5 * (ph.entropy_vars(Pa, G) + ph.entropy_vars(Pb, G)), G)
    lo, _, hi = ph.eigen_speeds_rhd(Pf[:, None], G, n[:, None])
    lhat = max(abs(at + L * float(lo[0])), abs(at + L * float(hi[0])))
    sel = ph.comps(phys, 2)
    jumpU = (ph.cons(Pb[:, None], G) - ph.cons(Pa[:, None], G))[sel, 0]
    want = lhat * jumpU / (2.0 * g.dxi[0])
    return float(np.max(np.abs(diff[:, 0, i] - want)) / np.max(np.abs(want)))


def test_dissipation_scale_pin_catches_a_doubled_term(monkeypatch):
    assert _first_order_limit_error(ph.RHD) < 5e-5
    bad = _mutant(rs, "residual", "Ff = Ff - 0.5 * dd.reshape", "Ff = Ff - 1.0 * dd.reshape")
    monkeypatch.setattr(rs, "residual", bad)
    assert _first_order_limit_error(ph.RHD) > 0.5


def _round_trip_error(rng):
    P = rand_P(500, rng, ph.RMHD, 2, vmax=0.99, lo=0.01)
    Q = ph.prim_from_entropy_vars(ph.entropy_vars(P, G), G)
    return float(np.max(np.abs(Q - P) / np.maximum(np.abs(P), 1.0)))


def test_entropy_inverse_pin_catches_a_wrong_b0_line(monkeypatch):
    assert _round_trip_error(np.random.default_rng(2)) < 1e-12
    bad = _mutant(ph, "prim_from_entropy_vars", "b0 = _dot(u, b) / W", "b0 = _dot(u, b) * W")
    monkeypatch.setattr(ph, "prim_from_entropy_vars", bad)
    assert _round_trip_error(np.random.default_rng(2)) > 1e-3


@pytest.mark.parametrize("mutation", [("np.abs(abar[0][:, None] + L[:, None] * lam)", "np.abs(L[:, None] * lam)")])
def test_rmhd_lambda_hat_pin_catches_a_dropped_temporal_metric(monkeypatch, mutation):
    # the RMHD branch: lambda^ against the fast roots of the characteristic quartic
    rng = np.random.default_rng(5 + 7 * ph.RMHD + 2)
    N = 12
    Pst, ast = pins._face_case(rng, ph.RMHD, 2, N)
    bad = _mutant(ds, "face_dissipation", *mutation)
    errs = []
    for fn in (ds.face_dissipation, bad):
        _, info = fn(Pst, ast, G, ph.RMHD, 2, 1e-6, details=True)
        abar = 0.5 * (ast[0] + ast[1])
        ax = np.zeros((3, N))
        ax[:2] = abar[1:]
        L = np.linalg.norm(ax, axis=0)
        n = ax / L
        Pf = ph.prim_from_entropy_vars(0.5 * (ph.entropy_vars(Pst[2], G) + ph.entropy_vars(Pst[3], G)), G)
        want = np.zeros(N)
        for f in range(N):
            lo, hi = pins._outer_roots(pins._fast_quartic(Pf[:, f], n[:, f]))
            want[f] = max(abs(abar[0, f] + L[f] * lo), abs(abar[0, f] + L[f] * hi))
        errs.append(float(np.max(np.abs(info["lhat"] - want) / want)))
    assert errs[0] < 1e-9 and errs[1] > 1e-2, errs
