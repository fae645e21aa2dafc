"""Pins for the high-order coefficients and the central difference operator
(Proposition 4.1, eq. HOCoeff; Section 3.3 delta_k)."""
import json
import os
from fractions import Fraction

import numpy as np

from oracle import metrics as mt

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hocoeff.json")


def test_alpha_matches_golden_rationals():
    gold = json.load(open(GOLD))["alpha"]
    for p, vals in gold.items():
        a = mt.alpha(int(p))
        want = [float(Fraction(n, d)) for n, d in vals]
        np.testing.assert_allclose(a, want, rtol=1e-14, atol=1e-15)


def test_alpha_p3_is_textbook_sixth_order_stencil():
    # delta[a]_0 = 3/4 (a1 - a-1) - 3/20 (a2 - a-2) + 1/60 (a3 - a-3)
    a = mt.alpha(3)
    np.testing.assert_allclose(0.5 * a, [45 / 60, -9 / 60, 1 / 60], rtol=1e-14)


def test_delta_exact_on_polynomials_up_to_degree_2p():
    h = 0.1
    x = np.arange(-6, 7) * h + 0.37
    for p in (1, 2, 3, 4):
        for q in range(0, 2 * p + 2):
            f = x ** q
            d = mt.delta(f, 0, p)[len(x) // 2 - p] / h      # node at index 6
            exact = q * 0.37 ** (q - 1) if q > 0 else 0.0
            if q <= 2 * p:
                assert abs(d - exact) < 1e-10 * max(1.0, abs(exact)), (p, q, d, exact)
            else:
                assert abs(d - exact) > 1e-8, (p, q)
