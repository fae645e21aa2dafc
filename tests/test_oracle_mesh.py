"""Pins for the adaptive mesh redistribution (Section 5)."""
import itertools

import numpy as np
import pytest

from oracle import mesh as msh
from paper_2107_12027_amd import workloads as wl


def _brute_jacobi(grid, w, x):
    """Pure-Python loop version of one Jacobi sweep on a 2D grid (tiny inputs)."""
    ny, nx = grid.shape
    out = x.copy()

    def get(a, j, i, comp=None):
        sx = sy = 0.0
        if grid.bc[0] == 0:
            if i < 0:
                i += nx; sx = -grid.period[0]
            elif i >= nx:
                i -= nx; sx = grid.period[0]
        if grid.bc[1] == 0:
            if j < 0:
                j += ny; sy = -grid.period[1]
            elif j >= ny:
                j -= ny; sy = grid.period[1]
        v = a[j, i]
        if comp == 0:
            v += sx
        if comp == 1:
            v += sy
        return v

    for j in range(ny):
        for i in range(nx):
            free = [grid.bc[0] == 0 or 0 < i < nx - 1, grid.bc[1] == 0 or 0 < j < ny - 1]
            den = 0.0
            num = [0.0, 0.0]
            for k, (di, dj) in enumerate(((1, 0), (0, 1))):
                if not free[k]:
                    continue
                wp, wm = get(w, j + dj, i + di), get(w, j - dj, i - di)
                den += 2 * w[j, i] + wp + wm
                for c in range(2):
                    num[c] += (w[j, i] + wp) * get(x[c], j + dj, i + di, c) + (w[j, i] + wm) * get(x[c], j - dj, i - di, c)
            for c in range(2):
                if free[c] and den > 0:
                    out[c][j, i] = num[c] / den
    return out


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (0, 1, 0)])
def test_jacobi_sweep_matches_brute_force(bc):
    rng = np.random.default_rng(sum(bc))
    g = wl.make_grid(2, (7, 6, 1), bc)
    x = wl.perturbed_mesh(g, rng, amp=0.05)
    w = rng.uniform(1, 3, size=g.shape)
    np.testing.assert_allclose(msh.jacobi_sweep(g, w, x), _brute_jacobi(g, w, x), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("dim,bc", [(2, (0, 0, 0)), (2, (1, 1, 0)), (3, (1, 1, 1)), (3, (0, 1, 0))])
def test_uniform_monitor_fixes_uniform_mesh(dim, bc):
    g = wl.make_grid(dim, (6, 7, 5), bc)
    x = wl.uniform_mesh(g)
    w = np.full(g.shape, 2.5)
    np.testing.assert_allclose(msh.jacobi_sweep(g, w, x), x, atol=1e-15)


def test_lowpass_weights_and_constants():
    g = wl.make_grid(2, (7, 7, 1), (0, 0, 0))
    w = np.zeros(g.shape)
    w[3, 3] = 1.0
    out = msh.lowpass(g, w)
    want = np.zeros(g.shape)
    for dj, di in itertools.product((-1, 0, 1), repeat=2):
        want[3 + dj, 3 + di] = 0.5 ** (abs(dj) + abs(di) + 2)
    np.testing.assert_allclose(out, want, atol=1e-16)
    g3 = wl.make_grid(3, (5, 4, 6), (1, 0, 1))
    c = np.full(g3.shape, 1.7)
    np.testing.assert_allclose(msh.lowpass(g3, c), c, rtol=1e-15)


def test_monitor_forms_on_linear_sigma():
    g = wl.make_grid(2, (9, 8, 1), (1, 1, 0))
    x = wl.uniform_mesh(g)
    P = np.zeros((8,) + g.shape)
    P[0] = 1.0 + 0.5 * x[0] + 0.25 * x[1]
    mon = wl.Monitor(enabled=1, sigma=0, form=0, alpha=12.0)
    np.testing.assert_allclose(msh.monitor(g, mon, P), np.sqrt(13.0), rtol=1e-13)
    mon = wl.Monitor(enabled=1, sigma=0, form=1, alpha=10.0)
    np.testing.assert_allclose(msh.monitor(g, mon, P), np.sqrt(1 + 10 * (0.5 ** 2 + 0.25 ** 2)), rtol=1e-13)
    P[0] = 1.0
    mon = wl.Monitor(enabled=1, sigma=1, form=0, alpha=12.0)
    np.testing.assert_array_equal(msh.monitor(g, mon, P), 1.0)


def test_laplacian_xi_closed_forms():
    # a quadratic on a bounded grid: every three-point second difference (central
    # or one-sided) is exact, Lap_xi sigma = 2 a L_1^2 + 2 b L_2^2 (x = lo + L xi)
    g = wl.make_grid(2, (9, 7, 1), (1, 1, 0), lo=(0.3, -0.2, 0.0), length=(2.0, 1.5, 1.0))
    x = wl.uniform_mesh(g)
    s = 0.7 * x[0] ** 2 - 1.1 * x[1] ** 2 + 0.4 * x[0] * x[1] + x[0]
    np.testing.assert_allclose(msh.laplacian_xi(g, s), 2 * 0.7 * 4.0 - 2 * 1.1 * 2.25, rtol=1e-12)
    # a sinusoid on a periodic 3D grid: the central difference scales it by
    # (2 cos(2 pi k h) - 2) / h^2 per axis
    g = wl.make_grid(3, (8, 10, 12), (0, 0, 0))
    x = wl.uniform_mesh(g)
    s = np.sin(2 * np.pi * (x[0] + 2 * x[1] + 3 * x[2]))
    fac = sum((2 * np.cos(2 * np.pi * k / n) - 2) * n * n for k, n in ((1, 8), (2, 10), (3, 12)))
    np.testing.assert_allclose(msh.laplacian_xi(g, s), fac * s, rtol=1e-10, atol=1e-9)


def test_gradlap_monitor_matches_brute_force():
    # node-by-node loops with explicit index wrap / one-sided stencils on a tiny
    # mixed-boundary grid
    rng = np.random.default_rng(5)
    g = wl.make_grid(2, (7, 6, 1), (0, 1, 0))
    P = np.zeros((8,) + g.shape)
    P[0] = rng.uniform(0.5, 2.0, g.shape)
    mon = wl.Monitor(enabled=1, sigma=1, form=2, alpha=20.0, alpha2=10.0)
    sig = np.log(P[0])
    n0, n1 = g.n[0], g.n[1]
    h0, h1 = g.dxi[0], g.dxi[1]
    grad = np.zeros(g.shape)
    lap = np.zeros(g.shape)
    for j in range(n1):
        for i in range(n0):
            d0 = (sig[j, (i + 1) % n0] - sig[j, (i - 1) % n0]) / (2 * h0)
            l0 = (sig[j, (i + 1) % n0] - 2 * sig[j, i] + sig[j, (i - 1) % n0]) / h0 ** 2
            if j == 0:
                d1 = (sig[1, i] - sig[0, i]) / h1
                l1 = (sig[2, i] - 2 * sig[1, i] + sig[0, i]) / h1 ** 2
            elif j == n1 - 1:
                d1 = (sig[j, i] - sig[j - 1, i]) / h1
                l1 = (sig[j, i] - 2 * sig[j - 1, i] + sig[j - 2, i]) / h1 ** 2
            else:
                d1 = (sig[j + 1, i] - sig[j - 1, i]) / (2 * h1)
                l1 = (sig[j + 1, i] - 2 * sig[j, i] + sig[j - 1, i]) / h1 ** 2
            grad[j, i] = np.hypot(d0, d1)
            lap[j, i] = abs(l0 + l1)
    want = np.sqrt(1 + 20 * grad / grad.max() + 10 * lap / lap.max())
    np.testing.assert_allclose(msh.monitor(g, mon, P), want, rtol=1e-13)


def test_move_limiter_matches_brute_force_and_keeps_order():
    rng = np.random.default_rng(3)
    for bc in ((0, 0, 0), (1, 1, 0)):
        g = wl.make_grid(2, (8, 7, 1), bc)
        x = wl.perturbed_mesh(g, rng, amp=0.03)
        dx = rng.normal(size=x.shape) * 0.2
        if bc[0] == 1:
            dx[0][:, [0, -1]] = 0
            dx[1][[0, -1], :] = 0
        ny, nx = g.shape
        best = 1.0
        for j in range(ny):
            for i in range(nx):
                for k, (di, dj) in enumerate(((1, 0), (0, 1))):
                    d = dx[k][j, i]
                    if d == 0:
                        continue
                    jj, ii = (j + dj, i + di) if d > 0 else (j - dj, i - di)
                    sh = 0.0
                    if ii < 0 or ii >= nx:
                        sh = np.sign(ii) * g.period[0] if k == 0 else 0.0
                        ii %= nx
                    if jj < 0 or jj >= ny:
                        sh = np.sign(jj) * g.period[1] if k == 1 else 0.0
                        jj %= ny
                    nb = x[k][jj, ii] + sh
                    best = min(best, (nb - x[k][j, i]) / (2 * d))
        got = msh.move_limiter(g, x, dx)
        assert abs(got - best) < 1e-15 * max(1.0, best)
        xn = x + got * dx
        # no node overtakes its neighbour along its own index direction
        assert np.all(np.diff(xn[0], axis=1) > 0) and np.all(np.diff(xn[1], axis=0) > 0)
