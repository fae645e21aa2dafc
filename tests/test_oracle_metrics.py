"""Pins for the discrete metrics (Section 3.3, eq. SCLCoeff, eq. VCLCoeff, Appendix B)."""
import numpy as np
import pytest

from oracle import metrics as mt, residual as rs
from paper_2107_12027_amd import workloads as wl

GRIDS = [
    (2, (12, 10, 1), (0, 0, 0)),
    (2, (12, 10, 1), (1, 1, 0)),
    (2, (9, 11, 1), (0, 1, 0)),
    (3, (8, 9, 7), (0, 0, 0)),
    (3, (8, 7, 9), (1, 1, 1)),
]


def scl_residual(grid, met):
    """sum_k delta_k[J dxi_k/dx_j]/dxi_k on the interior, per j (eq. DiscSCL_O2p)."""
    d = grid.dim
    out = []
    for j in range(d):
        s = 0.0
        for k in range(d):
            a = rs._line_view(met[k * (d + 1) + 1 + j][None], grid, k, 1)[0]
            s = s + mt.delta(a, d - 1 - k, 3) / grid.dxi[k]
        out.append(s)
    return out


@pytest.mark.parametrize("dim,n,bc", GRIDS)
def test_discrete_scl_on_random_curvilinear_meshes(dim, n, bc):
    rng = np.random.default_rng(sum(n) + sum(bc))
    g = wl.make_grid(dim, n, bc)
    x = wl.perturbed_mesh(g, rng, amp=0.04)
    # non-smooth random jitter keeps periodicity / fixed boundary normals
    jit = rng.uniform(-0.1, 0.1, size=x.shape) * min(g.dxi[:dim])
    for k in range(dim):
        if bc[k] == 1:
            ax = dim - 1 - k
            sl = [slice(None)] * dim
            sl[ax] = 0
            jit[k][tuple(sl)] = 0
            sl[ax] = n[k] - 1
            jit[k][tuple(sl)] = 0
    met = mt.metrics(g, x + jit, None)
    scale = max(np.max(np.abs(met)) / min(g.dxi[:dim]), 1.0)
    for r in scl_residual(g, met):
        assert np.max(np.abs(r)) < 1e-13 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_mesh_gives_exact_cofactors(dim):
    rng = np.random.default_rng(3)
    n = (10, 9, 8)
    g = wl.make_grid(dim, n, (1, 1, 1))
    A = np.eye(dim) + 0.3 * rng.normal(size=(dim, dim))
    xi = wl.uniform_mesh(g)                        # = xi for bounded unit axes
    x = np.einsum("ab,b...->a...", A, xi) + 0.2
    met = mt.metrics(g, x, None)
    # J dxi_k/dx_j = cof(A)_{jk} = det(A) (A^{-1})_{kj}
    inv = np.linalg.inv(A) * np.linalg.det(A)
    for k in range(dim):
        for j in range(dim):
            np.testing.assert_allclose(met[k * (dim + 1) + 1 + j], inv[k, j], atol=1e-11)
    J = mt.jacobian(g, x)
    np.testing.assert_allclose(J, np.linalg.det(A), rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_metrics_converge_to_analytic_cofactors(dim):
    errs = []
    for N in (12, 24, 48) if dim == 2 else (10, 20):
        g = wl.make_grid(dim, (N, N, N), (0, 0, 0))
        xi = wl.uniform_mesh(g)
        x = xi.copy()
        x[0] = xi[0] + 0.05 * np.sin(2 * np.pi * xi[1]) * (np.cos(2 * np.pi * xi[2]) if dim == 3 else 1)
        x[1] = xi[1] + 0.05 * np.sin(2 * np.pi * xi[0])
        if dim == 3:
            x[2] = xi[2] + 0.05 * np.sin(2 * np.pi * xi[0]) * np.sin(2 * np.pi * xi[1])
        # analytic Jacobian matrix dx_a/dxi_b
        M = np.zeros((dim, dim) + g.shape)
        c = 0.05 * 2 * np.pi
        for a in range(dim):
            M[a, a] = 1.0
        if dim == 2:
            M[0, 1] = c * np.cos(2 * np.pi * xi[1])
            M[1, 0] = c * np.cos(2 * np.pi * xi[0])
        else:
            M[0, 1] = c * np.cos(2 * np.pi * xi[1]) * np.cos(2 * np.pi * xi[2])
            M[0, 2] = -c * np.sin(2 * np.pi * xi[1]) * np.sin(2 * np.pi * xi[2])
            M[1, 0] = c * np.cos(2 * np.pi * xi[0])
            M[2, 0] = c * np.cos(2 * np.pi * xi[0]) * np.sin(2 * np.pi * xi[1])
            M[2, 1] = c * np.sin(2 * np.pi * xi[0]) * np.cos(2 * np.pi * xi[1])
        Mt = np.moveaxis(M, (0, 1), (-2, -1))
        cof = np.moveaxis(np.linalg.inv(Mt) * np.linalg.det(Mt)[..., None, None], (-2, -1), (0, 1))
        met = mt.metrics(g, x, None)
        err = 0.0
        for k in range(dim):
            for j in range(dim):
                err = max(err, np.max(np.abs(rs.interior(met[k * (dim + 1) + 1 + j][None], g)[0] - cof[k, j])))
        errs.append(err)
        Jerr = np.max(np.abs(mt.jacobian(g, x) - np.linalg.det(Mt)))
        assert Jerr < 50 * err + 1e-12
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 5.5, (errs, rates)


def test_temporal_metrics_definition_and_ghost_velocity():
    rng = np.random.default_rng(5)
    g = wl.make_grid(2, (10, 12, 1), (1, 0, 0))
    x = wl.perturbed_mesh(g, rng, amp=0.03)
    xd = rng.normal(size=x.shape)
    met = mt.metrics(g, x, xd)
    met0 = mt.metrics(g, x, None)
    xde = [mt.extend(xd[c], g, 3, "velocity") for c in range(2)]
    for k in range(2):
        want = -(xde[0] * met0[3 * k + 1] + xde[1] * met0[3 * k + 2])
        np.testing.assert_allclose(met[3 * k], want, rtol=1e-14, atol=1e-14)
    # odd reflection of the velocity on the bounded axis: xdot_{-a} = 2 xdot_0 - xdot_a
    np.testing.assert_allclose(xde[0][:, 2], 2 * xde[0][:, 3] - xde[0][:, 4])
