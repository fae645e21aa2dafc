"""Oracle discrete metrics (test infrastructure only).

Section 3.3 (Discrete GCLs): spatial metrics by the conservative metric method
(eq. CMM_SCL, eq. SCLCoeff) with the 2p-th order central difference
    delta_k[a]_i = 1/2 sum_{n=1}^{p} alpha_{p,n} (a_{i,k,+n} - a_{i,k,-n}),
temporal metrics J d(xi_k)/dt = -sum_j xdot_j (J d(xi_k)/dx_j) (eq. VCLCoeff);
the 2D explicit form of Appendix B with the 1/Delta xi factors of eq. SCLCoeff.

Ghost handling (a reading; the paper does not fix it): the mesh is extended beyond the index
box by a periodic copy plus the period shift, or by odd reflection
x_{-a} = 2 x_0 - x_a on bounded axes; the metrics on the ghost strips (ghost(p)
wide) are evaluated from that extended mesh with the same formula as inside.

Array layout: node fields are C-ordered [z][y][x]; index axis k (xi_{k+1}) is
array axis ndim-1-k.  ``met`` has d(d+1) components on the ghost-padded box
(each axis grown by ghost(p) on both sides): met[k(d+1)] = J dxi_k/dt and
met[k(d+1)+1+j] = J dxi_k/dx_j.
"""
from __future__ import annotations

import numpy as np

NG = 3      # ghost layers of the padded box for p <= 3


def ghost(p: int) -> int:
    """Ghost layers of the padded box for the 2p-th order scheme: its stencils reach
    p nodes past an edge (the EC pairs (i, i+n), n <= p, the metrics' delta_k and,
    for the dissipation, WENO-(2p-1) on nodes i-p+1..i+p); p = 2 keeps the layout
    of p = 3."""
    return max(NG, p)


def alpha(p: int):
    """alpha_{p,n}, n = 1..p: the solution of eq. HOCoeff
    sum_n n alpha_n = 1, sum_n n^(2s-1) alpha_n = 0 (s = 2..p)."""
    A = np.array([[float(n) ** (2 * s - 1) for n in range(1, p + 1)] for s in range(1, p + 1)])
    rhs = np.zeros(p)
    rhs[0] = 1.0
    return np.linalg.solve(A, rhs)


def _ax(arr_ndim, k):
    return arr_ndim - 1 - k


def extend(f, grid, width, kind, comp=None):
    """Pad a node field (shape grid.shape) by ``width`` on every active axis.
    kind: 'mesh' (coordinate ``comp``; periodic wrap + shift / odd reflection),
          'velocity' (periodic wrap / odd reflection),
          'solution' (periodic wrap / zero-gradient copy)."""
    out = np.asarray(f)
    for k in range(grid.dim):
        ax = _ax(out.ndim, k)
        pw = [(0, 0)] * out.ndim
        pw[ax] = (width, width)
        if grid.bc[k] == 0:
            out = np.pad(out, pw, mode="wrap")
            if kind == "mesh" and comp == k:
                L = grid.period[k]
                idx = np.arange(out.shape[ax])
                shift = np.where(idx < width, -L, np.where(idx >= out.shape[ax] - width, L, 0.0))
                sh = [1] * out.ndim
                sh[ax] = -1
                out = out + shift.reshape(sh)
        else:
            if kind == "solution":
                out = np.pad(out, pw, mode="edge")
            else:
                out = np.pad(out, pw, mode="reflect", reflect_type="odd")
    return out


def delta(a, ax, p):
    """2p-th order central difference along array axis ``ax``; the result covers
    the input range shrunk by p on both sides of that axis."""
    al = alpha(p)
    n = a.shape[ax]
    out = 0.0
    for m in range(1, p + 1):
        plus = np.take(a, np.arange(p + m, n - p + m), axis=ax)
        minus = np.take(a, np.arange(p - m, n - p - m), axis=ax)
        out = out + 0.5 * al[m - 1] * (plus - minus)
    return out


def crop(a, ax, c):
    if c == 0:
        return a
    return np.take(a, np.arange(c, a.shape[ax] - c), axis=ax)


def spatial_metrics(grid, x, p=3):
    """J dxi_k/dx_j on the ghost-padded box: list [k][j]."""
    d = grid.dim
    ng = ghost(p)
    xe = [extend(x[c], grid, 2 * ng, "mesh", comp=c) for c in range(d)]
    nd = xe[0].ndim
    dxi = grid.dxi
    if d == 2:
        ax0, ax1 = _ax(nd, 0), _ax(nd, 1)
        # Appendix B: J xi_x = delta_eta[y]/deta, J xi_y = -delta_eta[x]/deta,
        #             J eta_x = -delta_xi[y]/dxi, J eta_y = delta_xi[x]/dxi
        def d_eta(f):
            return crop(crop(delta(f, ax1, p), ax1, ng - p), ax0, ng)

        def d_xi(f):
            return crop(crop(delta(f, ax0, p), ax0, ng - p), ax1, ng)
        return [[d_eta(xe[1]) / dxi[1], -d_eta(xe[0]) / dxi[1]],
                [-d_xi(xe[1]) / dxi[0], d_xi(xe[0]) / dxi[0]]]
    # 3D: eq. SCLCoeff, J dxi_k/dx_j = (d_k2[d_k1[x_j1] x_j2] - d_k1[d_k2[x_j1] x_j2]) / (dxi_k1 dxi_k2)
    out = [[None] * 3 for _ in range(3)]
    for k in range(3):
        k1, k2 = (k + 1) % 3, (k + 2) % 3
        a_k, a1, a2 = _ax(nd, k), _ax(nd, k1), _ax(nd, k2)
        for j in range(3):
            j1, j2 = (j + 1) % 3, (j + 2) % 3
            # term A = delta_k2[ delta_k1[x_j1] * x_j2 ]
            t = delta(xe[j1], a1, p) * crop(xe[j2], a1, p)
            tA = delta(t, a2, p)              # axes k1, k2 shrunk by p
            t = delta(xe[j1], a2, p) * crop(xe[j2], a2, p)
            tB = delta(t, a1, p)
            val = (tA - tB) / (dxi[k1] * dxi[k2])
            # shrink axis k by 2 ng - ng and axes k1, k2 by (2 ng - p) - ng
            val = crop(val, a_k, ng)
            val = crop(val, a1, ng - p)
            val = crop(val, a2, ng - p)
            out[k][j] = val
    return out


def metrics(grid, x, xdot=None, p=3):
    """Full metric array (d(d+1), *padded shape): temporal metric of eq. VCLCoeff
    from the extended mesh velocity, then the spatial metrics."""
    d = grid.dim
    S = spatial_metrics(grid, x, p)
    pshape = S[0][0].shape
    met = np.zeros((d * (d + 1),) + pshape)
    if xdot is not None:
        xde = [extend(xdot[c], grid, ghost(p), "velocity") for c in range(d)]
    for k in range(d):
        at = np.zeros(pshape)
        for j in range(d):
            met[k * (d + 1) + 1 + j] = S[k][j]
            if xdot is not None:
                at = at - xde[j] * S[k][j]
        met[k * (d + 1)] = at
    return met


def jacobian(grid, x, p=3):
    """Initial J on the interior nodes: 2D J = (delta_xi[x] delta_eta[y] -
    delta_eta[x] delta_xi[y]) / (dxi deta); 3D J = sum_k (J dxi_k/dx_1) delta_k[x_1]/dxi_k
    (cofactor expansion with the CMM metrics).  Any 2p-th order J^0 keeps the
    free-stream and EC properties; this one is exact for affine meshes."""
    d = grid.dim
    xe = [extend(x[c], grid, p, "mesh", comp=c) for c in range(d)]
    nd = xe[0].ndim
    if d == 2:
        ax0, ax1 = _ax(nd, 0), _ax(nd, 1)
        dx_xi = crop(delta(xe[0], ax0, p), ax1, p)
        dy_xi = crop(delta(xe[1], ax0, p), ax1, p)
        dx_eta = crop(delta(xe[0], ax1, p), ax0, p)
        dy_eta = crop(delta(xe[1], ax1, p), ax0, p)
        return (dx_xi * dy_eta - dx_eta * dy_xi) / (grid.dxi[0] * grid.dxi[1])
    S = spatial_metrics(grid, x, p)
    J = 0.0
    for k in range(3):
        dk = delta(xe[0], _ax(nd, k), p)
        for kk in range(3):
            if kk != k:
                dk = crop(dk, _ax(nd, kk), p)
        Sk = S[k][0]
        for kk in range(3):
            Sk = crop(Sk, _ax(nd, kk), ghost(p))
        J = J + Sk * dk / grid.dxi[k]
    return J
