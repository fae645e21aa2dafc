"""Oracle adaptive mesh redistribution (test infrastructure only).

Section 5 of the paper: Winslow's choice G_k = omega I in the mesh functional
(eq. mesh_func, eq. mesh_EL), the monitor (eq. monitor), the 3^d-point low-pass
filter, the Jacobi iteration of the central-difference mesh equations, the move
limiter Delta_tau and the mesh velocity xdot = Delta_tau delta_tau x / Delta t.
Boundary treatment, the gradient discretisation, the squared-gradient monitor
form and the limiter typo are readings of the paper, not its printed text.
"""
from __future__ import annotations

import numpy as np

from .metrics import extend, crop

SIGMA_RHO, SIGMA_LNRHO = 0, 1
MON_PAPER, MON_SQGRAD, MON_GRADLAP = 0, 1, 2


def _shift(a, grid, k, s, ax):
    """Neighbour value along index axis k with offset s (+1/-1) from an array
    extended by one layer on every active axis; cropped back to the interior."""
    n = a.shape[ax]
    idx = np.arange(1 + s, n - 1 + s)
    out = np.take(a, idx, axis=ax)
    for kk in range(grid.dim):
        if kk != k:
            axk = out.ndim - 1 - kk
            out = crop(out, axk, 1)
    return out


def _free_mask(grid, k):
    """True where node is free along index axis k (periodic, or not on a bounded edge)."""
    m = np.ones(grid.shape, dtype=bool)
    if grid.bc[k] != 0:
        ax = grid.dim - 1 - k
        idx = [slice(None)] * grid.dim
        idx[ax] = 0
        m[tuple(idx)] = False
        idx[ax] = grid.n[k] - 1
        m[tuple(idx)] = False
    return m


def laplacian_xi(grid, sigma):
    """sum_k d^2 sigma / d xi_k^2 by the three-point second difference: central in
    the interior and on periodic axes, one-sided (the three nearest nodes on the
    axis) on bounded edges."""
    lap = np.zeros(grid.shape)
    for k in range(grid.dim):
        ax = grid.dim - 1 - k
        n = grid.n[k]
        h2 = grid.dxi[k] ** 2
        if grid.bc[k] == 0:
            lap = lap + (np.roll(sigma, -1, axis=ax) - 2 * sigma + np.roll(sigma, 1, axis=ax)) / h2
            continue
        d = np.zeros(grid.shape)
        for i in range(n):
            j = min(max(i, 1), n - 2)          # centre of the three-point stencil
            idx = [slice(None)] * grid.dim
            idx[ax] = i
            d[tuple(idx)] = (np.take(sigma, j + 1, axis=ax) - 2 * np.take(sigma, j, axis=ax)
                             + np.take(sigma, j - 1, axis=ax)) / h2
        lap = lap + d
    return lap


def monitor(grid, mon, Pin):
    """omega = sqrt(1 + alpha |grad_xi sigma| / max |grad_xi sigma|) (eq. monitor), or
    omega = sqrt(1 + alpha |grad_xi sigma|^2), or (eq. RMHD_2DVortex_Monitor)
    omega = sqrt(1 + alpha |grad_xi sigma| / max |grad_xi sigma|
                   + alpha2 |Lap_xi sigma| / max |Lap_xi sigma|);
    second-order central differences in xi, one-sided on bounded edges; a
    normalised term whose maximum is zero is left out (omega = 1 for a constant
    sigma)."""
    sigma = Pin[0] if mon.sigma == SIGMA_RHO else np.log(Pin[0])
    g2 = np.zeros(grid.shape)
    for k in range(grid.dim):
        ax = grid.dim - 1 - k
        n = grid.n[k]
        if grid.bc[k] == 0:
            d = (np.roll(sigma, -1, axis=ax) - np.roll(sigma, 1, axis=ax)) / (2 * grid.dxi[k])
        else:
            d = np.zeros(grid.shape)
            inner = [slice(None)] * grid.dim
            inner[ax] = slice(1, n - 1)
            d[tuple(inner)] = (np.take(sigma, np.arange(2, n), axis=ax)
                               - np.take(sigma, np.arange(0, n - 2), axis=ax)) / (2 * grid.dxi[k])
            e0 = [slice(None)] * grid.dim
            e0[ax] = 0
            d[tuple(e0)] = (np.take(sigma, 1, axis=ax) - np.take(sigma, 0, axis=ax)) / grid.dxi[k]
            e1 = [slice(None)] * grid.dim
            e1[ax] = n - 1
            d[tuple(e1)] = (np.take(sigma, n - 1, axis=ax) - np.take(sigma, n - 2, axis=ax)) / grid.dxi[k]
        g2 = g2 + d * d
    if mon.form == MON_SQGRAD:
        return np.sqrt(1.0 + mon.alpha * g2)
    g = np.sqrt(g2)
    mx = float(np.max(g))
    w2 = np.ones(grid.shape)
    if mx > 0.0:
        w2 = w2 + mon.alpha * g / mx
    if mon.form == MON_GRADLAP:
        lap = np.abs(laplacian_xi(grid, sigma))
        ml = float(np.max(lap))
        if ml > 0.0:
            w2 = w2 + mon.alpha2 * lap / ml
    return np.sqrt(w2)


def lowpass(grid, w):
    """One pass of w_i <- sum_{j in {-1,0,1}^d} 2^{-(|j|_1 + d)} w_{i+j} (Remark in Section 5);
    ghost values by periodic wrap or zero-gradient copy."""
    we = extend(w, grid, 1, "solution")
    out = np.zeros(grid.shape)
    d = grid.dim
    offs = np.array(np.meshgrid(*([[-1, 0, 1]] * d), indexing="ij")).reshape(d, -1).T
    for o in offs:
        # o[k] is the offset along index axis k
        sl = []
        for ax in range(d):
            k = d - 1 - ax
            sl.append(slice(1 + o[k], 1 + o[k] + grid.n[k]))
        out = out + 0.5 ** (np.sum(np.abs(o)) + d) * we[tuple(sl)]
    return out


def jacobi_sweep(grid, w, x):
    """One Jacobi sweep of sum_k [(w_i + w_{i+e_k})(x_{i+e_k} - x_i) - (w_i + w_{i-e_k})(x_i - x_{i-e_k})] = 0
    (Section 5), over the index axes along which a node is free; on bounded edges the
    normal coordinate stays fixed and the tangential ones follow the lower-dimensional
    rule along the edge; corners stay fixed."""
    d = grid.dim
    we = extend(w, grid, 1, "solution")
    xe = [extend(x[c], grid, 1, "mesh", comp=c) for c in range(d)]
    num = [np.zeros(grid.shape) for _ in range(d)]
    den = np.zeros(grid.shape)
    free = [_free_mask(grid, k) for k in range(d)]
    wc = w
    for k in range(d):
        ax = d - 1 - k
        wp = _shift(we, grid, k, +1, ax)
        wm = _shift(we, grid, k, -1, ax)
        f = free[k]
        den = den + np.where(f, 2 * wc + wp + wm, 0.0)
        for c in range(d):
            xp = _shift(xe[c], grid, k, +1, ax)
            xm = _shift(xe[c], grid, k, -1, ax)
            num[c] = num[c] + np.where(f, (wc + wp) * xp + (wc + wm) * xm, 0.0)
    out = x.copy()
    for c in range(d):
        upd = free[c] & (den > 0)
        out[c] = np.where(upd, num[c] / np.where(den > 0, den, 1.0), x[c])
    return out


def move_limiter(grid, x, dx):
    """Delta_tau = min(1, min over nodes and axes k of the bound
    -(x_k,i - x_k,i-e_k)/(2 dx_k) if dx_k < 0, (x_k,i+e_k - x_k,i)/(2 dx_k) if dx_k > 0)
    (Section 5, with the (x_1) -> (x_k) typo corrected)."""
    d = grid.dim
    best = 1.0
    for k in range(d):
        ax = d - 1 - k
        xe = extend(x[k], grid, 1, "mesh", comp=k)
        xp = _shift(xe, grid, k, +1, ax)
        xm = _shift(xe, grid, k, -1, ax)
        dk = dx[k]
        neg = dk < 0
        pos = dk > 0
        if np.any(neg):
            best = min(best, float(np.min(-(x[k][neg] - xm[neg]) / (2 * dk[neg]))))
        if np.any(pos):
            best = min(best, float(np.min((xp[pos] - x[k][pos]) / (2 * dk[pos]))))
    return best


def redistribute(grid, mon, Pin, x, dt):
    """Monitor, filter, mu Jacobi sweeps, limiter: returns (x^{n+1}, xdot, omega, dtau)."""
    w = monitor(grid, mon, Pin)
    for _ in range(mon.filter_passes):
        w = lowpass(grid, w)
    xi = x.copy()
    for _ in range(mon.sweeps):
        xi = jacobi_sweep(grid, w, xi)
    dx = xi - x
    dtau = move_limiter(grid, x, dx)
    xnew = x + dtau * dx
    xdot = dtau * dx / dt
    return xnew, xdot, w, dtau
