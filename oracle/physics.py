"""Oracle physics: ideal-gas RMHD/RHD in the lab frame (test infrastructure only).

Internally every state is the full 8-slot primitive vector
    P = (rho, u_1, u_2, u_3, p, B_1, B_2, B_3),   u = W v,
and the full 8-slot conservative vector U = (D, m_1, m_2, m_3, E, B_1, B_2, B_3).
``comps(phys, dim)`` selects the slots a system evolves: 2D RHD keeps
(D, m_1, m_2, E) (v_3 = 0, B = 0), 3D RHD keeps the first five, RMHD keeps all
eight (all three components of v and B are kept in 2D).

Sources (Section 1, Section 2 of the paper):
  * EOS p = (Gamma-1) rho e, h = 1 + e + p/rho                     (eq. EOS)
  * U, F_k, D = rho W, m, E, p_tot = p + |b|^2/2                   (eq. RMHDdiv2)
  * b^alpha = W (v.B, B/W^2 + v (v.B)), |b|^2 = |B|^2/W^2 + (v.B)^2 (Section 1)
  * entropy pair eta = -rho W s/(Gamma-1), q_k = eta v_k          (eq. EntropyPair)
  * entropy variables V                                           (Section 2, after eq. Phi)
  * Phi = rho W (v.B)/p and Phi'(V)                               (eq. Phi)
  * potentials phi = V.U - eta, psi_k = V.F_k + Phi B_k - q_k      (eq. EntropyPotential)
Every function accepts real or complex arrays (complex inputs are used for
complex-step derivatives in ``dissipation``).
"""
from __future__ import annotations

import numpy as np

RHD = 0
RMHD = 1


def comps(phys: int, dim: int):
    """Slots of the 8-vector that the (phys, dim) system evolves."""
    if phys == RMHD:
        return [0, 1, 2, 3, 4, 5, 6, 7]
    return [0, 1, 2, 4] if dim == 2 else [0, 1, 2, 3, 4]


def nvars(phys: int, dim: int) -> int:
    return len(comps(phys, dim))


def full_prim(rho, u, p, B):
    """Stack the 8-slot primitive vector from the workload fields."""
    return np.concatenate([np.asarray(rho)[None], np.asarray(u), np.asarray(p)[None],
                           np.asarray(B)], axis=0).astype(np.result_type(rho, u, p, B, np.float64))


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def state(P, G):
    """Derived per-node quantities from the full primitive vector."""
    rho, u, p, B = P[0], P[1:4], P[4], P[5:8]
    W = np.sqrt(1.0 + _dot(u, u))
    v = u / W
    beta = rho / p
    h = 1.0 + G / (G - 1.0) * p / rho
    vB = _dot(v, B)
    b0 = W * vB                      # b^0 = W v.B = u.B
    b = B / W + W * vB * v           # spatial b = B/W^2 * W + W v (v.B)
    bsq = _dot(B, B) / (W * W) + vB * vB
    return dict(rho=rho, u=u, p=p, B=B, W=W, v=v, beta=beta, h=h, vB=vB, b0=b0, b=b,
                bsq=bsq, BB=_dot(B, B))


def cons(P, G):
    """Conservative 8-vector U(P) (eq. RMHDdiv2)."""
    s = state(P, G)
    rho, W, v, B, p, h, vB, bsq = s["rho"], s["W"], s["v"], s["B"], s["p"], s["h"], s["vB"], s["bsq"]
    Z = rho * h * W * W
    D = rho * W
    m = (Z + s["BB"]) * v - vB * B
    E = Z - p - 0.5 * bsq + s["BB"]
    return np.concatenate([D[None], m, E[None], B], axis=0)


def flux(P, G, j):
    """Physical flux F_j(P) in direction x_j (eq. RMHDdiv2), full 8-vector."""
    s = state(P, G)
    rho, W, v, B, p, vB, bsq = s["rho"], s["W"], s["v"], s["B"], s["p"], s["vB"], s["bsq"]
    U = cons(P, G)
    ptot = p + 0.5 * bsq
    out = []
    out.append(U[0] * v[j])
    for c in range(3):
        val = U[1 + c] * v[j] - B[j] * (B[c] / (W * W) + vB * v[c])
        if c == j:
            val = val + ptot
        out.append(val)
    out.append(U[1 + j])
    for c in range(3):
        out.append(v[j] * B[c] - B[j] * v[c])
    return np.stack(out)


def entropy_vars(P, G):
    """Entropy variables V = eta'(U)^T (Section 2): with beta = rho/p,
    V = (Gamma/(Gamma-1) + ln rho + ln beta/(Gamma-1) + beta, beta u, -beta W, beta b)."""
    s = state(P, G)
    beta = s["beta"]
    V1 = G / (G - 1.0) + np.log(s["rho"]) + np.log(beta) / (G - 1.0) + beta
    return np.concatenate([V1[None], beta * s["u"], (-beta * s["W"])[None], beta * s["b"]], axis=0)


def prim_from_entropy_vars(V, G):
    """Explicit inverse of the entropy-variable map: with beta^2 = V_5^2 - |V_2..4|^2
    (since W^2 - |u|^2 = 1), u = V_2..4/beta, W = -V_5/beta,
    ln rho = V_1 - Gamma/(Gamma-1) - ln(beta)/(Gamma-1) - beta, p = rho/beta, b = V_6..8/beta,
    b^0 = u.b/W (from b = (B + b^0 u)/W and b^0 = u.B) and B = W b - b^0 u."""
    beta = np.sqrt(V[4] ** 2 - _dot(V[1:4], V[1:4]))
    u = V[1:4] / beta
    W = -V[4] / beta
    rho = np.exp(V[0] - G / (G - 1.0) - np.log(beta) / (G - 1.0) - beta)
    p = rho / beta
    b = V[5:8] / beta
    b0 = _dot(u, b) / W
    B = W * b - b0 * u
    return np.concatenate([rho[None], u, p[None], B], axis=0)


def entropy(P, G):
    """eta = -rho W s/(Gamma-1), s = ln(p/rho^Gamma) (eq. EntropyPair)."""
    s = state(P, G)
    sth = np.log(s["p"]) - G * np.log(s["rho"])
    return -s["rho"] * s["W"] * sth / (G - 1.0)


def potentials(P, G):
    """phi, psi_k (eq. EntropyPotential) and Phi (eq. Phi)."""
    s = state(P, G)
    half = 0.5 * s["beta"] * s["bsq"]
    phi = s["rho"] * s["W"] + half * s["W"]
    psi = s["rho"] * s["u"] + half * s["u"]
    Phi = s["beta"] * s["b0"]
    return phi, psi, Phi


def phi_prime(P, G):
    """Phi'(V) = (0, B/W^2 + v (v.B), v.B, v) in the U slots (eq. Phi)."""
    s = state(P, G)
    W, v, B, vB = s["W"], s["v"], s["B"], s["vB"]
    z = np.zeros_like(W)
    return np.concatenate([z[None], B / (W * W) + vB * v, vB[None], v], axis=0)


def eigen_speeds_rhd(P, G, n):
    """Closed-form RHD characteristic speeds along unit normal n (textbook):
    lambda_0 = v_n and lambda_+- = [v_n (1 - c^2) +- c sqrt((1-v^2)(1 - v^2 c^2 - v_n^2 (1 - c^2)))]
    / (1 - v^2 c^2), with c^2 = Gamma p/(rho h).  Used only as a pin for the numeric
    eigen-structure in ``dissipation``."""
    s = state(P, G)
    v = s["v"]
    vn = _dot(v, n)
    v2 = _dot(v, v)
    cs2 = G * s["p"] / (s["rho"] * s["h"])
    disc = np.sqrt((1 - v2) * (1 - v2 * cs2 - vn * vn * (1 - cs2)))
    lp = (vn * (1 - cs2) + np.sqrt(cs2) * disc) / (1 - v2 * cs2)
    lm = (vn * (1 - cs2) - np.sqrt(cs2) * disc) / (1 - v2 * cs2)
    return lm, vn, lp


# ---------------------------------------------------------------------------
# Conservative -> primitive recovery (the paper only states that a nonlinear
# algebraic equation must be solved, Section 1).  The reading used here: a
# bracketed bisection to full precision on the scalar equation for p (RHD) or
# for Z = rho h W^2 (RMHD); the root is unique, so any converged solver agrees.
# ---------------------------------------------------------------------------

def con2prim_rhd(U, G, dim, maxit=400):
    """U = (D, m_1..m_d, E) -> full 8-slot P.  Solves
    g(p) = (Gamma-1)[(E+p)(1-v^2) - p - D sqrt(1-v^2)] - p = 0,  v = |m|/(E+p),
    which follows from E + p = rho h W^2, D = rho W.  g is strictly decreasing and
    the root lies in (max(|m|-E, 0), (Gamma-1) E].
    Returns (P, ok) where ok marks admissible nodes (D > 0, E > sqrt(D^2+|m|^2))."""
    D = U[0]
    m = np.zeros((3,) + D.shape)
    m[:dim] = U[1:1 + dim]
    E = U[1 + dim]
    mm = np.sqrt(_dot(m, m))
    ok = (D > 0) & (E > np.sqrt(D * D + mm * mm))
    Dc = np.where(ok, D, 1.0)
    Ec = np.where(ok, E, 2.0)
    mc = np.where(ok, mm, 0.0)

    def g(p):
        v = mc / (Ec + p)
        sq = np.sqrt(1 - v * v)
        return (G - 1) * ((Ec + p) * (1 - v * v) - p - Dc * sq) - p

    lo = np.maximum(mc - Ec, 0.0)
    hi = (G - 1) * Ec
    for _ in range(maxit):
        mid = 0.5 * (lo + hi)
        gm = g(mid)
        pos = gm > 0
        new_lo = np.where(pos, mid, lo)
        new_hi = np.where(pos, hi, mid)
        if np.array_equal(new_lo, lo) and np.array_equal(new_hi, hi):
            break
        lo, hi = new_lo, new_hi
    p = 0.5 * (lo + hi)
    v = m / (Ec + p)
    W = 1.0 / np.sqrt(1.0 - _dot(v, v))
    rho = Dc / W
    P = np.zeros((8,) + D.shape)
    P[0] = rho
    P[1:4] = W * v
    P[4] = p
    P[:, ~ok] = np.nan
    return P, ok


def con2prim_rmhd(U, G, maxit=400):
    """U = (D, m, E, B) -> full P.  Unknown Z = rho h W^2 with
    v.B = (m.B)/Z,  |v|^2 = (Z^2|m|^2 + (m.B)^2 (2Z + |B|^2)) / (Z^2 (Z + |B|^2)^2),
    p = (Gamma-1)/Gamma (Z/W^2 - D/W),
    f(Z) = Z - p + |B|^2 - |B|^2/(2W^2) - (m.B)^2/(2 Z^2) - E = 0,
    all from the definitions of m and E (eq. RMHDdiv2).  The physical root has
    |v| < 1 and p > 0; it is found by bisection on the bracket where |v| < 1."""
    D, m, E, B = U[0], U[1:4], U[4], U[5:8]
    mm2 = _dot(m, m)
    BB = _dot(B, B)
    mB = _dot(m, B)

    def vsq(Z):
        return (Z * Z * mm2 + mB * mB * (2 * Z + BB)) / (Z * Z * (Z + BB) ** 2)

    def f(Z):
        v2 = np.minimum(vsq(Z), 1 - 1e-300)
        W2 = 1.0 / (1.0 - v2)
        W = np.sqrt(W2)
        p = (G - 1) / G * (Z / W2 - D / W)
        return Z - p + BB - BB / (2 * W2) - mB * mB / (2 * Z * Z) - E

    # bracket: lower end where |v| -> 1 (vsq is decreasing in Z), upper end (Z <= E + p <= ...)
    hi = 2.0 * (E + 1.0) + BB
    lo = np.zeros_like(E) + 1e-300
    # find lower bound with vsq < 1 by bisection on vsq - 1
    a, b = lo, hi
    for _ in range(maxit):
        mid = 0.5 * (a + b)
        bad = vsq(mid) >= 1
        na = np.where(bad, mid, a)
        nb = np.where(bad, b, mid)
        if np.array_equal(na, a) and np.array_equal(nb, b):
            break
        a, b = na, nb
    lo = b
    for _ in range(maxit):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        neg = fm < 0
        nlo = np.where(neg, mid, lo)
        nhi = np.where(neg, hi, mid)
        if np.array_equal(nlo, lo) and np.array_equal(nhi, hi):
            break
        lo, hi = nlo, nhi
    Z = 0.5 * (lo + hi)
    vB = mB / Z
    v = (m + vB * B) / (Z + BB)
    W = 1.0 / np.sqrt(1.0 - _dot(v, v))
    rho = D / W
    p = (G - 1) / G * (Z / (W * W) - rho)
    P = np.concatenate([rho[None], W * v, p[None], B], axis=0)
    ok = (D > 0) & (p > 0) & np.isfinite(p)
    P[:, ~ok] = np.nan
    return P, ok
