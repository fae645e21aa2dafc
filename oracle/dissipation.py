"""Oracle entropy-stable dissipation (test infrastructure only).

Section 4 (eq. ESFlux_HO): at the face (i, k, +1/2)
    F^_{i+1/2} = F~^{2p}_{i+1/2} - 1/2 D Y <<V~>>^{WENO},   D = lambda^ T^{-1} R(T U),
with
  * T = diag{1, T_0, 1} (RHD) or diag{1, T_0, 1, T_0} (RMHD), T_0 the rotation
    whose first row is the unit metric normal (read with atan2 semantics and no
    trigonometry);
  * lambda^ = max_m |J dxi_k/dt + L_k lambda_m(T U)|, L_k = |J grad xi_k|;
  * R scaled eigenvectors: dU/dV = R R^T, dF_1/dU = R Lambda R^{-1} (for RMHD the
    Godunov-Powell modified Jacobian dF_1/dU + Phi'(V)^T dB_1/dU);
  * WENO-(2p-1) (Jiang-Shu) of V~ = R^T T V along the line, <<V~>> = V~^+ - V~^-;
  * Y_ll = 1 iff <<V~_l>> and [V~_l] = V~_{i+1} - V~_i have the same sign
    (strictly positive product), a jump below Y_TOL |r_l|_1 (|T V_i|_max +
    |T V_i+1|_max) counting as zero.
The face state (the state whose entropy variables are the mean of the two
nodes', so that R R^T [V] = A0(V_mid)[V] is the midpoint rule for
[U] = int A0 dV along the straight path in V), the face metrics and the choice of
basis inside the degenerate eigenvalue cluster are readings of the paper.

The eigen-structure is computed generically and numerically, so that it shares
nothing with any closed form: the primitive-variable Jacobians dU/dP, dF_1/dP,
dV/dP are taken by complex-step differentiation of the physics functions, the
eigenpairs of A_P = (dU/dP)^{-1} dF_1/dP come from LAPACK, and each eigenvector
dP_m maps to dU_m = (dU/dP) dP_m and dV_m = (dV/dP) dP_m.  Scaling r_m = dU_m /
sqrt(dU_m . dV_m) gives R^T A0^{-1} R = I, i.e. R R^T = A0.  In the cluster
lambda = v_n the columns are the canonical A0^{-1}-orthonormal basis obtained
from the cluster projector P_c applied to fixed seed vectors.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph

H_CS = 1e-30
Y_TOL = 1e-10


def rotation(n):
    """T_0 (3x3 per face) with first row n (unit), second row (-n2, n1, 0)/rho_perp,
    third row (-n3 n1/rho_perp, -n3 n2/rho_perp, rho_perp), rho_perp = sqrt(n1^2+n2^2);
    rows (0,1,0), (-n3,0,0) when rho_perp = 0."""
    n1, n2, n3 = n
    rp = np.sqrt(n1 * n1 + n2 * n2)
    safe = rp > 0
    rps = np.where(safe, rp, 1.0)
    T = np.zeros(n1.shape + (3, 3))
    T[..., 0, 0], T[..., 0, 1], T[..., 0, 2] = n1, n2, n3
    T[..., 1, 0] = np.where(safe, -n2 / rps, 0.0)
    T[..., 1, 1] = np.where(safe, n1 / rps, 1.0)
    T[..., 2, 0] = np.where(safe, -n3 * n1 / rps, -n3)
    T[..., 2, 1] = np.where(safe, -n3 * n2 / rps, 0.0)
    T[..., 2, 2] = np.where(safe, rp, 0.0)
    return T


def rotate_full(X, T0, slots):
    """Apply T_0 to the 3-vector slots of a full 8-vector field X (8, N)."""
    out = X.copy()
    for s in slots:
        vec = X[s:s + 3]
        out[s:s + 3] = np.einsum("nab,bn->an", T0, vec)
    return out


def unrotate_full(X, T0, slots):
    out = X.copy()
    for s in slots:
        vec = X[s:s + 3]
        out[s:s + 3] = np.einsum("nba,bn->an", T0, vec)
    return out


def _jac(fun, P, sel, G):
    """Complex-step Jacobian d fun_sel / d P_sel, shape (N, m, m)."""
    m = len(sel)
    N = P.shape[1]
    J = np.zeros((N, m, m))
    for b, sb in enumerate(sel):
        Pc = P.astype(complex)
        Pc[sb] = Pc[sb] + 1j * H_CS
        val = fun(Pc)
        J[:, :, b] = (val[sel].imag / H_CS).T
    return J


def cluster_size(phys, dim):
    if phys == ph.RMHD:
        return 2
    return 2 if dim == 2 else 3


def cluster_seeds(phys, dim):
    """Seed slots (selected-system indices) for the canonical cluster basis:
    e_D then the transverse momenta (RHD), e_D then e_{B_n} (RMHD)."""
    if phys == ph.RMHD:
        return [0, 5]
    return [0, 2] if dim == 2 else [0, 2, 3]


# RMHD eigen-groups: eigenvalues closer than GROUP_TOL form one group (the
# eigenvectors of nearly equal eigenvalues are ill-conditioned, those of equal
# ones not unique); a seed contributes a basis vector when its projection left
# after Gram-Schmidt exceeds SEED_TOL times its A0^{-1} norm.
GROUP_TOL = 1e-6
SEED_TOL = 1e-3
SEEDS_CLUSTER = [0, 5, 1, 2, 3, 4, 6, 7]      # e_D, e_{B_n}, then the other slots
SEEDS_OTHER = [0, 1, 2, 3, 4, 5, 6, 7]


def _eigensystem_rmhd(JU, JF, JV, vn):
    """Scaled eigen-structure of the Godunov-Powell modified RMHD Jacobian with a
    canonical basis in every group of (nearly) equal eigenvalues.

    In entropy variables A0 = dU/dV = JU JV^{-1} is SPD and S = dF/dV = JF JV^{-1}
    symmetric; with A0 = L L^T and L^{-1} S L^{-T} = Z diag(lam) Z^T, the columns
    r = L z satisfy R R^T = A0 and (dF/dU) R = R diag(lam), and r_a^T A0^{-1} r_b =
    z_a . z_b.  In each group g (connected chains of eigenvalues within GROUP_TOL)
    the basis is the A0^{-1}-Gram-Schmidt sequence of the projections of unit seeds
    e_s onto the group's eigenspace, P_g e_s = sum_{a in g} r_a (r_a^T A0^{-1} e_s);
    the group holding v_n (entropy and div B waves) takes the seeds e_D, e_{B_n}
    first, every other group e_1, e_2, ...  The result does not depend on how the
    eigensolver chose bases inside a group.  Columns in ascending eigenvalue order."""
    N, m, _ = JU.shape
    X = np.linalg.inv(JV)
    A0 = np.einsum("nab,nbc->nac", JU, X)
    S = np.einsum("nab,nbc->nac", JF, X)
    A0 = 0.5 * (A0 + np.transpose(A0, (0, 2, 1)))
    S = 0.5 * (S + np.transpose(S, (0, 2, 1)))
    L = np.linalg.cholesky(A0)
    Linv = np.linalg.inv(L)
    Q = np.einsum("nab,nbc,ndc->nad", Linv, S, Linv)
    Q = 0.5 * (Q + np.transpose(Q, (0, 2, 1)))
    lam, Z = np.linalg.eigh(Q)                        # ascending; Z columns orthonormal
    return lam, canonical_group_basis(lam, Z, L, Linv, vn)


def group_labels(lam):
    """Eigen-groups of (N, m) ascending eigenvalues: label of each eigenvalue = the
    smallest index of its chain of neighbours closer than GROUP_TOL."""
    N, m = lam.shape
    lab = np.tile(np.arange(m), (N, 1))
    close = np.abs(lam[:, :, None] - lam[:, None, :]) <= GROUP_TOL
    for _ in range(m):
        lab = np.min(np.where(close, lab[:, None, :], m), axis=2)
    return lab


# the group labels and the seed slot accepted for every column of the last
# canonical_group_basis call (for studies of the decisions' sensitivity)
last_group_decisions = {}


def canonical_group_basis(lam, Z, L, Linv, vn):
    """R (N, m, m) from eigenvalues lam (N, m), orthonormal eigenvectors Z of
    L^{-1} S L^{-T} (columns) and the Cholesky factor L of A0 (see _eigensystem_rmhd)."""
    N, m = lam.shape
    rows = np.arange(N)
    lab = group_labels(lam)
    lab_c = lab[rows, np.argmin(np.abs(lam - vn[:, None]), axis=1)]
    C = np.einsum("nia,nis->nas", Z, Linv)            # z_a . (L^{-1} e_s)
    ynorm = np.sqrt(np.sum(Linv * Linv, axis=1))      # |L^{-1} e_s| (A0^{-1} norm of e_s)
    canon = np.zeros((N, m, m))                       # canon[:, :, i]: z-space column i
    seed_of = np.full((N, m), -1)
    for i in range(m):
        ing = lab == lab[:, i:i + 1]                  # (N, m) members of the group of i
        is_c = lab[:, i] == lab_c
        done = np.zeros(N, dtype=bool)
        for t in range(m):
            sidx = np.where(is_c, SEEDS_CLUSTER[t], SEEDS_OTHER[t])
            coef = C[rows, :, sidx] * ing              # (N, m)
            p = np.einsum("nia,na->ni", Z, coef)
            for j in range(i):
                same = (lab[:, j] == lab[:, i])[:, None]
                qj = canon[:, :, j]
                p = p - same * np.sum(qj * p, axis=1)[:, None] * qj
            nrm = np.sqrt(np.sum(p * p, axis=1))
            acc = (~done) & (nrm > SEED_TOL * ynorm[rows, sidx])
            canon[acc, :, i] = p[acc] / nrm[acc, None]
            seed_of[acc, i] = sidx[acc]
            done |= acc
    last_group_decisions["labels"] = lab
    last_group_decisions["seeds"] = seed_of
    return np.einsum("nab,nbc->nac", L, canon)


def eigensystem(Pr, G, phys, dim):
    """Numeric scaled eigen-structure at rotated face states Pr (8, N):
    returns (lam (N, m), R (N, m, m)) with R R^T = dU/dV and (dF_1/dU) R = R diag(lam)."""
    sel = ph.comps(phys, dim)
    m = len(sel)
    JU = _jac(lambda P: ph.cons(P, G), Pr, sel, G)
    JF = _jac(lambda P: ph.flux(P, G, 0), Pr, sel, G)
    JV = _jac(lambda P: ph.entropy_vars(P, G), Pr, sel, G)
    vn = Pr[1] / np.sqrt(1.0 + Pr[1] ** 2 + Pr[2] ** 2 + Pr[3] ** 2)
    if phys == ph.RMHD:
        # Godunov-Powell modification: + Phi'(V) (dB_1/dP), B_1 is primitive slot 5
        Phip = ph.phi_prime(Pr, G)[sel].T          # (N, m)
        JF = JF.copy()
        JF[:, :, 5] += Phip
        return _eigensystem_rmhd(JU, JF, JV, vn)
    AP = np.linalg.solve(JU, JF)
    lam = np.linalg.eigvals(AP).real
    c = cluster_size(phys, dim)
    order = np.argsort(np.abs(lam - vn[:, None]), axis=1)
    # Eigenvectors of the simple eigenvalues: the null vector of A_P - lambda I from
    # an SVD.  (LAPACK's general eigenvector routine balances the matrix first; with
    # entries of order 1e-50 next to entries of order one, as at a state at rest up
    # to rounding, the balanced back-transformation returned vectors with residuals
    # of order one.)
    eye = np.eye(m)[None]
    dP = np.empty_like(AP)
    for k in range(m):
        _, _, vk = np.linalg.svd(AP - lam[:, k, None, None] * eye)
        dP[:, :, k] = vk[:, m - 1, :]
    # The cluster lambda = v_n is semi-simple: its invariant subspace is taken from
    # the null space of A_P - v_n I (SVD), which stays well conditioned where the
    # individual eigenvectors of a repeated eigenvalue are not.
    _, _, vh = np.linalg.svd(AP - vn[:, None, None] * np.eye(m)[None])
    null = np.transpose(vh[:, m - c:, :], (0, 2, 1))                   # (N, m, c)
    idx_cl = order[:, :c]
    for q in range(c):
        np.put_along_axis(dP, idx_cl[:, q][:, None, None].repeat(m, axis=1),
                          null[:, :, q][:, :, None], axis=2)
    dU = np.einsum("nab,nbm->nam", JU, dP)
    dV = np.einsum("nab,nbm->nam", JV, dP)
    # non-degenerate columns
    norm = np.sqrt(np.einsum("nam,nam->nm", dU, dV))
    R = dU / norm[:, None, :]
    # cluster: canonical A0^{-1}-orthonormal basis from the projector
    A0inv = np.einsum("nab,nbc->nac", JV, np.linalg.inv(JU))
    A0inv = 0.5 * (A0inv + np.transpose(A0inv, (0, 2, 1)))
    K = np.take_along_axis(dU, idx_cl[:, None, :].repeat(m, axis=1), axis=2)   # (N, m, c)
    Gm = np.einsum("nac,nab,nbd->ncd", K, A0inv, K)
    Pc = np.einsum("nac,ncd,nbd,nbe->nae", K, np.linalg.inv(Gm), K, A0inv)
    cols = []
    for s in cluster_seeds(phys, dim):
        w_ = Pc[:, :, s].copy()
        for r in cols:
            w_ = w_ - np.einsum("na,nab,nb->n", r, A0inv, w_)[:, None] * r
        w_ = w_ / np.sqrt(np.einsum("na,nab,nb->n", w_, A0inv, w_))[:, None]
        cols.append(w_)
    for q in range(c):
        np.put_along_axis(R, idx_cl[:, q][:, None, None].repeat(m, axis=1),
                          cols[q][:, :, None], axis=2)
        np.put_along_axis(lam, idx_cl[:, q][:, None], vn[:, None], axis=1)
    # canonical column order: the other eigenvalues ascending, then the cluster
    # columns in seed order (so that a column index names the same wave at nearby
    # states)
    rest = order[:, c:]
    rest = np.take_along_axis(rest, np.argsort(np.take_along_axis(lam, rest, axis=1), axis=1), axis=1)
    perm = np.concatenate([rest, idx_cl], axis=1)                     # (N, m)
    lam = np.take_along_axis(lam, perm, axis=1)
    R = np.take_along_axis(R, perm[:, None, :].repeat(m, axis=1), axis=2)
    return lam, R


def weno5_minus(a, b, c, d, e, eps):
    """WENO5-JS value at i+1/2 from v_{i-2..i+2} = (a, b, c, d, e) (Jiang-Shu 1996)."""
    q0 = (2 * a - 7 * b + 11 * c) / 6.0
    q1 = (-b + 5 * c + 2 * d) / 6.0
    q2 = (2 * c + 5 * d - e) / 6.0
    b0 = 13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
    a0 = 0.1 / (eps + b0) ** 2
    a1 = 0.6 / (eps + b1) ** 2
    a2 = 0.3 / (eps + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def weno3_minus(a, b, c, eps):
    """WENO3-JS value at i+1/2 from v_{i-1..i+1} = (a, b, c) (Jiang-Shu 1996, w = 3):
    candidates (3b - a)/2 and (b + c)/2 with linear weights 1/3, 2/3 and
    smoothness indicators (b - a)^2, (c - b)^2."""
    q0 = (-a + 3 * b) / 2.0
    q1 = (b + c) / 2.0
    a0 = (1.0 / 3.0) / (eps + (b - a) ** 2) ** 2
    a1 = (2.0 / 3.0) / (eps + (c - b) ** 2) ** 2
    return (a0 * q0 + a1 * q1) / (a0 + a1)


def _frac_solve(A, b):
    """Exact solution of A y = b over the rationals (Gauss-Jordan, no pivoting needed
    for the nonsingular Vandermonde-like systems below beyond a nonzero search)."""
    from fractions import Fraction
    n = len(A)
    M = [[Fraction(v) for v in row] + [Fraction(b[r])] for r, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b_ for a, b_ in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def weno_js_tables(r):
    """The WENO-JS scheme of order 2r - 1 (Jiang and Shu 1996; Balsara and Shu 2000 for
    r = 4) written out from its definition, in exact rational arithmetic, for the value
    at x_{i+1/2} from v_{i-r+1..i+r-1} (unit spacing, node i at x = 0, v read as the
    averages over the cells [l - 1/2, l + 1/2], as finite-difference WENO does):
      * candidate k = 0..r-1 on the cells i-r+1+k..i+k: the polynomial p_k of degree
        r-1 with those averages, evaluated at x = 1/2: q_k = c_k . v_{S_k};
      * its smoothness indicator beta_k = sum_{l=1}^{r-1} int_{-1/2}^{1/2} (p_k^(l))^2 dx,
        a quadratic form v_{S_k}^T B_k v_{S_k};
      * linear weights d_k with sum_k d_k q_k = the value of the degree 2r-2 polynomial
        with the averages of all 2r-1 cells.
    Returns (c, B, d): c (r, r), B (r, r, r), d (r,) as Fractions.  (For evaluation
    see weno_js_squares: B_k written as a weighted sum of squares.)"""
    from fractions import Fraction

    def cell_avg_row(l, deg):
        # int_{l-1/2}^{l+1/2} x^m dx for m = 0..deg
        a, b = Fraction(2 * l - 1, 2), Fraction(2 * l + 1, 2)
        return [(b ** (m + 1) - a ** (m + 1)) / (m + 1) for m in range(deg + 1)]

    def value_weights(cells, x0):
        # weights w with p(x0) = w . averages for the interpolating polynomial of the cells
        deg = len(cells) - 1
        A = [cell_avg_row(l, deg) for l in cells]              # averages = A coef
        At = [[A[rr][cc] for rr in range(len(cells))] for cc in range(deg + 1)]
        e = [x0 ** m for m in range(deg + 1)]                  # p(x0) = e . coef = e . A^{-1} avg
        return _frac_solve(At, e)                              # w = A^{-T} e

    half = Fraction(1, 2)
    c, B = [], []
    for k in range(r):
        cells = list(range(-r + 1 + k, k + 1))
        c.append(value_weights(cells, half))
        # beta_k: coefficients of p_k are A^{-1} v; the l-th derivative and the
        # integrals of products of monomials over [-1/2, 1/2]
        deg = r - 1
        A = [cell_avg_row(l, deg) for l in cells]
        Ainv_cols = []
        for j in range(r):
            ej = [Fraction(int(i == j)) for i in range(r)]
            Ainv_cols.append(_frac_solve(A, ej))                # coefficients of the basis p with avg e_j
        Q = [[Fraction(0)] * r for _ in range(r)]
        for l in range(1, r):
            # derivative of order l of the monomial coefficient vectors
            def deriv(coef):
                out = list(coef)
                for _ in range(l):
                    out = [out[m] * m for m in range(1, len(out))]
                return out
            D = [deriv(col) for col in Ainv_cols]
            for a in range(r):
                for b in range(r):
                    acc = Fraction(0)
                    for m1, u in enumerate(D[a]):
                        for m2, w in enumerate(D[b]):
                            if (m1 + m2) % 2 == 0:              # odd powers integrate to 0
                                acc += u * w * 2 * half ** (m1 + m2 + 1) / (m1 + m2 + 1)
                    Q[a][b] += acc
        B.append(Q)
    big = value_weights(list(range(-r + 1, r)), half)          # 2r - 1 cells
    # sum_k d_k (c_k placed at offset k) = big: an overdetermined consistent system,
    # solved on the first r rows (the cells i-r+1..i) where the triangular structure
    # fixes d_0, d_1, ... in turn, then checked on all rows
    M = [[c[k][row - k] if 0 <= row - k < r else Fraction(0) for k in range(r)] for row in range(2 * r - 1)]
    d = _frac_solve(M[:r], big[:r])
    for row in range(2 * r - 1):
        assert sum(M[row][k] * d[k] for k in range(r)) == big[row]
    return c, B, d


def weno_js_squares(r):
    """beta_k of weno_js_tables as a weighted sum of squares, beta_k = sum_m D_m (w_km . v)^2:
    the integrals of the squared derivatives are a positive definite quadratic form
    G in the non-constant Taylor coefficients (c_1..c_{r-1}) of p_k at the cell
    centre, G = L diag(D) L^T (exact LDL^T), and w_km = (L^T)_m (those coefficients as
    linear forms in the stencil values).  Each w_km annihilates constants, so the
    squares are of differences of v: this evaluation has none of the cancellation of
    the expanded quadratic form, whose terms are larger than beta by the square of
    the data over its variation.  Returns (D (r-1,), W (r, r-1, r)) as Fractions."""
    from fractions import Fraction
    half = Fraction(1, 2)
    deg = r - 1

    def mono_int(e):       # int_{-1/2}^{1/2} x^e dx
        return Fraction(0) if e % 2 else 2 * half ** (e + 1) / (e + 1)

    # G[a][b] over monomials a, b = 1..deg: sum_l int (x^a)^(l) (x^b)^(l)
    def falling(a, l):
        out = 1
        for t in range(l):
            out *= a - t
        return out
    G = [[sum(falling(a, l) * falling(b, l) * mono_int(a + b - 2 * l)
              for l in range(1, deg + 1) if l <= a and l <= b)
          for b in range(1, deg + 1)] for a in range(1, deg + 1)]
    # LDL^T
    n = deg
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    D = [Fraction(0)] * n
    for j in range(n):
        D[j] = G[j][j] - sum(L[j][t] ** 2 * D[t] for t in range(j))
        for i in range(j + 1, n):
            L[i][j] = (G[i][j] - sum(L[i][t] * L[j][t] * D[t] for t in range(j))) / D[j]
    W = []
    for k in range(r):
        cells = list(range(-r + 1 + k, k + 1))
        A = [[(Fraction(2 * l + 1, 2) ** (m + 1) - Fraction(2 * l - 1, 2) ** (m + 1)) / (m + 1)
              for m in range(r)] for l in cells]
        # rows 1..deg of A^{-1}: the Taylor coefficients c_1..c_deg as linear forms
        inv_cols = [_frac_solve(A, [Fraction(int(i == j)) for i in range(r)]) for j in range(r)]
        Crow = [[inv_cols[j][m] for j in range(r)] for m in range(1, r)]
        Wk = [[sum(L[t][mm] * Crow[t][j] for t in range(n)) for j in range(r)] for mm in range(n)]
        W.append(Wk)
    return D, W


_WENO_TABLES = {}


def weno_js_minus(vs, eps):
    """The WENO-JS value at i+1/2 (order 2r - 1) from the 2r - 1 values v_{i-r+1..i+r-1},
    with the tables of weno_js_tables (beta_k by weno_js_squares): nonlinear weights
    d_k / (eps + beta_k)^2."""
    r = (len(vs) + 1) // 2
    if r not in _WENO_TABLES:
        c, _, d = weno_js_tables(r)
        Dm, W = weno_js_squares(r)
        _WENO_TABLES[r] = (np.array([[float(v) for v in row] for row in c]),
                           np.array([float(v) for v in Dm]),
                           np.array([[[float(v) for v in row] for row in Wk] for Wk in W]),
                           np.array([float(v) for v in d]))
    c, Dm, W, d = _WENO_TABLES[r]
    num = 0.0
    den = 0.0
    for k in range(r):
        S = vs[k:k + r]
        q = sum(c[k][j] * S[j] for j in range(r))
        beta = sum(Dm[m] * sum(W[k][m][j] * S[j] for j in range(r)) ** 2 for m in range(r - 1))
        alpha = d[k] / (eps + beta) ** 2
        num = num + alpha * q
        den = den + alpha
    return num / den


def weno_minus(vs, eps):
    """The w-th order WENO-JS value at i+1/2 from the w values v_{i-(w-1)/2..i+(w-1)/2}:
    WENO5 and WENO3 in their published closed forms, WENO7 from weno_js_tables."""
    if len(vs) == 5:
        return weno5_minus(*vs, eps)
    if len(vs) == 3:
        return weno3_minus(*vs, eps)
    if len(vs) == 7:
        return weno_js_minus(vs, eps)
    raise ValueError("WENO order %d is not implemented" % len(vs))


def face_dissipation(Pst, ast, G, phys, dim, eps, details=False, Y_fixed=None, eig_fixed=None):
    """ES dissipation vector d = D Y <<V~>> at faces.
    Pst: (2p, 8, N) full primitive states of the stencil nodes i-p+1..i+p of each
    face (p = 3: WENO5 on i-2..i+3; p = 2: WENO3 on i-1..i+2, w = 2p - 1);
    ast: (2, d+1, N) metric vectors of nodes i and i+1.
    Y_fixed: optional (m, N) sign-switch values to use instead of evaluating Y
    (the switch held fixed, for difference quotients of the smooth part).
    eig_fixed: optional (R, lhat) of an earlier call, used instead of the face
    eigen-structure (held fixed for the same purpose).
    Returns the full 8-slot d (8, N) (zeros in unused slots)."""
    sel = ph.comps(phys, dim)
    m = len(sel)
    abar = 0.5 * (ast[0] + ast[1])
    ax = np.zeros((3,) + abar.shape[1:])
    ax[:dim] = abar[1:1 + dim]
    L = np.sqrt(np.sum(ax * ax, axis=0))
    n = ax / L
    T0 = rotation(n)
    slots = [1, 5] if phys == ph.RMHD else [1]
    # face state: the state whose entropy variables are the mean of the two nodes'
    ns = len(Pst)
    ci = ns // 2 - 1                      # stencil index of node i (i+1 is ci + 1)
    Vbar = 0.5 * (ph.entropy_vars(Pst[ci], G) + ph.entropy_vars(Pst[ci + 1], G))
    Pbar = ph.prim_from_entropy_vars(Vbar, G)
    if phys == ph.RHD:
        Pbar[5:8] = 0.0
    Pr = rotate_full(Pbar, T0, slots)
    lam, R = eigensystem(Pr, G, phys, dim)
    lhat = np.max(np.abs(abar[0][:, None] + L[:, None] * lam), axis=1)
    if eig_fixed is not None:
        R, lhat = eig_fixed
    Vt = []
    for j in range(ns):
        Vj = rotate_full(ph.entropy_vars(Pst[j], G), T0, slots)[sel]   # (m, N)
        Vt.append(np.einsum("nab,an->bn", R, Vj))                       # R^T T V
    vm = weno_minus(Vt[0:ns - 1], eps)                                  # from the left
    vp = weno_minus(Vt[ns - 1:0:-1], eps)                               # from the right
    jump_weno = vp - vm
    jump = Vt[ci + 1] - Vt[ci]
    # sign(0) reading: a jump [V~_l] within rounding of zero counts as zero, so Y_l = 0.
    # Rounding level: Y_TOL times |r_l|_1 (|T V_i|_max + |T V_i+1|_max), a scale that
    # does not shrink with the components a column happens to touch (the transverse
    # momentum entries of a state at rest are themselves rounding residue).
    Vi = rotate_full(ph.entropy_vars(Pst[ci], G), T0, slots)[sel]
    Vj = rotate_full(ph.entropy_vars(Pst[ci + 1], G), T0, slots)[sel]
    scale = np.sum(np.abs(R), axis=1).T * (np.max(np.abs(Vi), axis=0) + np.max(np.abs(Vj), axis=0))[None, :]
    Y = ((jump_weno * jump > 0) & (np.abs(jump) > Y_TOL * scale)).astype(np.float64)
    if Y_fixed is not None:
        Y = Y_fixed
    coef = Y * jump_weno                                                 # (m, N)
    dsel = lhat[None, :] * np.einsum("nab,bn->an", R, coef)              # R (Y <<V~>>)
    dfull = np.zeros((8,) + dsel.shape[1:])
    dfull[sel] = dsel
    dfull = unrotate_full(dfull, T0, slots)                              # T^{-1}
    if details:
        return dfull, dict(lam=lam, R=R, lhat=lhat, jump=jump, jump_weno=jump_weno, Y=Y,
                           T0=T0, Pr=Pr, L=L)
    return dfull
