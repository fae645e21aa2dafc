"""Small helpers shared by the oracle tests (no method arithmetic)."""
import numpy as np

from oracle import physics as ph
from paper_2107_12027_amd import workloads as wl


def rand_P(n, rng, phys=ph.RHD, dim=2, vmax=0.99, lo=0.01):
    pr = wl.random_prim((n,), rng, phys=phys, dim=dim, vmax=vmax, rho_rng=(lo, 1.0),
                        p_rng=(lo, 1.0))
    return ph.full_prim(pr["rho"], pr["u"], pr["p"], pr["B"])


def cstep(fun, P, slot, h=1e-30):
    Pc = P.astype(complex)
    Pc[slot] = Pc[slot] + 1j * h
    return fun(Pc).imag / h


def prim_from_V(V, G, phys, dim):
    """Explicit inverse of the entropy-variable map (Section 2): beta = sqrt(V_5^2 - |V_u|^2),
    u = V_u/beta, ln rho = V_1 - Gamma/(Gamma-1) - ln(beta)/(Gamma-1) - beta,
    B = W b - b^0 u with b = V_B/beta and b^0 = u.b/W ... (b^0 = u.B, b = (B + b^0 u)/W
    => u.b = b^0 (1 + |u|^2)/W = b^0 W, so b^0 = u.b / W and B = W b - b^0 u)."""
    beta = np.sqrt(V[4] ** 2 - V[1] ** 2 - V[2] ** 2 - V[3] ** 2)
    u = V[1:4] / beta
    W = -V[4] / beta
    lnrho = V[0] - G / (G - 1) - np.log(beta) / (G - 1) - beta
    rho = np.exp(lnrho)
    p = rho / beta
    b = V[5:8] / beta
    b0 = (u[0] * b[0] + u[1] * b[1] + u[2] * b[2]) / W
    B = W * b - b0 * u
    return np.concatenate([rho[None], u, p[None], B], axis=0)
