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
