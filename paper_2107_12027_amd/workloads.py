"""Seeded synthetic workloads: grids, initial primitive states and scheme parameters.

This module only describes inputs.  It holds none of the scheme's arithmetic (no
conservative variables, fluxes, metrics or mesh equations): both the CPU oracle
and the HIP path start from the same primitive fields and uniform mesh produced
here and convert them with their own code.

Conventions shared by every consumer
------------------------------------
* Node arrays are C-ordered ``[z][y][x]`` (x fastest); a 2D array is ``[y][x]``.
* Axis k of the computational index space (xi_1, xi_2, xi_3) maps to array axis
  ``-1 - k``.
* Periodic axes use nodes x_i = a + i*L/N (no duplicated end point) and
  dxi = 1/N; bounded (outflow) axes use x_i = a + i*L/(N-1) and dxi = 1/(N-1).
  The computational coordinate is xi in [0, 1], so J is about the physical
  cell volume ratio (L/1)^d.
* Primitive fields: rho, u = W v (spatial part of the four-velocity, 3 comps),
  p, B (3 comps).  The velocity spec of a workload (v) is turned into u here
  because u is the field the interface carries.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

PERIODIC = 0
OUTFLOW = 1

RHD = 0
RMHD = 1

SIGMA_RHO = 0
SIGMA_LNRHO = 1
MON_PAPER = 0     # omega = sqrt(1 + alpha |grad sigma| / max |grad sigma|)
MON_SQGRAD = 1    # omega = sqrt(1 + alpha |grad sigma|^2)
MON_GRADLAP = 2   # omega = sqrt(1 + alpha |grad sigma| / max + alpha2 |Lap sigma| / max)


@dataclasses.dataclass
class Grid:
    dim: int
    n: Tuple[int, int, int]          # interior nodes along xi_1, xi_2, xi_3 (n[2] = 1 in 2D)
    bc: Tuple[int, int, int]         # PERIODIC / OUTFLOW per axis
    dxi: Tuple[float, float, float]
    period: Tuple[float, float, float]  # physical period (mesh shift) for periodic axes
    lo: Tuple[float, float, float]
    length: Tuple[float, float, float]

    @property
    def shape(self) -> Tuple[int, ...]:
        """Array shape of an interior node field (C order, x fastest)."""
        if self.dim == 2:
            return (self.n[1], self.n[0])
        return (self.n[2], self.n[1], self.n[0])

    @property
    def nnodes(self) -> int:
        return int(np.prod(self.shape))


@dataclasses.dataclass
class Scheme:
    phys: int = RHD
    gamma: float = 5.0 / 3.0
    order_p: int = 3            # 2p-th order EC flux, WENO-(2p-1) dissipation
    dissipation: int = 1        # 0 = entropy conservative, 1 = entropy stable
    weno_eps: float = 1e-6
    cfl: float = 0.4
    mixed: int = 0              # 1 = FP32 flux/WENO arithmetic with FP64 accumulation


@dataclasses.dataclass
class Monitor:
    enabled: int = 0
    sigma: int = SIGMA_RHO
    form: int = MON_PAPER
    alpha: float = 0.0
    filter_passes: int = 3
    sweeps: int = 10
    alpha2: float = 0.0         # Laplacian weight of MON_GRADLAP


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    scheme: Scheme
    monitor: Monitor
    prim: Dict[str, np.ndarray]      # rho (shape), u (3, *shape), p (shape), B (3, *shape)
    x: np.ndarray                    # (dim, *shape) uniform initial mesh
    steps: int
    t_end: Optional[float] = None


def make_grid(dim: int, n: Sequence[int], bc: Sequence[int],
              lo: Sequence[float] = (0.0, 0.0, 0.0),
              length: Sequence[float] = (1.0, 1.0, 1.0)) -> Grid:
    n3 = [int(n[0]), int(n[1]), int(n[2]) if dim == 3 else 1]
    bc3 = [int(bc[0]), int(bc[1]), int(bc[2]) if dim == 3 else PERIODIC]
    dxi, period = [], []
    for k in range(3):
        if k >= dim:
            dxi.append(1.0)
            period.append(0.0)
        elif bc3[k] == PERIODIC:
            dxi.append(1.0 / n3[k])
            period.append(float(length[k]))
        else:
            dxi.append(1.0 / (n3[k] - 1))
            period.append(0.0)
    return Grid(dim, tuple(n3), tuple(bc3), tuple(dxi), tuple(period),
                tuple(float(a) for a in lo), tuple(float(a) for a in length))


def uniform_mesh(grid: Grid) -> np.ndarray:
    """Uniform initial mesh x(xi): (dim, *shape)."""
    axes = []
    for k in range(grid.dim):
        nk = grid.n[k]
        if grid.bc[k] == PERIODIC:
            axes.append(grid.lo[k] + grid.length[k] * np.arange(nk) / nk)
        else:
            axes.append(grid.lo[k] + grid.length[k] * np.arange(nk) / (nk - 1))
    if grid.dim == 2:
        Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
        return np.stack([X, Y]).astype(np.float64)
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X, Y, Z]).astype(np.float64)


def _four_velocity(v: np.ndarray) -> np.ndarray:
    v2 = np.sum(v * v, axis=0)
    return v / np.sqrt(1.0 - v2)


def _prim(rho, v, p, B) -> Dict[str, np.ndarray]:
    return {"rho": np.ascontiguousarray(rho, dtype=np.float64),
            "u": np.ascontiguousarray(_four_velocity(v), dtype=np.float64),
            "p": np.ascontiguousarray(p, dtype=np.float64),
            "B": np.ascontiguousarray(B, dtype=np.float64)}


# ---------------------------------------------------------------------------
# The five workload families.  Sizes are parameters so tests can run small
# instances with the same structure as the full-size ones.
# ---------------------------------------------------------------------------

def advected_sine(n: int = 64) -> Workload:
    """2D RHD, periodic [0,1)^2, rho = 1 + 0.2 sin 2pi(x+y), v = (0.2, 0.2), p = 1,
    adaptive mesh with omega = sqrt(1 + 10 |grad_xi rho|^2), 10 Jacobi sweeps; run to t = 0.2.
    The density is advected exactly: rho(x, y, t) = 1 + 0.2 sin 2pi(x + y - 0.4 t)."""
    g = make_grid(2, (n, n, 1), (PERIODIC, PERIODIC, PERIODIC))
    x = uniform_mesh(g)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (x[0] + x[1]))
    v = np.zeros((3,) + g.shape)
    v[0] = 0.2
    v[1] = 0.2
    p = np.ones(g.shape)
    B = np.zeros((3,) + g.shape)
    return Workload("rhd2d_advected_sine_%d" % n, g,
                    Scheme(phys=RHD, cfl=0.4),
                    Monitor(enabled=1, sigma=SIGMA_RHO, form=MON_SQGRAD, alpha=10.0,
                            filter_passes=3, sweeps=10),
                    _prim(rho, v, p, B), x, steps=0, t_end=0.2)


def quadrant_riemann(n: int = 400, seed: int = 0, steps: int = 300) -> Workload:
    """2D RHD quadrant Riemann problem on [0,1]^2 with outflow boundaries.  Four
    constant states drawn from ``seed`` in the order NE, NW, SW, SE; per quadrant
    rho ~ U[0.01,1], p ~ U[0.01,1], |v| ~ U[0,0.99), angle ~ U[0,2pi), v_3 = 0.
    Adaptive mesh: paper monitor with alpha = 1200 on sigma = ln rho, 10 sweeps."""
    g = make_grid(2, (n, n, 1), (OUTFLOW, OUTFLOW, PERIODIC))
    x = uniform_mesh(g)
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        r = rng.uniform(0.01, 1.0)
        pr = rng.uniform(0.01, 1.0)
        vm = rng.uniform(0.0, 0.99)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        states.append((r, pr, vm * math.cos(ang), vm * math.sin(ang)))
    east = x[0] > 0.5
    north = x[1] > 0.5
    quads = [east & north, (~east) & north, (~east) & (~north), east & (~north)]
    rho = np.zeros(g.shape)
    p = np.zeros(g.shape)
    v = np.zeros((3,) + g.shape)
    for q, (r, pr, vx, vy) in zip(quads, states):
        rho[q] = r
        p[q] = pr
        v[0][q] = vx
        v[1][q] = vy
    B = np.zeros((3,) + g.shape)
    return Workload("rhd2d_quadrant_riemann_%d_seed%d" % (n, seed), g,
                    Scheme(phys=RHD, cfl=0.4),
                    Monitor(enabled=1, sigma=SIGMA_LNRHO, form=MON_PAPER, alpha=1200.0,
                            filter_passes=3, sweeps=10),
                    _prim(rho, v, p, B), x, steps=steps)


def rmhd_rotor(n: int = 512, steps: int = 200) -> Workload:
    """2D RMHD rotor on [0,1]^2, outflow, static mesh: disk r < r0 = 0.1 about
    (0.5, 0.5) with rho = 10 rotating rigidly at |v| = 0.99 r/r0; rho = 1 outside
    r1 = 0.115; p = 1; B = (1, 0, 0).  Between r0 and r1 the density and the
    speed fall linearly, rho = 1 + 9 f, |v| = 0.99 f with f = (r1 - r)/(r1 - r0),
    the taper of the usual rotor setups (without it the ES scheme, which has no
    positivity limiter, leaves the admissible set in the first step from 128^2)."""
    g = make_grid(2, (n, n, 1), (OUTFLOW, OUTFLOW, PERIODIC))
    x = uniform_mesh(g)
    dx = x[0] - 0.5
    dy = x[1] - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    r0, r1 = 0.1, 0.115
    f = np.clip((r1 - r) / (r1 - r0), 0.0, 1.0)
    inside = r < r0
    rho = np.where(inside, 10.0, 1.0 + 9.0 * f)
    speed = np.where(inside, 0.99 * r / r0, 0.99 * f)
    rs = np.where(r > 0, r, 1.0)
    v = np.zeros((3,) + g.shape)
    v[0] = -speed * dy / rs
    v[1] = speed * dx / rs
    p = np.ones(g.shape)
    B = np.zeros((3,) + g.shape)
    B[0] = 1.0
    return Workload("rmhd2d_rotor_%d" % n, g, Scheme(phys=RMHD, cfl=0.4),
                    Monitor(enabled=0), _prim(rho, v, p, B), x, steps=steps)


def blast3d(n: int = 128, seed: int = 0, steps: int = 100, p_in: float = 1000.0) -> Workload:
    """3D RHD blast wave on [0,1]^3, outflow, adaptive mesh (paper monitor on
    sigma = rho, alpha = 800, 5 sweeps), CFL 0.3: sphere r < 0.1 about the centre
    with p = p_in (1000), p = 1 outside, rho = 1 + U[-0.01, 0.01] iid noise."""
    g = make_grid(3, (n, n, n), (OUTFLOW, OUTFLOW, OUTFLOW))
    x = uniform_mesh(g)
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-0.01, 0.01, size=g.shape)
    r = np.sqrt((x[0] - 0.5) ** 2 + (x[1] - 0.5) ** 2 + (x[2] - 0.5) ** 2)
    p = np.where(r < 0.1, p_in, 1.0)
    v = np.zeros((3,) + g.shape)
    B = np.zeros((3,) + g.shape)
    return Workload("rhd3d_blast_%d" % n, g, Scheme(phys=RHD, cfl=0.3),
                    Monitor(enabled=1, sigma=SIGMA_RHO, form=MON_PAPER, alpha=800.0,
                            filter_passes=3, sweeps=5),
                    _prim(rho, v, p, B), x, steps=steps)


def fourier_modes(seed: int = 0, nmodes: int = 8):
    """The 8 Fourier modes of the adjoint workload: (k_m, l_m) from {-4..4}^2 \\ {0}
    without replacement, then theta_m ~ U[0, 2pi), then c_m ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    pairs = [(a, b) for a in range(-4, 5) for b in range(-4, 5) if (a, b) != (0, 0)]
    idx = rng.choice(len(pairs), size=nmodes, replace=False)
    kl = np.array([pairs[i] for i in idx], dtype=np.float64)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    c = rng.uniform(-1.0, 1.0, size=nmodes)
    return kl, theta, c


def fourier_basis(x: np.ndarray, seed: int = 0) -> np.ndarray:
    """The 8 density modes phi_m = (1/8) cos(2 pi (k_m x + l_m y) + theta_m) on the
    mesh x, shape (8, *shape): rho = 1 + eps sum_m c_m phi_m."""
    kl, theta, c = fourier_modes(seed)
    return np.stack([np.cos(2 * np.pi * (kl[m, 0] * x[0] + kl[m, 1] * x[1]) + theta[m]) / len(c)
                     for m in range(len(c))])


def rhd_fourier(n: int = 256, seed: int = 0, steps: int = 100, eps: float = 0.05,
                coeffs: Optional[np.ndarray] = None) -> Workload:
    """The RHD counterpart of rmhd_fourier (B = 0): 2D RHD, periodic [0,1)^2,
    static mesh, rho = 1 + eps f(x, y) from the same 8 seeded modes, p = 1,
    v = (0.3, 0.2)."""
    g = make_grid(2, (n, n, 1), (PERIODIC, PERIODIC, PERIODIC))
    x = uniform_mesh(g)
    _, _, c = fourier_modes(seed)
    if coeffs is not None:
        c = np.asarray(coeffs, dtype=np.float64)
    rho = 1.0 + eps * np.tensordot(c, fourier_basis(x, seed), axes=1)
    v = np.zeros((3,) + g.shape)
    v[0] = 0.3
    v[1] = 0.2
    p = np.ones(g.shape)
    B = np.zeros((3,) + g.shape)
    return Workload("rhd2d_fourier_%d" % n, g, Scheme(phys=RHD, cfl=0.4),
                    Monitor(enabled=0), _prim(rho, v, p, B), x, steps=steps)


def rmhd_fourier(n: int = 256, seed: int = 0, steps: int = 100, eps: float = 0.05,
                 coeffs: Optional[np.ndarray] = None) -> Workload:
    """2D RMHD, periodic [0,1)^2, static mesh: rho = 1 + eps f(x, y) with
    f = (1/8) sum_m c_m cos(2 pi (k_m x + l_m y) + theta_m), p = 1, v = (0.3, 0.2),
    B = (0.5, 0.5, 0)."""
    g = make_grid(2, (n, n, 1), (PERIODIC, PERIODIC, PERIODIC))
    x = uniform_mesh(g)
    kl, theta, c = fourier_modes(seed)
    if coeffs is not None:
        c = np.asarray(coeffs, dtype=np.float64)
    f = np.zeros(g.shape)
    for m in range(len(c)):
        f += c[m] * np.cos(2 * np.pi * (kl[m, 0] * x[0] + kl[m, 1] * x[1]) + theta[m])
    f /= len(c)
    rho = 1.0 + eps * f
    v = np.zeros((3,) + g.shape)
    v[0] = 0.3
    v[1] = 0.2
    p = np.ones(g.shape)
    B = np.zeros((3,) + g.shape)
    B[0] = 0.5
    B[1] = 0.5
    return Workload("rmhd2d_fourier_%d" % n, g, Scheme(phys=RMHD, cfl=0.4),
                    Monitor(enabled=0), _prim(rho, v, p, B), x, steps=steps)


# ---------------------------------------------------------------------------
# The paper's fixed-state 2D examples, run as MM-O5 (adaptive) and UM-O5 (the
# same scheme on the static uniform mesh) for the time-to-solution comparison.
# ---------------------------------------------------------------------------

# Section 6, RHD Riemann problems I-III: (rho, v1, v2, p) in the quadrants
# x1 > 0.5 & x2 > 0.5, x1 < 0.5 & x2 > 0.5, x1 < 0.5 & x2 < 0.5, x1 > 0.5 & x2 < 0.5
RIEMANN_2D = {
    1: ((0.5, 0.5, -0.5, 5.0), (1.0, 0.5, 0.5, 5.0), (3.0, -0.5, 0.5, 5.0), (1.5, -0.5, -0.5, 5.0)),
    2: ((1.0, 0.0, 0.0, 1.0), (0.5771, -0.3529, 0.0, 0.4), (1.0, -0.3529, -0.3529, 1.0),
        (0.5771, 0.0, -0.3529, 0.4)),
    3: ((0.035145216124503, 0.0, 0.0, 0.162931056509027), (0.1, 0.7, 0.0, 1.0), (0.5, 0.0, 0.0, 1.0),
        (0.1, 0.0, 0.7, 1.0)),
}


def riemann2d(case: int, n: int = 200, adaptive: bool = True) -> Workload:
    """2D RHD Riemann problem I, II or III of Section 6 on [0,1]^2 with outflow
    boundaries, Gamma = 5/3, CFL 0.4, run to t = 0.4.  Adaptive mesh (MM-O5): the
    paper monitor with alpha = 1200 on sigma = ln rho, 3 filter passes, 10 Jacobi
    sweeps; adaptive = False gives UM-O5."""
    g = make_grid(2, (n, n, 1), (OUTFLOW, OUTFLOW, PERIODIC))
    x = uniform_mesh(g)
    east = x[0] > 0.5
    north = x[1] > 0.5
    quads = [east & north, (~east) & north, (~east) & (~north), east & (~north)]
    rho = np.zeros(g.shape)
    p = np.zeros(g.shape)
    v = np.zeros((3,) + g.shape)
    for q, (r, vx, vy, pr) in zip(quads, RIEMANN_2D[case]):
        rho[q] = r
        v[0][q] = vx
        v[1][q] = vy
        p[q] = pr
    B = np.zeros((3,) + g.shape)
    mon = (Monitor(enabled=1, sigma=SIGMA_LNRHO, form=MON_PAPER, alpha=1200.0, filter_passes=3, sweeps=10)
           if adaptive else Monitor(enabled=0))
    return Workload("rhd2d_riemann%d_%s_%d" % (case, "mm" if adaptive else "um", n), g,
                    Scheme(phys=RHD, gamma=5.0 / 3.0, cfl=0.4), mon, _prim(rho, v, p, B), x,
                    steps=0, t_end=0.4)


def rmhd_blast2d(n: int = 150, adaptive: bool = True) -> Workload:
    """2D RMHD blast of Section 6 on [-6,6]^2 with outflow boundaries, Gamma = 4/3,
    CFL 0.4, run to t = 4: rho = 0.01, p = 1 for r < 0.8; rho = 1e-4, p = 5e-4 for
    r > 1; linear in r in between; v = 0; B = (0.1, 0, 0).  Adaptive mesh (MM-O5):
    the paper monitor with alpha = 800 on sigma = ln rho, 3 filter passes, 10
    Jacobi sweeps; adaptive = False gives UM-O5."""
    g = make_grid(2, (n, n, 1), (OUTFLOW, OUTFLOW, PERIODIC), lo=(-6.0, -6.0, 0.0), length=(12.0, 12.0, 1.0))
    x = uniform_mesh(g)
    r = np.sqrt(x[0] * x[0] + x[1] * x[1])
    f = np.clip((1.0 - r) / 0.2, 0.0, 1.0)       # 1 inside r = 0.8, 0 outside r = 1
    rho = 1e-4 + (0.01 - 1e-4) * f
    p = 5e-4 + (1.0 - 5e-4) * f
    v = np.zeros((3,) + g.shape)
    B = np.zeros((3,) + g.shape)
    B[0] = 0.1
    mon = (Monitor(enabled=1, sigma=SIGMA_LNRHO, form=MON_PAPER, alpha=800.0, filter_passes=3, sweeps=10)
           if adaptive else Monitor(enabled=0))
    return Workload("rmhd2d_blast_%s_%d" % ("mm" if adaptive else "um", n), g,
                    Scheme(phys=RMHD, gamma=4.0 / 3.0, cfl=0.4), mon, _prim(rho, v, p, B), x,
                    steps=0, t_end=4.0)


def rmhd_shock_cloud(n: Sequence[int] = (210, 150), adaptive: bool = True) -> Workload:
    """2D RMHD shock-cloud interaction of Section 6 on [-0.2, 1.2] x [0, 1], Gamma =
    5/3, CFL 0.4, run to t = 1.2: a planar shock at x_1 = 0.05 with the post-shock
    state (rho, v, p, B) = (3.86859, (0.68, 0, 0), 1.25115, (0, 0.84981, -0.84981))
    on its left and, on its right, rho = 1, v = 0, p = 0.05, B = (0, 0.16106,
    0.16106) (the printed right tuple ends 0, 0.16106, 0.16106, 0.05, which gives
    p = 0 in the order of the left tuple; read here as B followed by p); a cloud of
    radius 0.15 about (0.25, 0.5) with rho = 30 in the right state.  The paper specifies inflow on the left boundary: the
    left state is super-fast there (every characteristic speed of the x_1
    Jacobian is positive, the slowest being about 0.12), so the zero-gradient
    outflow rule leaves it unchanged and stands in for the inflow condition while
    no wave reaches that boundary.  Adaptive mesh (MM-O5): the paper monitor with
    alpha = 800 on sigma = ln rho, 3 filter passes, 10 Jacobi sweeps."""
    nx, ny = int(n[0]), int(n[1])
    g = make_grid(2, (nx, ny, 1), (OUTFLOW, OUTFLOW, PERIODIC), lo=(-0.2, 0.0, 0.0), length=(1.4, 1.0, 1.0))
    x = uniform_mesh(g)
    left = x[0] < 0.05
    rho = np.where(left, 3.86859, 1.0)
    p = np.where(left, 1.25115, 0.05)
    v = np.zeros((3,) + g.shape)
    v[0] = np.where(left, 0.68, 0.0)
    B = np.zeros((3,) + g.shape)
    B[1] = np.where(left, 0.84981, 0.16106)
    B[2] = np.where(left, -0.84981, 0.16106)
    cloud = (x[0] - 0.25) ** 2 + (x[1] - 0.5) ** 2 < 0.15 ** 2
    rho = np.where(cloud, 30.0, rho)
    mon = (Monitor(enabled=1, sigma=SIGMA_LNRHO, form=MON_PAPER, alpha=800.0, filter_passes=3, sweeps=10)
           if adaptive else Monitor(enabled=0))
    return Workload("rmhd2d_shock_cloud_%s_%dx%d" % ("mm" if adaptive else "um", nx, ny), g,
                    Scheme(phys=RMHD, gamma=5.0 / 3.0, cfl=0.4), mon, _prim(rho, v, p, B), x,
                    steps=0, t_end=1.2)


# (MM-O5 size, UM-O5 size, the paper's MM-O5 / UM-O5 CPU-time ratio)
PAPER_COMPARISONS = {
    "rp1": (lambda n, a: riemann2d(1, n, a), 200, 500, 0.178),
    "rp2": (lambda n, a: riemann2d(2, n, a), 200, 500, 0.306),
    "rp3": (lambda n, a: riemann2d(3, n, a), 200, 600, 0.137),
    "rmhd_blast": (lambda n, a: rmhd_blast2d(n, a), 150, 600, 0.0726),
    "shock_cloud": (lambda n, a: rmhd_shock_cloud(n, a), (210, 150), (560, 400), 0.105),
}


# ---------------------------------------------------------------------------
# The paper's RMHD isentropic vortices (Section 6): closed-form solutions used by
# the accuracy tests, with the prescribed mesh motions of those tests.
#
# The 2D RMHD isentropic vortex of Section 6 (example RMHD_2DVortex): the
# closed-form solution at time t on the periodic domain [-R, R]^2, written out from
# the paper's formulas (a stationary vortex in its rest frame, seen from a frame
# moving with velocity (1/2, 1/2), so that it translates with (-1/2, -1/2)):
#   rho = (1 - sigma e^{1 - r^2})^{1/(Gamma-1)}, p = rho^Gamma,
#   x^_k = 2 k_k R + x_k + t/2 - 1 in [-R, R), x~_k = x^_k + (sqrt 2 - 1)(x^_1 + x^_2)/2,
#   (v~_1, v~_2) = (-x~_2, x~_1) f, f = sqrt(kappa e^{1-r^2} / (kappa r^2 e^{1-r^2}
#       + (Gamma-1) rho + Gamma p)), kappa = 2 Gamma sigma rho + (Gamma-1) B_0^2 (2 - r^2),
#   v = ((2+sqrt2) v~_1 + (2-sqrt2) v~_2 - 2, (2+sqrt2) v~_2 + (2-sqrt2) v~_1 - 2, 0)
#       / (4 - 2 (v~_1 + v~_2)),
#   (B~_1, B~_2) = B_0 e^{(1-r^2)/2} (-x~_2, x~_1),
#   B = ((sqrt2+1) B~_1 - (sqrt2-1) B~_2, (sqrt2+1) B~_2 - (sqrt2-1) B~_1, 0) / 2,
# with Gamma = 5/3, sigma = 0.2, B_0 = 0.05, R = 5.  Complex arguments are allowed
# (complex-step derivatives in t).
#
# Reading of the field profile: the paper prints B~ = B_0 e^{1-r^2}(-x~_2, x~_1).
# The radial balance of the rest-frame vortex (azimuthal v and B, b^2 = B_phi^2,
# b^phi = W B_phi) is d(p + B_phi^2/2)/dr = (rho h W^2 v^2 - B_phi^2)/r; with
# p = rho^Gamma and v = r f it yields exactly the printed f and kappa = 2 Gamma sigma
# rho + (Gamma-1) B_0^2 (2 - r^2) when B_phi = B_0 r e^{(1-r^2)/2}, and a different
# kappa for B_phi = B_0 r e^{1-r^2}.  With the printed exponent the residual of the
# rest-frame vortex stalls at 1e-4 (momentum) under refinement; with the half
# exponent it converges at the design order, so the half exponent is taken.
# ---------------------------------------------------------------------------

VORTEX_GAMMA, VORTEX_SIGMA, VORTEX_B0, VORTEX_R = 5.0 / 3.0, 0.2, 0.05, 5.0


def vortex2d_state(x1, x2, t):
    """(rho, v (3), p, B (3)) of the 2D RMHD vortex at the points (x1, x2) and
    time t (see the section comment above; complex arguments allowed)."""
    s2 = np.sqrt(2.0)
    xh1 = x1 + t / 2.0 - 1.0
    xh2 = x2 + t / 2.0 - 1.0
    # periodic representative in [-R, R) (the shift is real)
    xh1 = xh1 - 2 * VORTEX_R * np.floor((np.real(xh1) + VORTEX_R) / (2 * VORTEX_R))
    xh2 = xh2 - 2 * VORTEX_R * np.floor((np.real(xh2) + VORTEX_R) / (2 * VORTEX_R))
    xt1 = xh1 + (s2 - 1.0) * (xh1 + xh2) / 2.0
    xt2 = xh2 + (s2 - 1.0) * (xh1 + xh2) / 2.0
    r2 = xt1 * xt1 + xt2 * xt2
    e = np.exp(1.0 - r2)
    rho = (1.0 - VORTEX_SIGMA * e) ** (1.0 / (VORTEX_GAMMA - 1.0))
    p = rho ** VORTEX_GAMMA
    kappa = 2 * VORTEX_GAMMA * VORTEX_SIGMA * rho + (VORTEX_GAMMA - 1.0) * VORTEX_B0 ** 2 * (2.0 - r2)
    f = np.sqrt(kappa * e / (kappa * r2 * e + (VORTEX_GAMMA - 1.0) * rho + VORTEX_GAMMA * p))
    vt1, vt2 = -xt2 * f, xt1 * f
    den = 4.0 - 2.0 * (vt1 + vt2)
    v1 = ((2 + s2) * vt1 + (2 - s2) * vt2 - 2.0) / den
    v2 = ((2 + s2) * vt2 + (2 - s2) * vt1 - 2.0) / den
    eb = np.exp(0.5 * (1.0 - r2))
    Bt1, Bt2 = -VORTEX_B0 * eb * xt2, VORTEX_B0 * eb * xt1
    Bx = 0.5 * ((s2 + 1) * Bt1 - (s2 - 1) * Bt2)
    By = 0.5 * ((s2 + 1) * Bt2 - (s2 - 1) * Bt1)
    z = 0.0 * rho
    return rho, np.stack([v1, v2, z]), p, np.stack([Bx, By, z])


def vortex3d_state(x1, x2, x3, t):
    """(rho, v (3), p, B (3)) of the 3D RMHD vortex of Section 6 (example
    RMHD_3DVortex) on the periodic domain [-R, R]^2 x [-5R, 5R]: the rest-frame
    vortex above (same f, kappa and, by the same reading, B~ = B_0 e^{(1-r^2)/2}
    (-x~_2, x~_1)) seen from a frame moving with velocity (1, 1, 1)/2 (W = 2):
      x^_k = x_k + (x_1 + x_2 + x_3)/3 + t,
      (x~_1, x~_2) = (x^_1, x^_2) + k_1 (40/3, 10/3) + k_2 (10/3, 40/3),
      v = (4 v~_1 + v~_2 - 3, 4 v~_2 + v~_1 - 3, v~_1 + v~_2 - 3) / (6 - 3 (v~_1 + v~_2)),
      B = (5 B~_1 - B~_2, 5 B~_2 - B~_1, -B~_1 - B~_2) / 3.
    The lattice (k_1, k_2) is the image of the domain's periods (2R, 0, 0),
    (0, 2R, 0) and (0, 0, 10R) in the rest frame; the representative taken is the
    image nearest to the vortex axis (the paper's Omega_0 is not spelled out; the
    other images differ by less than 1e-9 where they meet)."""
    S = (x1 + x2 + x3) / 3.0
    xh1 = x1 + S + t
    xh2 = x2 + S + t
    best = None
    for k1 in range(-3, 4):
        for k2 in range(-3, 4):
            a1 = xh1 + (40.0 * k1 + 10.0 * k2) / 3.0
            a2 = xh2 + (10.0 * k1 + 40.0 * k2) / 3.0
            rr = np.real(a1) ** 2 + np.real(a2) ** 2
            if best is None:
                best, xt1, xt2 = rr, a1, a2
            else:
                sel = rr < best
                best = np.where(sel, rr, best)
                xt1 = np.where(sel, a1, xt1)
                xt2 = np.where(sel, a2, xt2)
    r2 = xt1 * xt1 + xt2 * xt2
    e = np.exp(1.0 - r2)
    rho = (1.0 - VORTEX_SIGMA * e) ** (1.0 / (VORTEX_GAMMA - 1.0))
    p = rho ** VORTEX_GAMMA
    kappa = 2 * VORTEX_GAMMA * VORTEX_SIGMA * rho + (VORTEX_GAMMA - 1.0) * VORTEX_B0 ** 2 * (2.0 - r2)
    f = np.sqrt(kappa * e / (kappa * r2 * e + (VORTEX_GAMMA - 1.0) * rho + VORTEX_GAMMA * p))
    vt1, vt2 = -xt2 * f, xt1 * f
    den = 6.0 - 3.0 * (vt1 + vt2)
    v = np.stack([4 * vt1 + vt2 - 3.0, 4 * vt2 + vt1 - 3.0, vt1 + vt2 - 3.0]) / den
    eb = np.exp(0.5 * (1.0 - r2))
    Bt1, Bt2 = -VORTEX_B0 * eb * xt2, VORTEX_B0 * eb * xt1
    B = np.stack([5 * Bt1 - Bt2, 5 * Bt2 - Bt1, -Bt1 - Bt2]) / 3.0
    return rho, v, p, B


def vortex_mesh_shape(grid: Grid):
    """(x°, s) of the prescribed node motion of the vortex accuracy tests (eq.
    RMHD_2DVortex_MovingMesh, eq. RMHD_3DVortex_MovingMesh): the mesh at time t is
    x° + a(t) s with a(t) = 0.2 cos(pi t / 4), x° the nodes of the uniform periodic
    mesh and s = (sin(3 pi x°_2/R), sin(3 pi x°_1/R)) in 2D,
    (s_2 s_3, s_3 s_1, s_1 s_2), s_k = sin(3 pi x°_k / L_k), L = (R, R, 5R), in 3D.
    The paper's x° = 2 i R/(N-1) lists both ends of a period on a periodic axis;
    the nodes here are x° = -R + i L/N of the periodic grid (the same displacement
    field up to its sign)."""
    xr = uniform_mesh(grid)
    R = VORTEX_R
    if grid.dim == 2:
        shape = np.stack([np.sin(3 * np.pi * xr[1] / R), np.sin(3 * np.pi * xr[0] / R)])
    else:
        s1 = np.sin(3 * np.pi * xr[0] / R)
        s2 = np.sin(3 * np.pi * xr[1] / R)
        s3 = np.sin(3 * np.pi * xr[2] / (5 * R))
        shape = np.stack([s2 * s3, s3 * s1, s1 * s2])
    return xr, shape


def vortex_mesh_amplitude(t: float) -> float:
    """a(t) = 0.2 cos(pi t / 4) of the prescribed vortex mesh motion."""
    return 0.2 * math.cos(math.pi * t / 4.0)


def vortex_mesh(grid: Grid, t: float):
    """(x, xdot) of the prescribed vortex mesh motion at time t."""
    xr, shape = vortex_mesh_shape(grid)
    return xr + vortex_mesh_amplitude(t) * shape, -0.05 * math.pi * math.sin(math.pi * t / 4.0) * shape


def rmhd_vortex(dim: int, n: int, t: float = 0.0, dissipation: int = 0,
                adaptive: bool = False) -> Workload:
    """The RMHD vortex example of Section 6 in 2D (N x N nodes on [-R, R]^2, run to
    t = 4) or 3D (N x N x 5N nodes on [-R, R]^2 x [-5R, 5R], run to t = 0.1),
    periodic, Gamma = 5/3, CFL 0.4 in 2D and 0.3 in 3D (the paper's numbers for its
    2D and 3D tests), with the state at time t.  adaptive = False: the
    prescribed moving mesh at t (MM-O6 with the EC scheme, dissipation = 0;
    dissipation = 1 runs the ES scheme on it).  adaptive = True: the uniform mesh
    and the adaptive redistribution with the monitor of eq.
    RMHD_2DVortex_Monitor, sigma = rho, alpha = 20 on the gradient and 10 on the
    Laplacian, 3 filter passes and 10 Jacobi sweeps (MM-O5 with dissipation = 1;
    the 3D example takes a monitor like the 2D one)."""
    R = VORTEX_R
    if dim == 2:
        g = make_grid(2, (n, n, 1), (PERIODIC, PERIODIC, PERIODIC), lo=(-R, -R, 0.0),
                      length=(2 * R, 2 * R, 1.0))
    else:
        g = make_grid(3, (n, n, 5 * n), (PERIODIC, PERIODIC, PERIODIC), lo=(-R, -R, -5 * R),
                      length=(2 * R, 2 * R, 10 * R))
    if adaptive:
        x = uniform_mesh(g)
        mon = Monitor(enabled=1, sigma=SIGMA_RHO, form=MON_GRADLAP, alpha=20.0, alpha2=10.0,
                      filter_passes=3, sweeps=10)
    else:
        x, _ = vortex_mesh(g, t)
        mon = Monitor(enabled=0)
    if dim == 2:
        rho, v, p, B = vortex2d_state(x[0], x[1], t)
    else:
        rho, v, p, B = vortex3d_state(x[0], x[1], x[2], t)
    return Workload("rmhd%dd_vortex_%s_%d" % (dim, "mm_adaptive" if adaptive else "mm_prescribed", n), g,
                    Scheme(phys=RMHD, gamma=VORTEX_GAMMA, cfl=0.4 if dim == 2 else 0.3,
                           dissipation=dissipation), mon,
                    _prim(rho, v, p, B), x, steps=0, t_end=4.0 if dim == 2 else 0.1)


# ---------------------------------------------------------------------------
# Random test inputs (parity and invariant tests).
# ---------------------------------------------------------------------------

def random_prim(shape, rng: np.random.Generator, phys: int = RHD, dim: int = 2,
                vmax: float = 0.9, rho_rng=(0.1, 1.0), p_rng=(0.1, 1.0),
                bmax: float = 1.0) -> Dict[str, np.ndarray]:
    """Admissible random primitive state per node (non-smooth)."""
    rho = rng.uniform(*rho_rng, size=shape)
    p = rng.uniform(*p_rng, size=shape)
    ncomp = 3 if (dim == 3 or phys == RMHD) else 2
    dirs = rng.normal(size=(3,) + tuple(shape))
    dirs[ncomp:] = 0.0
    dirs /= np.sqrt(np.sum(dirs * dirs, axis=0))
    vm = rng.uniform(0.0, vmax, size=shape)
    v = dirs * vm
    B = np.zeros((3,) + tuple(shape))
    if phys == RMHD:
        B = rng.uniform(-bmax, bmax, size=(3,) + tuple(shape))
    return _prim(rho, v, p, B)


def smooth_prim(x: np.ndarray, rng: np.random.Generator, phys: int = RHD,
                amp: float = 0.2, period=(1.0, 1.0, 1.0)) -> Dict[str, np.ndarray]:
    """Smooth periodic primitive state on physical points x (dim, *shape)."""
    dim = x.shape[0]
    shape = x.shape[1:]

    def field(scale, off):
        kx = rng.integers(1, 3, size=dim)
        ph = rng.uniform(0, 2 * np.pi)
        arg = sum(2 * np.pi * kx[k] * x[k] / period[k] for k in range(dim))
        return off + scale * np.sin(arg + ph)

    rho = field(amp, 1.0)
    p = field(amp, 1.0)
    ncomp = 3 if (dim == 3 or phys == RMHD) else 2
    v = np.zeros((3,) + shape)
    for c in range(ncomp):
        v[c] = field(0.2, 0.1 * (c + 1))
    B = np.zeros((3,) + shape)
    if phys == RMHD:
        for c in range(3):
            B[c] = field(0.3, 0.4 - 0.2 * c)
    return _prim(rho, v, p, B)


def perturbed_mesh(grid: Grid, rng: np.random.Generator, amp: float = 0.02,
                   t: float = 0.0) -> np.ndarray:
    """Smooth sinusoidal deformation of the uniform mesh that keeps periodicity
    and the bounded-edge normal coordinates (used as a curvilinear test mesh)."""
    x = uniform_mesh(grid)
    xi = []
    for k in range(grid.dim):
        nk = grid.n[k]
        if grid.bc[k] == PERIODIC:
            a = np.arange(nk) / nk
        else:
            a = np.arange(nk) / (nk - 1)
        xi.append(a)
    if grid.dim == 2:
        E2, E1 = np.meshgrid(xi[1], xi[0], indexing="ij")
        E = [E1, E2]
    else:
        E3, E2, E1 = np.meshgrid(xi[2], xi[1], xi[0], indexing="ij")
        E = [E1, E2, E3]
    ph = rng.uniform(0, 2 * np.pi, size=(grid.dim, grid.dim))
    c = np.cos(np.pi * t / 4.0)
    for k in range(grid.dim):
        disp = np.ones(grid.shape)
        for j in range(grid.dim):
            if j == k:
                continue
            disp = disp * np.sin(2 * np.pi * E[j] + ph[k, j])
        # vanish on bounded faces normal to k so the domain stays fixed
        if grid.bc[k] != PERIODIC:
            disp = disp * np.sin(np.pi * E[k])
        else:
            disp = disp * (1.0 + 0.5 * np.sin(2 * np.pi * E[k] + ph[k, k]))
        x[k] = x[k] + amp * c * grid.length[k] * disp
    return x
