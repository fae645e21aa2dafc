"""CPU reference oracle for the entropy-stable adaptive moving-mesh scheme of
Duan & Tang, "High-order accurate entropy stable adaptive moving mesh finite
difference schemes for special relativistic (magneto)hydrodynamics"
(arXiv 2107.12027).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
HIP path never calls it, and it shares no code with the HIP path: the only
common module is ``paper_2107_12027_amd.workloads`` (seeded input generators,
which hold none of the scheme's arithmetic).

Plain numpy in float64, vectorised over nodes and faces only; every function
follows a passage of the paper (cited by section and equation label) or a
stated reading of it where the paper is silent or garbled.

Modules
  physics      equation of state, U/F/V, entropy pair, potentials, con2prim
  ecflux       logarithmic mean, two-point EC fluxes (RHD and RMHD)
  metrics      conservative-metric-method spatial metrics, temporal metrics, J
  dissipation  rotation T, eigen-structure, WENO, sign switch, ES dissipation
  residual     the 2p-th order semi-discrete scheme and the VCL
  mesh         monitor, low-pass filter, Jacobi sweeps, mesh-move limiter
  stepper      CFL time step and SSP-RK3 step
"""
