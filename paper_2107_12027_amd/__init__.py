"""MI355X (gfx950) implementation of the entropy-stable adaptive moving-mesh
finite-difference residual of Duan & Tang (arXiv 2107.12027) for 2D/3D special
relativistic hydrodynamics and magnetohydrodynamics.

The compute path lives in ``csrc/`` (HIP kernels behind the C ABI declared in
``include/es.h``); ``es`` is the thin ctypes binding.  Import ``es`` explicitly:
this package ``__init__`` imports nothing so that ``workloads`` can be used on
its own.
"""
