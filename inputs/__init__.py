"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package synthesises the data the multigrid method acts on: SU(3) gauge
fields, 5D sources and the random starting vectors of the adaptive setup.  It
holds none of the method's arithmetic (no Dirac operator, no transfer, no
solver): both sides of every parity test receive identical arrays from here.

Canonical interchange layout (C order, complex128):

* 4D site index ``x4 = ((t*Lz + z)*Ly + y)*Lx + x``; direction mu = 0,1,2,3 is
  x, y, z, t.
* fermion field: shape ``(Lt, Lz, Ly, Lx, Ls, 4, 3)`` = (site, s, spin, colour).
* gauge field: shape ``(Lt, Lz, Ly, Lx, 4, 3, 3)`` = U_mu(x)[a, b].

The two-dimensional U(1) problem has its own generators (``u1_2d``).
"""

from .lattice import (  # noqa: F401
    LatticeShape,
    fermion_shape,
    gauge_shape,
    gell_mann,
    random_su3_field,
    ape_smear,
    prepare_gauge,
    gaussian_fermion,
    point_sources,
    random_starts,
    random_coarse_starts,
    random_gauge_transform,
)
from .u1_2d import (  # noqa: F401
    fermion2d_shape,
    plaquette_angles,
    quenched_u1_2d,
    gaussian_fermion2d,
    point_sources2d,
    random_starts2d,
    random_u1_transform,
)
