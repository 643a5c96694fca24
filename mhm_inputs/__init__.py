"""Seeded synthetic inputs shared by the oracle and the HIP path.

Holds mesh topology, lattice conventions and random fields only; none of the
local-problem arithmetic lives here.
"""
from .mesh import coarse_mesh, element_vertices, n_nodes, subtri_centroids, subtri_lattice_centroids  # noqa: F401
from .configs import make, sub_batch, build_batch  # noqa: F401
