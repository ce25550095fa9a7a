"""MI355X (gfx950) implementation of the semi-implicit SPH viscous solve:
the robust, reduction-friendly BiCGSTAB of Bilotta et al. (arXiv 2206.14780)
over a neighbour-sum viscous operator, as hand-written HIP kernels behind a
C-ABI library (`include/sph.h`).

`paper_2206_14780_amd.sph` is the Python binding (argument marshalling only);
`paper_2206_14780_amd.workloads` lays out seeded synthetic particle fields.
Nothing is loaded at import time.
"""
__all__ = ["sph", "workloads"]
