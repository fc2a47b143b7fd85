"""Filtered spectral-element lattice Boltzmann (SELBM) time step with flux
bounce-back walls, for AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``lib/libsel.so`` (hand-written HIP
kernels); ``paper_2509_19171_amd.sel`` is its thin ctypes binding, and
``paper_2509_19171_amd.inputs`` generates seeded meshes and initial fields.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""

__all__ = ["inputs", "sel"]
