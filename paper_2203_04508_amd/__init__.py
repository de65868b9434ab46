"""mcb: pseudopotential multiphase lattice Boltzmann with the multiphase curved boundary
condition of arXiv 2203.04508, as gfx950 HIP kernels behind a C ABI (``libmcb.so``).

The HIP library is loaded lazily by :mod:`paper_2203_04508_amd.mcb`; importing the package
itself loads nothing.
"""
