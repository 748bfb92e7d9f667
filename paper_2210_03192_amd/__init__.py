"""df3c: 3-center Coulomb integrals (P|ab) and density-fitted J on MI355X.

The GPU library (``libdf3c.so``, HIP for gfx950) is loaded lazily by
``paper_2210_03192_amd.df3c``; importing this package does not touch the GPU.
"""
