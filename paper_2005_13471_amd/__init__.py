"""MI355X-native pixel-basis (box-spline) Gram filtering, back projection and
CG for parallel-beam X-ray CT (Shu & Entezari, arXiv 2005.13471).

The compute path is the HIP library libgramct.so (C ABI in include/gramct.h);
``gramct`` is its Python binding.  ``inputs`` holds the seeded synthetic
workload generators.
"""
