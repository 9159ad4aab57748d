"""MI355X-native direction-splitting step for weakly compressible flow in
spherical geometry (Frolov, Minev & Takhirov, arXiv 2004.13887).

Submodules:
  inputs   seeded synthetic workloads (grids, materials, initial states)
  dsw      Python binding of the HIP C-ABI library ``libdsw.so``
"""
__all__ = ["inputs", "dsw"]
