"""MI355X-native LBM - Kinematic / Dynamic immersed boundary solver for
deformable capsules (arXiv:1903.03356).

Modules:
  lbib       ctypes binding of the C-ABI HIP library (include/lbib.h)
  workloads  seeded synthetic inputs (grids, walls, capsules)
  build      hipcc build of liblbib.so for gfx950
"""
__all__ = ["lbib", "workloads", "build"]
