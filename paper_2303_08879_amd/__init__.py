"""MI355X-native selective Fock-amplitude library (hot path of arXiv:2303.08879).

Submodules:
  fockdiag   ctypes binding of libfockdiag.so (the C ABI, same names)
  ops        torch-facing helpers and the autograd.Function
  workloads  seeded synthetic inputs (circuits -> Bargmann triples)
  build      hipcc build of the library for gfx950
"""
