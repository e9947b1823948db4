"""M(s)stab(l) / IDR(s)stab(l) on AMD MI355X (gfx950).

Sequences A x^(i) = b^(i) with a fixed sparse nonsymmetric A, solved by the
recycling Krylov method of Neuenhofen (arXiv 1604.06043) with hand-written
HIP kernels behind the C ABI of include/mstab.h.

Submodules:
  mstab   -- ctypes binding of libmstab.so (same names as the C functions)
  inputs  -- seeded synthetic workloads (no solver arithmetic)
  build   -- compiles libmstab.so for gfx950
Importing the package loads nothing; the library is loaded on first use.
"""
