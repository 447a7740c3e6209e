"""MI355X (gfx950) shifted-HSS Helmholtz solver.

libhelm.so (HIP kernels + C ABI, see include/helm.h) holds the whole hot
path; `paper_2506_18694_amd.helm` is its thin ctypes binding.
"""

from .helm import Solver, Server, HelmError, lib, LIB_PATH, EXPORTS  # noqa: F401
