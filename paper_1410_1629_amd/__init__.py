"""MI355X-native Monte Carlo dust radiative transfer: the photon-package life
cycle (emission, grid traversal, forced scattering with continuous absorption,
Henyey-Greenstein scattering, peel-off) and its path-replay adjoint, as HIP
kernels for gfx950 behind a C ABI (include/mcrt.h).

Submodules are imported on demand: `workloads` builds seeded inputs and
needs no GPU; `binding` loads the HIP library and fails loudly without it.
"""
__all__ = ["workloads", "binding", "autograd"]
