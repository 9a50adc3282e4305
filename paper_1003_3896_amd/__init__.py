"""MI355X-native (gfx950, HIP) direct-summation N-body hot path.

Softened all-pairs gravity (NBSymple Sect. 2, Eqs. 4-5), the kick/drift stages of the
2nd-order leapfrog and the 6th-order symplectic composition (Sect. 3.1), an analytic external
galactic field (Eq. 3) and the energy / momentum diagnostics of Sect. 5.1, exposed through a
small C ABI (``include/nbody.h``) implemented in ``csrc/`` and bound here with ctypes.

Submodules:
  inputs   seeded synthetic initial conditions (NumPy only)
  nbody    ctypes binding with the C ABI's names (loads ``libnbody.so``; fails loudly if absent)
  serve    continuous-batching request loop on top of ``nbody_substep``
  autotune tile-shape search, cached as JSON
"""
__all__ = ["inputs"]
