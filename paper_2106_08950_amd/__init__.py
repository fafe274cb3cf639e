"""MI355X-native DI-LBM time step (Liu, Huang, Chai & Shi, diffuse-interface lattice
Boltzmann method for fluid-particle interaction).

The step itself is hand-written HIP for gfx950 in ``csrc/`` and built into
``libdilbm.so`` behind the C ABI declared in ``include/dilbm.h``.  ``dilbm`` is the thin
ctypes binding of that ABI; ``serve`` is the continuous-batching request loop; ``inputs``
draws the seeded synthetic workloads.  Importing this package does not load the native
library; the first call into ``dilbm`` does, and raises if it is missing.
"""

__all__ = ["dilbm", "inputs", "serve"]
