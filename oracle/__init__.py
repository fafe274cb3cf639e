"""FP64 CPU reference of the DI-LBM time step -- TEST INFRASTRUCTURE ONLY.

This package is the oracle the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import it; the
product package never does, and shares no code with it.

The arithmetic lives in ``dilbm_oracle.c`` (two dimensions, D2Q9) and
``dilbm3d_oracle.c`` (three dimensions, D3Q19, spheres), plain C in FP64 compiled with
``-O2 -ffp-contract=off``; ``binding`` and ``binding3d`` only marshal numpy arrays through
ctypes.
"""
from .binding import (  # noqa: F401
    OracleParams,
    OracleSolver,
    build_oracle,
    lattice,
    feq,
    phi,
    force_term,
    guo_term,
    collide_node,
    pp_force,
    pw_force,
    body_update,
    num_threads,
    set_num_threads,
)
from . import binding3d  # noqa: F401,E402
