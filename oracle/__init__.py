"""FP64 CPU oracle for the fused kinetic step and local kinetic sensors.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.
It shares no code with the HIP path.
"""
from .oracle import (  # noqa: F401
    build,
    lattice,
    equilibrium,
    moments,
    sensors,
    d2q9_step,
    d2q25_step,
    run,
    flags_from_sensors,
    ext_sensors,
    EXT_NAMES,
    cv_of,
    ddf_equilibrium,
    ddf_moments,
    ddf_step,
    ddf_run,
    ddf_ext_sensors,
    NSUMS,
)
