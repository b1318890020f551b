"""Named workloads: grid, lattice, parameters and frozen refinement thresholds.

Thresholds (theta1, theta2) per sensor (S_KL, S_NEQ, S_PI[, S_Q][, S_QE]) are frozen
from the FP64 reference run at the workload's final step, rounded to two
significant digits (the paper gives its thresholds only inside its figures):
the 90th and 99th percentiles over all cells for the smooth fields, 1 % and
10 % of the maximum for the Riemann problem.  They are inputs here; the
recipe that produced them lives with the test fixtures.
"""
import math

INF = math.inf

DOUBLE_SHEAR_128 = dict(
    name="double shear layer, D2Q9 BGK, 128x128 periodic, tau=0.55, 500 steps",
    lattice=9, nx=128, ny=128, tau=0.55, steps=500, flag_mask=1 | 2,
    thr=[[7.6e-06, 1.3e-05], [0.0014, 0.0019], [0.0018, 0.0024], [INF, INF]],
)

SMOOTH_4096 = dict(
    name="smooth random field, D2Q9 BGK, 4096x4096 periodic, tau=0.52, 100 steps",
    lattice=9, nx=4096, ny=4096, tau=0.52, steps=100, seed=0, cutoff=16,
    flag_mask=1 | 2 | 4,
    thr=[[1.6e-07, 3.1e-07], [0.00043, 0.00062], [0.00026, 0.00037], [INF, INF]],
)

SMOOTH_8192 = dict(
    name="smooth random field, D2Q9 BGK, 8192x8192 periodic, tau=0.52, 500 steps",
    lattice=9, nx=8192, ny=8192, tau=0.52, steps=500, seed=0, cutoff=16,
    flag_mask=1 | 2 | 4,
    thr=None,
)

RIEMANN_2048 = dict(
    name="four-quadrant Riemann problem, D2Q25 FV BGK, 2048x2048 outflow, mu=1e-3, 200 steps",
    lattice=25, nx=2048, ny=2048, mu=1e-3, cfl=0.01, steps=200, seed=0,
    flag_mask=1 | 2 | 4 | 8,
    thr=[[4e-05, 0.0004], [0.00068, 0.0068], [0.001, 0.01], [0.00058, 0.0058]],
)

RIEMANN_2048_DDF = dict(
    name="four-quadrant Riemann problem, D2Q25 FV double distribution (f, g) with the "
         "quasi-equilibrium collision, air (gamma=1.4, Pr=0.71), 2048x2048 outflow, mu=1e-3, "
         "200 steps",
    lattice=25, nx=2048, ny=2048, mu=1e-3, cfl=0.01, steps=200, seed=0, gamma=1.4, prandtl=0.71,
    flag_mask=1 | 2 | 4 | 8 | 16,
    thr=[[0.00041, 0.0041], [0.0022, 0.022], [0.0011, 0.011], [0.0011, 0.011]],
    thr_qe=[0.0006, 0.006],
)

ADJOINT_1024 = dict(
    name="KL-sensor gradient, D2Q9 BGK, 1024x1024 periodic, tau=0.52, 200 steps, checkpoint 20",
    lattice=9, nx=1024, ny=1024, tau=0.52, steps=200, checkpoint=20, seed=0, cutoff=16,
)
