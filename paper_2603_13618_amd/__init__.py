"""Fused lattice kinetic step with local kinetic refinement sensors, for
AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``liblks.so`` (hand-written HIP
kernels); ``paper_2603_13618_amd.lks`` is its thin Python binding and
``paper_2603_13618_amd.inputs`` produces the seeded synthetic initial fields.
Importing the package loads nothing: the binding loads the library on first
use and raises if it is missing.
"""
