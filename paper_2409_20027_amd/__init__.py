"""Parallel-in-time LQ subproblem solver for MI355X (gfx950).

The solver itself lives in the HIP library built from ``csrc/`` and is reached
through :mod:`paper_2409_20027_amd.lqscan`.  Importing this package loads
nothing; ``workloads`` only draws seeded synthetic inputs.
"""
