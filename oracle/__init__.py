"""FP64 CPU oracle for the grid-hopping hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the package smoke
check and the CPU-baseline leg of the benchmark may import or call anything in
this package.  The GPU library never routes through it, and it shares no code
with the GPU library (the two meet only at the seeded input arrays).

Everything here is plain numpy in float64, written from the paper
("Grid Hopping: Accelerating Direct Estimation Algorithms for Multistatic FMCW
Radar", Monnoyer et al.):

  radar.py   sensing functions, eqs. (1)-(2), and grid axes (Sec. III)
  maps.py    per-receiver zero-padded 2D range-Doppler maps (Sec. III, Sec. IV)
  gh.py      grid-hopping decision: interpolated map values, eq. (7)
  direct.py  direct decision: exact scalar products with the atoms of eq. (3)
  peaks.py   block and global argmax of a decision volume (eqs. (5)-(6))
  bomp.py    one Block-OMP iteration (multi-target extension, Sec. VI)
  refine.py  off-grid Newton refinement of the direct decision
  grad.py    decisions at continuous points with their gradients with respect
             to (x, y, vx, vy) and the receiver positions
  factor.py  the factorised location-then-velocity decisions of eqs. (5)-(6),
             direct and by grid hopping (range spectra with bilinear, Keys or
             polar range interpolation; nearest-bin Doppler)

Every function is pinned by tests in tests/test_oracle_*.py against closed
forms, brute force on tiny inputs, invariants, or values the paper prints.
No function is "parity unpinned".
"""
