"""Plain FP64 CPU oracle for diagonal IMEX SDC on the rotating shallow-water equations.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links this package:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It shares no code
with the HIP implementation; both sides take their seeded inputs from the separate
`workloads` module, which holds no arithmetic of the method.

Every routine is written from the paper (Freese, Goetschel, Lunet, Ruprecht, Schreiber,
"Parallel performance of shared memory parallel spectral deferred corrections"):

* quadrature.py -- Gauss-Legendre grid, Radau-right collocation nodes, the collocation matrix Q
  (Section 4.1) and the MIN-SR-FLEX diagonal coefficients (Section 4.2).
* legendre.py   -- orthonormal associated Legendre functions and H = (1-mu^2) dP/dmu on the grid
  (the spherical-harmonic transform behind Section 3.2).
* sht.py        -- scalar and vector spherical-harmonic transforms, written as direct sums.
* swe.py        -- the split right-hand side of the shallow-water equations of Section 3.2:
  f_I = L_g (implicit) and f_E = L_c + N_a + N_r (explicit), and the solver for
  u - alpha f_I(u) = beta (Section 4.2, required routines).
* sdc.py        -- the diagonal IMEX SDC step (Algorithm 2 with the node update of Section 4.2)
  and the grid loss used for gradients.
* imex2.py      -- IMEX-o2, the reference integrator of Section 3.2 (Strang splitting:
  Crank-Nicolson for L_g, Heun for the rest).

Floating point is FP64 throughout.  Parity status of each function is listed in its module
header; every function is pinned by a CPU test against a value fixed by the paper or by
mathematics (closed forms, library routines, brute force), see tests/test_oracle_*.py.
"""
