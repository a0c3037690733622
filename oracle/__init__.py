"""FP64 CPU oracle for the LRBMS two-phase scheme.

TEST INFRASTRUCTURE ONLY.  Nothing outside ``tests/``, the smoke check and
the CPU-baseline leg of the benchmark may import or call this package.  It
shares no code with the GPU path and exists to be read against the paper:
plain NumPy/SciPy, FP64, following the paper's definitions in order.

Module map (paper sections):
  fem        grid, P1 cell basis, Gauss quadrature, mobilities (Sec. 2, 3.1)
  pressure   SWIP bilinear/linear forms, fine solve, velocity reconstruction
             (Sec. 3.2-3.3, Def. pressureDG / velocityDG)
  transport  DG upwind explicit Euler saturation step and slope limiter
             (Sec. 3.4-3.5, Def. saturationDG, eq. limiterMain)
  tof        DG time-of-flight (Sec. 3.6, eq. timeOfFlight)
  offline    mobility profiles, snapshots, local Gram-Schmidt / PCA,
             affine terms b_q, c, d_q, e (Sec. 4.1-4.4, Alg. 2)
  online     least-squares fit, reduced assembly (AFFINE / DIRECT), reduced
             solve, reconstruction (Sec. 4.4 eq. reducedSystem, Alg. 3 step 5)
  schemes    Alg. 1 (fine IMPES) and Alg. 3 (LRBMS IMPES)
  brute      generic high-order-quadrature assembler for tiny grids (pins)

Pinning status: every function is pinned by tests under tests/oracle except
where its docstring says "parity unpinned".
"""
