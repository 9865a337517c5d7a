"""CPU FP64 oracle of the pressure projection -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded NumPy/SciPy code that defines what the HIP
library must compute.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the library: both receive the same seeded input
arrays (from the fixtures module) and compute everything else on their own.

Modules
    grid      one-dimensional grid metrics (Gridding section)
    geometry  fractional face areas, cell fractions, active set, small-cell
              merging (Enforcement of Body Boundary Conditions section)
    operator  density, face coefficients, the cut-cell flux-form operator and
              its group Jacobi diagonal, right-hand side, projection and
              divergence (eqs. density, pois, poisson1, integral2, runge1,
              diverge; Density Smoothing)
    solvers   Jacobi-preconditioned CG with true-residual restarts, the
              same CG with residual replacement (the continuation rule of the
              GPU's mixed-precision solve, in FP64), flexible CG with the
              stagnation fallback, the FP64 true residual.  There is no FP32
              solver here: a mixed-precision GPU result is checked against this
              module's FP64 true residual of its solution
    unet      the learned preconditioner: 3-D convolutions, pooling,
              upsampling, forward/backward, step loss and Adam, in FP64 on
              BF16-rounded storage points
    rk2       the two-stage Runge-Kutta cycle around the projection
              (Numerical Time Integration)
    boundary  inhomogeneous Neumann data: per-cell body flux, exit-face
              update (Radiation Conditions)
    vof       split VOF advection (Interface reconstruction and advection)
    gridgen   the stretched axis of eq. grid (Gridding)
    panels    signed distance from triangular panels (Enforcement of Body
              Boundary Conditions)
    multigrid aggregation multigrid V-cycle (a preconditioner the paper does
              not name)

Each function names the passage of the paper it follows.  Where the paper
is silent the docstring states the reading taken.
"""
