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
    operator  density, face coefficients, the cut-cell flux-form operator,
              right-hand side, projection and divergence (eqs. density,
              pois, poisson1, integral2, runge1, diverge; Density Smoothing)
    solvers   Jacobi-preconditioned CG, flexible CG, mixed-precision
              refinement, stagnation fallback
    unet      the learned preconditioner: 3-D convolutions, pooling,
              upsampling, forward/backward and Adam, in FP64

Each function names the passage of the paper it follows.  Where the paper
is silent the docstring states the reading taken.
"""
