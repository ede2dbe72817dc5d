"""FP64 CPU oracle for the FTK rigid-alignment hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under this package: only the tests, the package smoke check
and the benchmark's CPU-baseline leg use it.  It shares no code with the GPU
library (its Bessel functions, quadrature and SVD come from SciPy/NumPy, the
GPU planner has its own C++ implementations).

Modules:
  ftk      -- quadrature, operator SVD, transform, direct and FTK inner
              products, best poses, error scales (Sections 2-5 of the paper)
  mlp      -- FP64 forward/backward of the template-proposal MLP
"""
