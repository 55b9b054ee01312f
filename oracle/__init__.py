"""Plain FP64 CPU oracle for the randomized preconditioned SC-4DVAR hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library (no
kernels, headers, tables, constant generators or pre/post-processing); the two
meet only through the seeded raw draws produced by
``paper_2401_15758_amd.inputs``, which hold none of the method's arithmetic.

Every function cites the passage of arXiv:2401.15758 (Subrahmanya, Rao,
Saibaba, "Randomized Preconditioned Solvers for Strong Constraint 4D-Var Data
Assimilation") that it follows.  Everything is numpy float64; the only library
primitives used as steps are matmul, Cholesky, triangular solve, QR, SVD,
symmetric eigensolve and the FFT.

Modules
-------
burgers   periodic viscous Burgers, RK4 nonlinear model, its discrete RK
          tangent-linear and adjoint (Sec. 2.1 eq. (model), Sec. 2.2, Sec. 5.1)
bve       periodic barotropic vorticity, Arakawa Jacobian, spectral Poisson
prior     Gaussian-kernel background covariance and its symmetric square root
problem   the SC-4DVAR problem: observations, cost, gradient, the
          prior-preconditioned operator A, A^T and the Hessian (eqs. (4dvar_cf),
          (4dvar_gradient), (4dvar_hessian), (Rhalf))
sketch    RandSVD (Alg. 1), Nystrom (Alg. 2), Woodbury LMP (eq. (woodbury)),
          the W-form Woodbury of Remark 1 (eq. (randsvdsv))
pcg       preconditioned CG on (I + H) dx = b (Sec. 2.2.2, eq. (pcgsystem))
gn        one Gauss-Newton step and the reuse test kappa_re (eq. (condtext2))
analysis  intrinsic dimension, Psi_H bound, condition numbers (Sec. 4)
rng       the library's counter-based Gaussian stream (Philox4x32-10 +
          Box-Muller), written from its published definition, so that the
          oracle can reproduce draws the library makes on the device

Parity unpinned: none of the functions above is unpinned; see tests/test_oracle_*.
"""
