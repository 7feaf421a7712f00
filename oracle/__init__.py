"""Oracle: plain, slow, obviously-correct CPU reference of the method.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(the HIP path) never imports it, and it never imports the product library.

Contents
  lbm    -- ctypes wrapper over lbm_oracle.c: the FP64 lattice Boltzmann step
            (Eqs. 1-3, 8-11, 23, 31 of the paper), moments and mass.
  thermo -- equations of state, critical points, the Maxwell construction
            (Eq. 7) by two independent methods, and the mechanical stability
            condition (Eq. 26, any epsilon; Eq. 30 for epsilon = 2).
  mlp    -- FP64 forward/backward/Adam reference of the sigma surrogate, with
            optional bfloat16 rounding of the matmul operands.
"""
