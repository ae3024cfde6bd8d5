"""FP64 CPU oracle for the lock-exchange lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it. It shares no code, tables or constants
with the HIP library; it is written directly from the paper (Adekanye et al.,
"GPU accelerated lattice Boltzmann method simulations of dilute gravity
currents", arXiv 2112.08479) in plain PyTorch CPU float64, so that autograd
through it gives the reference adjoint.

Modules
  lattice   velocity sets and weights (Eq. 23-24, 31, 36)
  params    lattice-unit parameters (Sec. 2.5, Eq. 25, 30)
  ring      truncated moment-generating-function ring: cumulants (Eq. 54)
  collide   BGK + Guo (Eq. 21-26), Smagorinsky (Eq. 32-35), cumulant
            (Eq. 54-58) with given or parametrised higher-order rates
            (Sec. 2.3), scalar BGK (Eq. 28-30), factorized central moments
            (Eq. 37-51)
  lbm       gather with half-way bounce-back / periodic span, initial state,
            one time step (Eq. 17), moments (Eq. 18-20, 27)
  diag      mass, scalar mass, bottom-wall friction (Eq. 62, 64) and front
            position (Sec. 3.1)
  adjoint   objective J = x_f(end) + mean F_w and its autograd gradient

Parity status of each function is stated in its docstring; everything here is
pinned by the CPU tests except where a docstring says "parity unpinned".
"""
