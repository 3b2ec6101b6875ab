"""CPU FP64 oracle for the in-situ multipole 3PCF estimator (test infrastructure).

This package is the slow, plain reference that the GPU library is checked
against.  It is test infrastructure: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
It shares no code with the GPU library (``paper_2507_15209_amd``) and never
imports it; both are fed the same seeded inputs from ``mockgen``.

Every function follows the paper passage it cites (Ju, Feng, Huang, Sun &
Zhu, "An Optimal In-Situ Multipole Algorithm for the Isotropic Three-Point
Correlation Function"): Sec. 2.1 (translation windows, plane-wave expansion,
multiresolution reconstruction), Sec. 2.2 (connection coefficients, multipole
window, grid and particle summation) and Appendix A (rotation average of two
plane waves).  Arithmetic is float64 throughout; numpy/scipy FFTs, matrix
products and special functions serve as single steps, with no blocking,
fusion or reordering beyond what the definitions state.

Modules
  special    spherical Bessel functions, bin-averaged j_l, Y_lm, Legendre P_l
  basis      cubic B-spline basis, deposit / gather, connection coefficients
  basis_d4   Daubechies-4 scaling function (cascade table, deposit / gather,
             autocorrelation, |phi_hat|^2 by the infinite product, connection
             coefficients from the two-scale relation)
  estimator  multipole kernel, a_lm fields, zeta_l by nodal, grid-Gamma and
             particle summation
  adjoint    gradients of sum_l lambda_l . zeta_l w.r.t. the density grid and
             the particle weights

Parity status: every function is pinned by the CPU tests (``-m "not gpu"``)
against closed forms, brute force or finite differences; none is "parity
unpinned".
"""
from . import special, basis, basis_d4, estimator, adjoint  # noqa: F401
from .estimator import Plan  # noqa: F401
