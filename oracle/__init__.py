"""Oracle: a plain, slow, FP64 CPU implementation of the rational time stepper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (different language, independently derived formulas); the only
thing both sides share are the seeded inputs from ``workloads``.

What it computes (Haut, Babb, Martinsson, Wingate, arXiv:1402.5168):

* ``cheb``         Chebyshev-Lobatto nodes and spectral differentiation
                   (section 2.2).
* ``collocation``  the multidomain collocation system B u = f of section 2.2
                   assembled as one global sparse matrix and solved with a
                   sparse LU, i.e. the plain definition of the resolvent
                   solves that the hierarchical solver of section 2.3
                   reproduces exactly up to rounding; and the time step
                   sum_m b_m (tau L - alpha_m)^{-1} u (section 1.2).
* ``rational``     evaluation of R(ix) = sum_m b_m / (ix - alpha_m)
                   (eq. def_RM), the fit checks of eqs. RM_prop1/RM_prop2,
                   and the paper's Table 1 and Gaussian-sum formulas
                   (section 3).
* ``dense``        tiny grids only: the interior-node operator L_h as a dense
                   matrix, and V R(tau Lambda) V^{-1} u by eigendecomposition.

Parity status of each function is listed in its module docstring.
"""
