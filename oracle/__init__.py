"""Plain, slow, obviously-correct FP64 CPU oracle for the refined-wall solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the C-ABI library and its
Python binding) may import, call, link or execute anything in this package;
only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg use it.  It shares no code with the GPU path: it discretizes with NumPy's
own Gauss-Legendre rule, assembles dense matrices with NumPy and solves with
LAPACK through ``numpy.linalg``.

What it computes (Zhang, Gillman & Veerapaneni, arXiv:2108.07205):

* the interior Stokes Dirichlet problem (Sec. 2.1, eq. model_bvp) with the
  double-layer representation, Nystrom-discretized as
  ``A = -1/2 I + D + N`` (eqs. interior_BIE_discretized2 and null);
* the locally refined discretization and its index sets I_k, I_c, I_p
  (Sec. 3.1, eqs. originalLinearSystem / perturbedlLinearSystem);
* the refined solution ``tau_n = A_nn^{-1} g_n`` by dense LU -- the plain
  definition the fast method approximates;
* for tests of the method's algebra: the extended linear system (Sec. 3.2,
  eq. extendedlLinearSystem), the Woodbury formula (eq. wood), the
  interpolative decomposition (Definition 3.1), the block truncated-SVD
  factorizations (eq. uniform_concat) and the Woodbury-operator condition
  bound (Lemma thm:woodbury).

Modules: ``geometry`` (curve, panels, refinement), ``kernels`` (Stokeslet,
double layer, dense Nystrom assembly, velocity evaluation), ``solve`` (dense
solve, ELS, Woodbury, ID, SVD factors, lemma bound).
"""
from . import geometry, kernels, solve  # noqa: F401
