"""MI355X (gfx950) solver for N-dimensional Sylvester tensor equations
sum_k A_k x_k X = B by the Schur / Bartels-Stewart method of Cuesta & de la
Hoz (arXiv 2412.15840).  The compute path is libsylt.so (hand-written HIP);
``sylt`` is its thin Python binding.  Importing this package does not load
the library; the first call does, and fails loudly if it has not been built.
"""
from . import sylt  # noqa: F401
from .sylt import Plan, SchurSolve, sylvester_solve  # noqa: F401
