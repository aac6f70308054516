"""Plain CPU oracle for exp(tA)V by the rational approximation R_d(z) = 1/exp_d(-z).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, helpers, constants or pre/post-processing).

Layout
------
``oracle.scalar``  the scalar objects of the paper (Sec. 2 and Sec. 4):
                   truncated Taylor polynomial exp_d, its roots theta_k, the
                   residues a_k of Proposition pro:dec (eq. yoyo2, and the
                   alternatives of eq. yoyo234), R_d evaluated directly, the
                   bounds M_1 (Prop. pro:err) and M_2 (Prop. prop:digit).
``oracle.matrix``  the matrix function the library approximates (Sec. 3):
                   R_d(tA)V and exp(tA)V by Hermitian eigendecomposition, plus
                   independent routes used only to pin the oracle (exact
                   partial-fraction sum and product form at 50 digits, matrix
                   polynomial evaluation followed by a linear solve).

Every function is plain, slow and written for reading against the paper:
FP64 unless the function says it works at extended precision (mpmath).
"""

from . import scalar, matrix  # noqa: F401
