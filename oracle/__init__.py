"""Plain FP64 CPU oracle of the two-level Nystrom-Schur preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.

The oracle follows Al Daas, Rees & Scott, "Two-level Nystrom-Schur
Preconditioner for Sparse Symmetric Positive Definite Matrices" (arXiv
2101.12164): the doubly bordered block diagonal split (eq. perm_A), the block
LDL^T factorisation (eq. A_LDLT), the Schur complement (eq. schur_complement),
the Sherman-Morrison-Woodbury form (eq. S-1), Nystrom's method (Algorithm
alg:nystrom), the construction of M_2 (Algorithm alg:prec1, eq. left_prec_mat)
and PCG on S_Gamma w = f (eq. Sx=b), and the recursive construction the
conclusions name as future work (A_Gamma preconditioned one level down).
"""

from .nystrom_schur_oracle import (  # noqa: F401
    DBBD,
    Operators,
    orth,
    bf_bpcg,
    nystrom_core,
    NystromSchurOracle,
    GammaFactor,
    level2_order,
    level2_part,
    RecursiveGamma,
    pcg,
    dense_schur,
    ideal_s2,
    full_system_pcg,
)
from . import learned  # noqa: F401
