"""FP64 CPU oracle for the inverse-free split step -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct NumPy/SciPy implementation of
what the library computes, written from the paper (Ballard, Demmel, Dumitriu,
"Minimizing Communication for Eigenproblems and the Singular Value
Decomposition", arXiv 1011.3077):

* Alg. 1 (RURV), its QL twin RULV, and Alg. 2 (GRURV) for k = 2   -> rurv.py
* Alg. 3 (IRS, implicit repeated squaring)                        -> irs.py
* Alg. 4 (RGNEP) / Alg. 6 (RSEP) one split step, with the line-to-circle
  Moebius map of Sec. 3.3 and the split-point search of Alg. 4 line 5 -> split.py
* the randomized divide-and-conquer strategy of Sec. 3.3-3.5       -> eig_dc.py
* eigenvectors of an upper-triangular matrix or pencil (TREVC, Sec. 5) -> trevc.py
* the Philox4x32-10 counter-based generator (Salmon et al., SC'11) with a
  Box-Muller transform, for the Gaussian matrix RURV draws          -> philox.py

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library and
never imports it; the library never imports this package.

Every factorization uses LAPACK through SciPy (a library primitive) or the
pure-loop Householder in qr.py; nothing is blocked, fused or reordered
beyond what the paper's algorithms state.
"""
from .qr import (householder_qr_loop, qr_signed, rq_signed, ql_signed)  # noqa: F401
from .irs import irs, IRSResult  # noqa: F401
from .rurv import haar_from_gaussian, rurv, rulv, grurv2  # noqa: F401
from .split import (premap, split_search, split_sym, split_pencil, split_svd, split_nonsym,
                    SplitResult,  # noqa: F401
                    rank_from_rho, norm1, OK, NOT_CONVERGED, NO_SPLIT, RANK_AMBIGUOUS)
from .philox import philox4x32_10, gaussian_matrix  # noqa: F401
from .eig_dc import eig_dc, block_eigvals  # noqa: F401
from .trevc import trevc  # noqa: F401
