"""CPU FP64 oracle for QDWHpartial-EIG and QDWHpartial-SVD.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, step-by-step NumPy /
SciPy implementation of the paper's method (Algorithms 1 and 2 of Sec. 4) used
to check the HIP implementation.  Only the test-suite, the smoke entry point
and the CPU-baseline leg of the benchmark may import it; the product path
(the HIP library and its Python binding) never does, and the two share no code
(no kernels, helpers, tables or constant generators).  Seeded inputs come from
the separate ``synthetic`` package, which holds none of the method's arithmetic.

Every function cites the passage of the paper it follows.  Where the paper is
silent or ambiguous the reading taken is stated in the function's docstring.

Parity status of each function is recorded in ``PINS`` below; a function with
no independent pin says "parity unpinned".
"""
from .dwh import dwh_weights, dwh_map, compose, iteration_count, eig_schedule, svd_schedule  # noqa: F401
from .philox import philox4x32_10, gaussian  # noqa: F401
from .polar import qr_step, chol_step, halley_direct_step  # noqa: F401
from .estimator import lanczos_slq, choose_tau, choose_svd_threshold  # noqa: F401
from .partial import eig_partial, svd_partial  # noqa: F401
from .jacobi import jacobi_eig, jacobi_svd  # noqa: F401
from .metrics import eig_metrics, svd_metrics  # noqa: F401
from .zolo import zolo_coeffs, zolo_map, zolo_schedule, zolo_step  # noqa: F401
from .hermitian import heig_partial, heig_metrics, qr_step_h, chol_step_h  # noqa: F401

# What pins each oracle function (see tests/test_oracle_*.py).
PINS = {
    "dwh_weights": "Zolotarev optimality: max of r on [l,1] is 1, min is r(l); "
                   "(3,1,3) at l=1; perturbing a worsens the sup error",
    "iteration_count": "paper: <= 6 iterations for kappa <= 1e15; s=0.2 -> 3, s=0.875 -> 2 (by the O(u) band)",
    "philox4x32_10": "published known-answer vectors of Philox4x32-10",
    "qr_step/chol_step": "three independent formulations (Eq. 1 with an explicit inverse, Eq. 2, Eq. 3) agree; "
                         "planted iterates equal U r(Sigma) V^T of the scalar composite",
    "lanczos_slq": "Ritz values interlace the planted spectrum; count estimate brackets planted counts",
    "eig_partial": "planted eigenvalues to 1e-12; residual and orthogonality; brute-force Jacobi n<=64",
    "svd_partial": "planted singular values to 1e-12; residuals; brute-force one-sided Jacobi n<=64; "
                   "paper's threshold/fraction mapping for D[i] = 0.5^(100 i/N)",
    "jacobi_eig/jacobi_svd": "closed-form 2x2 and diagonal cases, orthogonality, reconstruction",
    "zolo_coeffs/zolo_map": "r = 1 equals the DWH closed form; composition (DWH twice = type (9,8), three "
                            "times = type (27,26)); equioscillation (r+1 maxima 1, r+1 minima Z(l)); "
                            "partial fractions reproduce the product",
    "zolo_step": "planted iterates equal U Z(Sigma) V^T; Cholesky and QR terms agree; r = 1 equals the "
                 "DWH step",
    "heig_partial": "real input gives the real eig_partial's result; planted complex spectra to 1e-12; "
                    "LAPACK zheevd on small n; complex steps on planted iterates equal U r(Sigma) V^H",
}
