"""CPU oracle of the truncated-SVD method (FP64, NumPy/SciPy).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP implementation; both are fed the same seeded inputs.
"""
from .svds_ref import svds, lbp, cgs2, small_svd, explicit_residuals, sign_normalize, as_operator, SvdsInfo
from .jacobi import jacobi_svd
from .philox import philox4x32_10, normal_vector
