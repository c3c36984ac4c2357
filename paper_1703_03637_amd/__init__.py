"""MI355X-native matrix-free H.v / Lanczos / TPQ for spin-1/2 and fermion lattices.

The computation lives in libhphi.so (HIP, gfx950) behind the C ABI of
include/hphi.h; `binding` exposes the same entry points to Python with
torch tensors as device memory.  There is no CPU fallback.
"""

from .binding import (  # noqa: F401
    Basis,
    Ham,
    DTYPE_NAMES,
    hphi_basis_build,
    hphi_basis_rank,
    hphi_basis_unrank,
    hphi_cg_refine,
    hphi_expect,
    hphi_ham_build,
    hphi_ham_nonfinite,
    hphi_hv,
    hphi_hv_elements,
    hphi_hv_tune,
    hphi_hv_cma,
    hphi_hv_cma_plan,
    hphi_lanczos,
    hphi_tpq_step,
    hphi_tpq_run,
    hphi_tpq_run_noalloc,
    version,
)
from ._lib import HphiError, LIB_PATH  # noqa: F401
