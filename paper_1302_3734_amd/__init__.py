"""MI355X-native wavelet-domain MCAO tomography solver (HIP kernels behind a C ABI).

The solve of the wavelet-domain MAP normal equations of Helin & Yudytskiy,
"Wavelet methods in multi-conjugate adaptive optics" (Sec. 5.1, eq. (19)),
by PCG with the modified Jacobi preconditioner and warm restart.  Every step
runs in libwmcao.so; importing a Plan without the built library raises.
"""
from ._abi import WmcaoError, WMCAO_FRAME_OK, WMCAO_FRAME_CONVERGED, WMCAO_FRAME_BREAKDOWN
from .plan import Plan, solve_multi

__all__ = ["Plan", "solve_multi", "WmcaoError", "WMCAO_FRAME_OK", "WMCAO_FRAME_CONVERGED",
           "WMCAO_FRAME_BREAKDOWN"]
