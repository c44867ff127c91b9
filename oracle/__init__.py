"""ORACLE: plain, slow FP64 CPU implementation of the wavelet-MCAO tomography
solve, written from the paper (Helin & Yudytskiy, "Wavelet methods in
multi-conjugate adaptive optics").

This is TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code, tables or
constants with the GPU library, and the GPU library never calls it.
"""
from .wavelet import (db3_lowpass, haar_lowpass, highpass, analysis_1d, synthesis_1d, fdwt2,
                      idwt2, fdwt1_multilevel, idwt1_multilevel, coefficient_level)
from .geometry import FootprintError
from .system import System
from .pcg import pcg, STATUS_OK, STATUS_CONVERGED, STATUS_BREAKDOWN
from .control import fit, Polc
