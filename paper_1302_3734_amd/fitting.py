"""Fitting step and pseudo-open-loop control on top of the solver plans.

Fitting (Sec. 4.1, eq. (15)): the mirror commands a minimise
|H a - P phi| over a set of field directions, H the piecewise-bilinear mirrors
seen along each direction and P the natural-guide-star projection of the
reconstructed layers.  Both maps are plans of this library with "phase"
sensors (one per direction, the pupil nodes as measurement points): P phi is
``forward_layers`` of the atmosphere plan, and the normal equations
(H^T H + alpha I) a = H^T P phi are solved by the same PCG kernels on the
mirror plan (its "layers" are the actuator grids, with no wavelet transform).

Pseudo-open-loop control (Sec. 4.2, Alg. 4.1) with a delay of two frames:
the residual slopes measured through the commands applied two frames ago are
turned back into open-loop slopes by adding what those commands contribute
(A^ maps commands to slopes: a plan whose layers are the mirror grids, seen by
the tomography's own sensors); R (tomography by warm-started PCG, Sec. 5.1,
then W^-1 and the fitting step) reconstructs commands from them, and an
integrator with gain g moves the latest commands a fraction g towards that
reconstruction, measured against the commands the slopes were taken with.
Every vector operation is a library kernel (``wmcao_axpby``).
"""
import ctypes as C

import torch

from . import _abi
from .plan import Plan, _ptr, _stream_ptr


def axpby(a, x, b, y, out):
    """out = a x + b y on the device (library kernel)."""
    dt = _abi.WMCAO_F32 if x.dtype == torch.float32 else _abi.WMCAO_F64
    assert x.dtype == y.dtype == out.dtype and x.numel() == y.numel() == out.numel()
    _abi.check(_abi.lib().wmcao_axpby(dt, C.c_int64(x.numel()), float(a), _ptr(x), float(b),
                                      _ptr(y), _ptr(out), _stream_ptr()), "wmcao_axpby")
    return out


class Fitter:
    """Layers -> mirror commands by CG on the fitting normal equations."""

    def __init__(self, atm_cfg, dm_cfg, dtype="f64", max_batch=1):
        ones = [1.0] * len(atm_cfg["wfs"])
        self.atm = Plan(atm_cfg, ones, dtype=dtype, max_batch=max_batch)
        self.dm = Plan(dm_cfg, ones, dtype=dtype, max_batch=max_batch)
        self.n_iter = int(dm_cfg.get("n_iter", 4))
        self.n_act = self.dm.n

    def fit(self, layers, a, n_iter=None, warm_start=True):
        """layers: [batch, n_layers_pixels] of the atmosphere plan; a: [batch,
        n_act] mirror commands (warm start in, result out)."""
        target = self.atm.forward_layers(layers)
        self.dm.solve(target, a, n_iter=self.n_iter if n_iter is None else n_iter,
                      warm_start=warm_start)
        return a

    def directions_phase(self, layers, a):
        """(P phi, H a) at the pupil nodes of every fitting direction."""
        return self.atm.forward_layers(layers), self.dm.forward_layers(a)

    def close(self):
        self.atm.close()
        self.dm.close()


class PolcController:
    """Pseudo-open-loop control with a two-step delay (Alg. 4.1)."""

    def __init__(self, tomo_cfg, sigmas, dm_wfs_cfg, fit_atm_cfg, fit_dm_cfg, dtype="f64",
                 gain=0.4, n_iter=10, cinv_blocks=None):
        self.tomo = Plan(tomo_cfg, sigmas, dtype=dtype, max_batch=1, cinv_blocks=cinv_blocks)
        self.ahat = Plan(dm_wfs_cfg, sigmas, dtype=dtype, max_batch=1)
        self.fitter = Fitter(fit_atm_cfg, fit_dm_cfg, dtype=dtype)
        self.gain = float(gain)
        self.n_iter = int(n_iter)
        tdt = self.tomo.torch_dtype
        na = self.fitter.n_act
        self.c = torch.zeros(1, self.tomo.n, dtype=tdt, device="cuda")      # tomography warm start
        self.a_hist = [torch.zeros(1, na, dtype=tdt, device="cuda") for _ in range(2)]  # a_{t-2}, a_{t-1}
        self.a_fit = torch.zeros(1, na, dtype=tdt, device="cuda")          # fitting warm start
        self.s_ol = torch.zeros(1, self.tomo.n_slopes, dtype=tdt, device="cuda")
        self.steps = 0

    def mirror_slopes(self, a):
        return self.ahat.forward_layers(a)

    def _open_loop(self, s, a_meas):
        """Slopes the atmosphere alone would give: s plus the contribution of
        the commands a_meas that were applied when s was measured."""
        axpby(1.0, s, 1.0, self.mirror_slopes(a_meas), self.s_ol)
        return self.s_ol

    def _reconstruct(self, s_ol):
        """R: tomography (warm-started after the first step), W^-1, fitting."""
        warm = self.steps > 0
        self.tomo.solve(s_ol, self.c, n_iter=self.n_iter, warm_start=warm)
        self.fitter.fit(self.tomo.coeffs_to_layers(self.c), self.a_fit, warm_start=warm)
        return self.a_fit

    def step(self, s):
        """One control step from the residual slopes s measured for the
        commands a_{t-2}; returns the new commands a_t."""
        a_meas, a_last = self.a_hist
        target = self._reconstruct(self._open_loop(s, a_meas))
        # integrator: a_last + g (target - a_meas), as (a_last - g a_meas) + g target
        a_new = torch.empty_like(a_last)
        axpby(1.0, a_last, -self.gain, a_meas, a_new)
        axpby(1.0, a_new, self.gain, target, a_new)
        self.a_hist = [a_last, a_new]
        self.steps += 1
        return a_new

    def close(self):
        self.tomo.close()
        self.ahat.close()
        self.fitter.close()
