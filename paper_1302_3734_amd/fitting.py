"""Fitting step and pseudo-open-loop control on top of the solver plans.

Fitting (Sec. 4.1, eq. (15)): the mirror commands a minimise
|H a - P phi| over a set of field directions, H the piecewise-bilinear mirrors
seen along each direction and P the natural-guide-star projection of the
reconstructed layers.  Both maps are plans of this library with "phase"
sensors (one per direction, the pupil nodes as measurement points): P phi is
``forward_layers`` of the atmosphere plan, and the normal equations
(H^T H + alpha I) a = H^T P phi are solved by the same PCG kernels on the
mirror plan (its "layers" are the actuator grids, with no wavelet transform).

Pseudo-open-loop control (Sec. 4.2, Alg. 4.1), with a two-frame delay:
    s_ol = s + A^ a_{t-2};   da = R s_ol - a_{t-2};   a_t = a_{t-1} + g da,
where R is tomography (warm-started PCG, Sec. 5.1) followed by W^-1 and the
fitting step, and A^ maps mirror commands to sensor slopes (a plan whose
layers are the mirror grids, seen by the tomography's own sensors).  Every
vector operation is a library kernel (``wmcao_axpby``).
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

    def step(self, s):
        """One control step from the residual slopes s measured for the
        commands a_{t-2}; returns the new commands a_t."""
        a2, a1 = self.a_hist
        axpby(1.0, s, 1.0, self.mirror_slopes(a2), self.s_ol)               # s_ol = s + A^ a_{t-2}
        self.tomo.solve(self.s_ol, self.c, n_iter=self.n_iter, warm_start=self.steps > 0)
        layers = self.tomo.coeffs_to_layers(self.c)
        self.fitter.fit(layers, self.a_fit, warm_start=self.steps > 0)      # R s_ol
        a_new = torch.empty_like(a1)
        axpby(1.0, self.a_fit, -1.0, a2, a_new)                            # da = R s_ol - a_{t-2}
        axpby(1.0, a1, self.gain, a_new, a_new)                            # a_t = a_{t-1} + g da
        self.a_hist = [a1, a_new]
        self.steps += 1
        return a_new

    def close(self):
        self.tomo.close()
        self.ahat.close()
        self.fitter.close()
