"""Oracle work for the GPU parity tests, run in spawned CPU worker processes.

Each job rebuilds (and caches per process) the FP64 oracle system of a named
configuration with the given noise levels, so that the references of many
frames can be computed in parallel on the host while the GPU results wait.
Nothing here touches the GPU.
"""
import numpy as np

import oracle as O
import workloads as WL
from tests.gpu_common import fp32_tol, solve_errors

_SYS = {}


def system(name, sig):
    key = (name, tuple(float(v) for v in sig))
    if key not in _SYS:
        cfg = WL.config_by_name(name)
        S = O.System(cfg, list(sig))
        precond = cfg.get("precond", True)
        _SYS.clear()
        _SYS[key] = (cfg, S, S.jacobi_separable() if precond else None)
    return _SYS[key]


def slopes(job):
    """Noisy slopes of one frame: (name, sig, frame, seed_frame)."""
    name, sig, frame, seed_frame = job
    cfg, S, _ = system(name, sig)
    truth = WL.layer_screens(cfg, frame, seed_frame=seed_frame)
    clean = S.forward_layers(truth)
    return WL.noisy_slopes(clean, sig, S.slope_off, WL.noise_draw(cfg["cfg_id"], frame, S.n_slopes))


def check(job):
    """Errors of a GPU iterate against the oracle's PCG iterate of the same
    inputs, and the bar each must meet.

    job: (name, sig, slopes as the GPU saw them, warm start as the GPU saw it
    or None, GPU iterate, iterations, "f64", "f32" or "f32-fixed").  Returns
    (errors, bars)."""
    name, sig, s_in, x0, x_gpu, k, dt = job
    cfg, S, J = system(name, sig)
    b = S.rhs(np.asarray(s_in, dtype=np.float64))
    x_ref, _ = O.pcg(S.apply_A, b, k, x0=x0, jacobi=J)
    e = solve_errors(S, np.asarray(x_gpu, dtype=np.float64), x_ref, b)
    if dt == "f64":
        bars = (1e-11,) * 3
    elif dt == "f32-fixed":      # the fixed FP32 bar, with no spread computed
        bars = (1e-5,) * 3
    else:
        bars = fp32_tol(S, b, k, J, x0)
    return e, bars
