"""Shared set-up of the GPU parity tests: a configuration, its noise levels,
the oracle system and a GPU plan built from the same inputs."""
import numpy as np
import pytest

import oracle as O
import workloads as WL


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1302_3734_amd import _abi
    _abi.lib()                     # raises if the HIP library is not built


def say(msg):
    print(msg, flush=True)


def setup(cfg, frame=0, seed_frame=None):
    """Oracle system with sigma from the clean slopes of ``frame`` (frozen
    flow from ``seed_frame`` if given), and that frame's noisy slopes."""
    S0 = O.System(cfg, [1.0] * len(cfg["wfs"]))
    truth = WL.layer_screens(cfg, frame, seed_frame=seed_frame)
    clean = S0.forward_layers(truth)
    sig = WL.sigmas_from_clean(cfg, clean, S0.slope_off)
    S = O.System(cfg, sig)
    s = WL.noisy_slopes(clean, sig, S.slope_off, WL.noise_draw(cfg["cfg_id"], frame, S.n_slopes))
    return S, sig, s, truth


def slopes_for(S, cfg, sig, frame, seed_frame=None):
    truth = WL.layer_screens(cfg, frame, seed_frame=seed_frame)
    clean = S.forward_layers(truth)
    return WL.noisy_slopes(clean, sig, S.slope_off, WL.noise_draw(cfg["cfg_id"], frame, S.n_slopes))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    """Largest element difference over the largest reference element."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def to_dev(x, dtype):
    import torch
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda").contiguous()


def to_np(t):
    return t.detach().double().cpu().numpy()
