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


def fp32_spread(S, b, k, J=None, x0=None):
    """Rounding sensitivity of the oracle's k-step PCG iterate to what the FP32
    precision mode stores in single precision by definition: the CG vectors
    (x, r, p and A p), the right side b and the preconditioner diagonal J.

    The oracle's PCG (FP64 arithmetic, FP64 operator) is rerun with those
    values rounded to FP32 where they are stored, and nothing else.  Returns
    its deviation (e_x, per-layer e_phi, e_res) from the plain FP64 iterate:
    how far any implementation of the same algorithm that keeps these vectors
    in FP32 moves from the FP64 iterate on this frame, however exact its
    operator.  It does not depend on how the implementation under test stores
    its operator's intermediates."""
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    x_ref, _ = O.pcg(S.apply_A, b, k, x0=x0, jacobi=J)
    Jd = f32(np.ones(S.n) if J is None else J)
    bb = f32(b)
    x = np.zeros_like(b) if x0 is None else f32(x0)
    r = f32(bb - S.apply_A(x)) if x0 is not None else bb
    z = r / Jd
    p = f32(z)
    rho = r @ z
    for _ in range(k):
        q = f32(S.apply_A(p))
        a = rho / (p @ q)
        x = f32(x + a * p)
        r = f32(r - a * q)
        z = r / Jd
        rn = r @ z
        p = f32(z + (rn / rho) * p)
        rho = rn
    e_x = rel(x, x_ref)
    e_phi = max(rel(u, v) for u, v in zip(S.to_layers(x), S.to_layers(x_ref)))
    e_res = float(np.linalg.norm(S.apply_A(x) - S.apply_A(x_ref)) / np.linalg.norm(b))
    return e_x, e_phi, e_res


def fp32_tol(S, b, k, J=None, x0=None, base=1e-5):
    """FP32 bar per error measure: 1e-5, or twice the frame's spread under
    FP32 storage of the CG vectors, b and J (fp32_spread) where that spread
    alone exceeds half of 1e-5 (the 8 m natural-guide-star systems at 10
    iterations from zero)."""
    return tuple(max(base, 2.0 * s) for s in fp32_spread(S, b, k, J, x0))


def solve_errors(S, x, x_ref, b):
    """(e_x, e_phi, e_res) of an iterate x against the oracle's x_ref: relative
    coefficient error, largest per-layer reconstruction error, and the
    difference of the residuals relative to |b|."""
    e_x = rel(x, x_ref)
    e_phi = max(rel(a, r) for a, r in zip(S.to_layers(x), S.to_layers(x_ref)))
    e_res = float(np.linalg.norm(S.apply_A(x) - S.apply_A(x_ref)) / np.linalg.norm(b))
    return e_x, e_phi, e_res


# worst errors seen per configuration, printed at the end of the session
WORST = {}


def record(config, dtype, errors, bars):
    """Keep the largest error of each measure and its ratio to the bar."""
    key = (config, dtype)
    cur = WORST.get(key)
    ratio = max(e / b for e, b in zip(errors, bars))
    if cur is None:
        WORST[key] = [list(errors), ratio, 1]
    else:
        cur[0] = [max(a, e) for a, e in zip(cur[0], errors)]
        cur[1] = max(cur[1], ratio)
        cur[2] += 1


def oracle_pool_map(fn, args, workers=16):
    """Map fn over args in fresh CPU worker processes (spawned, so that they
    never touch the GPU), for oracle references of many frames."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(workers, max(1, len(args)))) as pool:
        return pool.map(fn, args)
