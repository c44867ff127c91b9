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
    """Rounding sensitivity of the oracle's k-step PCG iterate at FP32 level.

    Runs the oracle's PCG (FP64 arithmetic) with FP32 rounding inserted where
    an FP32 implementation stores values: (i) the CG vectors, (ii) the CG
    vectors and the layer pixel fields, (iii) the right side, the
    preconditioner, the layer fields and the adjoint node fields, (iv) all of
    these plus each sensor's adjoint contribution to each layer.  Returns the
    largest deviation (e_x, per-layer e_phi, e_res) from the plain FP64
    iterate: the band within which an FP32-storage implementation of the same
    algorithm lands on this frame."""
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    ident = lambda a: a
    x_ref, _ = O.pcg(S.apply_A, b, k, x0=x0, jacobi=J)
    Jd = np.ones(S.n) if J is None else J

    def apply_rounded(c, rphi, rv, rimg):
        phi = S.to_layers(c)
        if rphi:
            phi = [f32(p) for p in phi]
        w = S.weight(S.forward_layers(phi))
        acc = [np.zeros((N, N)) for N in S.N]
        for m, sen in enumerate(S.sensors):
            v = S._measure_adjoint(sen, S.slopes_of(w, m))
            if rv:
                v = f32(v)
            for l, g in enumerate(S._project_adjoint(sen, v)):
                acc[l] += f32(g) if rimg else g
        return S.to_coeffs(acc) + S.alpha * S.D * c

    out = [0.0, 0.0, 0.0]
    for rvec, rb, rphi, rv, rimg in ((True, False, False, False, False),
                                     (True, False, True, False, False),
                                     (False, True, True, True, False),
                                     (True, True, True, True, True)):
        R = f32 if rvec else ident
        bb = f32(b) if rb else b
        JJ = f32(Jd) if rb else Jd
        x = np.zeros_like(b) if x0 is None else R(x0)
        r = R(bb - apply_rounded(x, rphi, rv, rimg)) if x0 is not None else R(bb)
        z = r / JJ
        p = R(z)
        rho = r @ z
        for _ in range(k):
            q = R(apply_rounded(p, rphi, rv, rimg))
            a = rho / (p @ q)
            x = R(x + a * p)
            r = R(r - a * q)
            z = r / JJ
            rn = r @ z
            p = R(z + (rn / rho) * p)
            rho = rn
        e_x = rel(x, x_ref)
        e_phi = max(rel(u, v) for u, v in zip(S.to_layers(x), S.to_layers(x_ref)))
        e_res = float(np.linalg.norm(S.apply_A(x) - S.apply_A(x_ref)) / np.linalg.norm(b))
        out = [max(out[0], e_x), max(out[1], e_phi), max(out[2], e_res)]
    return tuple(out)


def fp32_tol(S, b, k, J=None, x0=None, base=1e-5):
    """FP32 tolerance per error measure: the 1e-5 bar, or twice the frame's
    FP32 rounding spread where the frame is too ill-conditioned for it."""
    return tuple(max(base, 2.0 * s) for s in fp32_spread(S, b, k, J, x0))
