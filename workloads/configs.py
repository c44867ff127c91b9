"""Telescope, guide-star and atmosphere configurations.

The shapes follow the paper's E-ELT MCAO set-up (Sec. 5.1): 42 m pupil with
about 28 % obstructed, six sodium laser guide stars on a ring of 2 arcmin
diameter with 84x84 Shack-Hartmann sensors, three tip/tilt natural guide stars
on a ring of 8/3 arcmin diameter (2x2, 1x1, 1x1 sensors), and nine frozen
layers.  The paper's atmosphere comes from a closed simulator; these
configurations stand in for it with seeded synthetic layers.

A configuration is a plain dict (see ``_check``).  Noise levels are given as a
fraction of each sensor's clean-slope RMS; the caller turns that fraction into
sigma with whichever forward model it has (the oracle in tests, the GPU
library in the benchmark).
"""
import math

import numpy as np

ARCMIN = math.pi / 10800.0
LGS_HEIGHT = 90e3


def ring_angles(n, diameter_arcmin):
    """Directions of n stars on a ring: star k at angle 2*pi*k/n from +x."""
    r = 0.5 * diameter_arcmin * ARCMIN
    return [(r * math.cos(2 * math.pi * k / n), r * math.sin(2 * math.pi * k / n))
            for k in range(n)]


def _wfs(lgs, theta, n_sub, tt_aggregate=0, H=LGS_HEIGHT, remove_tt=None, in_precond=None):
    return {
        "lgs": bool(lgs),
        "theta": (float(theta[0]), float(theta[1])),
        "H": float(H),
        "n_sub": int(n_sub),
        "tt_aggregate": int(tt_aggregate),
        "remove_tt": bool(lgs) if remove_tt is None else bool(remove_tt),
        # high-order sensors enter the modified Jacobi preconditioner
        "in_precond": (n_sub > 2 and tt_aggregate == 0) if in_precond is None else bool(in_precond),
    }


def _layers(altitudes, weights, sizes, spacing=0.5):
    return [{"altitude": float(h), "weight": float(w), "spacing": float(spacing), "n": int(n)}
            for h, w, n in zip(altitudes, weights, sizes)]


def eelt_layer_sizes(altitudes, base=128, block=32):
    """Layer grids growing with altitude at a fixed 0.5 m spacing: 128 at the
    ground to 256 at 16 km, rounded up to a multiple of 32."""
    return [block * math.ceil(base * 2.0 ** (h / 16e3) / block) for h in altitudes]


def decreasing_cn2(cfg_id, n_layers):
    """Seeded decreasing Cn2 weights summing to one: n_layers uniform draws,
    sorted in decreasing order and normalised."""
    from .screens import rng_for
    w = rng_for(cfg_id, 0, 1).uniform(0.0, 1.0, n_layers)
    w = np.sort(w)[::-1]
    return list(w / w.sum())


def config_c1():
    """Tiny MCAO: 8 m, 16x16 Fried SH, 3 NGS on a 1 arcmin diameter ring,
    3 layers at 0/4/8 km of 64x64 at 0.5 m, db3 with 4 levels, 20 its from 0."""
    return _check({
        "name": "C1", "cfg_id": 1,
        "diameter": 8.0, "obstruction": 0.0,
        "layers": _layers([0.0, 4e3, 8e3], [0.6, 0.25, 0.15], [64, 64, 64]),
        "levels": 4,
        "wfs": [_wfs(False, t, 16) for t in ring_angles(3, 1.0)],
        "alpha": 1.0, "r0": 0.15, "L0": 25.0,
        "noise_frac": 0.1, "n_iter": 20, "warm": False,
    })


def config_c2():
    """E-ELT scale: 42 m (eps 0.28), 6 LGS at 90 km on a 2 arcmin diameter
    ring (84x84 SH, tip/tilt removed), 3 tip/tilt NGS on an 8/3 arcmin
    diameter ring (2x2, 1x1, 1x1 built from the fine grid), 9 layers at
    0..16 km of 128..256 pixels at 0.5 m, db3 with 5 levels, 10 PCG its warm."""
    alt = [2e3 * i for i in range(9)]
    wfs = [_wfs(True, t, 84) for t in ring_angles(6, 2.0)]
    tt = ring_angles(3, 8.0 / 3.0)
    wfs += [_wfs(False, tt[0], 84, tt_aggregate=2), _wfs(False, tt[1], 84, tt_aggregate=1),
            _wfs(False, tt[2], 84, tt_aggregate=1)]
    return _check({
        "name": "C2", "cfg_id": 2,
        "diameter": 42.0, "obstruction": 0.28,
        "layers": _layers(alt, decreasing_cn2(2, 9), eelt_layer_sizes(alt)),
        "levels": 5,
        "wfs": wfs,
        "alpha": 1.0, "r0": 0.15, "L0": 25.0,
        "noise_frac": 1.0 / 20.0, "n_iter": 10, "warm": True,
    })


def config_c4_classes():
    """The eight telescope classes mixed in one batch: {8 m/16x16/3 layers,
    16 m/32x32/5 layers, 39 m/78x78/9 layers, 42 m/84x84/9 layers} x
    {LGS-only: 6 LGS on a 1 arcmin radius ring at 90 km; NGS-only: 3
    high-order NGS on a 0.5 arcmin radius ring}."""
    out = []
    sizes = [(8.0, 16, 0.0, 3, [0.0, 4e3, 8e3], None, 4),
             (16.0, 32, 0.0, 5, [0.0, 4e3, 8e3, 12e3, 16e3], None, 4),
             (39.0, 78, 0.28, 9, [2e3 * i for i in range(9)], "eelt", 5),
             (42.0, 84, 0.28, 9, [2e3 * i for i in range(9)], "eelt", 5)]
    k = 0
    for (D, nsub, eps, nl, alt, grid, levels) in sizes:
        for lgs in (True, False):
            k += 1
            n = eelt_layer_sizes(alt) if grid == "eelt" else [64] * nl
            if lgs:
                wfs = [_wfs(True, t, nsub) for t in ring_angles(6, 2.0)]
            else:
                wfs = [_wfs(False, t, nsub) for t in ring_angles(3, 1.0)]
            out.append(_check({
                "name": f"C4-{int(D)}m-{'lgs' if lgs else 'ngs'}", "cfg_id": 40 + k,
                "diameter": D, "obstruction": eps,
                "layers": _layers(alt, decreasing_cn2(40 + k, nl), n),
                "levels": levels, "wfs": wfs,
                "alpha": 1.0, "r0": 0.15, "L0": 25.0,
                "noise_frac": (1.0 / 20.0) if lgs else 0.1, "n_iter": 10, "warm": True,
            }))
    return out


def config_by_name(name):
    if name == "C1":
        return config_c1()
    if name == "C2":
        return config_c2()
    if name == "C2-dm3":
        return config_c2_dm3()
    if name == "C2-cg9":
        return config_c2_cg9()
    for c in config_c4_classes():
        if c["name"] == name:
            return c
    raise KeyError(name)


def n_unknowns(cfg):
    return sum(L["n"] ** 2 for L in cfg["layers"])


def _check(cfg):
    J = cfg["levels"]
    for L in cfg["layers"]:
        assert L["n"] % (2 ** J) == 0, "layer size must be divisible by 2^levels"
        assert L["n"] >> (J - 1) >= 6, "coarsest transform length must hold the 6-tap filter"
    lgs_seen_ngs = False
    for w in cfg["wfs"]:
        if not w["lgs"]:
            lgs_seen_ngs = True
        else:
            assert not lgs_seen_ngs, "laser guide stars come first"
    return cfg


def sigmas_from_clean(cfg, clean_slopes, slope_offsets):
    """Noise level of each sensor: noise_frac * RMS of its clean slopes in
    the calibration frame."""
    f = float(cfg["noise_frac"])
    return [f * math.sqrt(float(np.mean(np.asarray(
        clean_slopes[slope_offsets[m]:slope_offsets[m + 1]], dtype=np.float64) ** 2)))
        for m in range(len(slope_offsets) - 1)]


def noisy_slopes(clean_slopes, sigmas, slope_offsets, xi):
    """clean + sigma_m * xi on sensor m's segment (xi standard normal)."""
    out = np.array(clean_slopes, dtype=np.float64, copy=True)
    for m, sg in enumerate(sigmas):
        a, b = slope_offsets[m], slope_offsets[m + 1]
        out[a:b] += sg * np.asarray(xi[a:b], dtype=np.float64)
    return out


def config_c2_dm3():
    """The paper's accelerated variant (Sec. 5.3): three layers reconstructed
    at the deformable-mirror altitudes 0, 4 and 12.7 km of the E-ELT set-up,
    PCG with the modified Jacobi preconditioner, 4 iterations, warm start.
    The 9-layer Cn2 profile is lumped onto the nearest mirror altitude."""
    base = config_c2()
    alt = [0.0, 4e3, 12.7e3]
    w = [0.0, 0.0, 0.0]
    for L in base["layers"]:
        k = int(np.argmin([abs(L["altitude"] - a) for a in alt]))
        w[k] += L["weight"]
    cfg = dict(base)
    cfg.update({"name": "C2-dm3", "cfg_id": 21,
                "layers": _layers(alt, w, eelt_layer_sizes(alt)), "n_iter": 4})
    return _check(cfg)


def config_c2_cg9():
    """The paper's quality variant (Sec. 5.2): nine layers, plain CG (no
    preconditioner), 10 iterations, warm start."""
    cfg = dict(config_c2())
    cfg.update({"name": "C2-cg9", "cfg_id": 22, "precond": False})
    return cfg
