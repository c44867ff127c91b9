"""Small configurations for tests (a few thousand unknowns)."""
import copy

from workloads.configs import ARCMIN, _check, _layers, _wfs, ring_angles


def tiny_config(tt=True, obstruction=0.2):
    """4 m pupil, 8x8 Fried sensors; 2 LGS (tip/tilt removed), 1 high-order
    NGS and optionally a 2x2 low-order NGS; 2 layers of 32x32, 3 levels."""
    lgs = ring_angles(2, 1.0)
    wfs = [_wfs(True, t, 8) for t in lgs]
    wfs.append(_wfs(False, (0.2 * ARCMIN, -0.1 * ARCMIN), 8))
    if tt:
        wfs.append(_wfs(False, (-0.3 * ARCMIN, 0.25 * ARCMIN), 8, tt_aggregate=2))
    return _check({
        "name": "tiny", "cfg_id": 900,
        "diameter": 4.0, "obstruction": obstruction,
        "layers": _layers([0.0, 6e3], [0.7, 0.3], [32, 32]),
        "levels": 3,
        "wfs": wfs,
        "alpha": 1.0, "r0": 0.15, "L0": 25.0,
        "noise_frac": 0.1, "n_iter": 8, "warm": False,
    })


def tiny_ragged_config():
    """Two layers of different, non-power-of-two sizes (40 and 48 = 5 and 6
    tiles of 8) so that tiled kernels see ragged edges."""
    cfg = tiny_config(tt=True)
    cfg = copy.deepcopy(cfg)
    cfg["name"] = "tiny-ragged"
    cfg["cfg_id"] = 901
    cfg["layers"] = _layers([0.0, 6e3], [0.7, 0.3], [40, 48])
    return _check(cfg)


def tiny_max_config():
    """The library's maximum sizes on a small pupil: 16 layers of 32x32 at
    0..15 km and 32 sensors (24 LGS, 7 high-order NGS, one 2x2 low-order
    NGS) of 8x8 subapertures within half an arcminute."""
    cfg = tiny_config(tt=False)
    cfg = copy.deepcopy(cfg)
    cfg["name"] = "tiny-max"
    cfg["cfg_id"] = 902
    alts = [1e3 * k for k in range(16)]
    w = [2.0 ** (-k / 4.0) for k in range(16)]
    tot = sum(w)
    cfg["layers"] = _layers(alts, [x / tot for x in w], [32] * 16)
    wfs = [_wfs(True, t, 8) for t in ring_angles(24, 0.5)]
    wfs += [_wfs(False, t, 8) for t in ring_angles(7, 0.3)]
    wfs.append(_wfs(False, (0.1 * ARCMIN, -0.2 * ARCMIN), 8, tt_aggregate=2))
    cfg["wfs"] = wfs
    return _check(cfg)


def tiny_edge_config():
    """Footprints that reach the layers' first pixel row and column: two
    16 x 16 layers (2 levels) and a high-order NGS 1.1 arcmin off axis in both
    directions, whose nodes on the 6 km layer start 0.16 pixel from the edge,
    plus an on-axis LGS.  With 16-pixel tiles the one level-1 analysis tile
    of a layer reads a window that wraps around both edges back into that
    footprint."""
    cfg = tiny_config(tt=False)
    cfg = copy.deepcopy(cfg)
    cfg["name"] = "tiny-edge"
    cfg["cfg_id"] = 903
    cfg["layers"] = _layers([0.0, 6e3], [0.7, 0.3], [16, 16])
    cfg["levels"] = 2
    cfg["wfs"] = [_wfs(True, (0.0, 0.0), 8), _wfs(False, (-1.1 * ARCMIN, -1.1 * ARCMIN), 8)]
    return _check(cfg)
