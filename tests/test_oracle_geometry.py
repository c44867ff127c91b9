"""Pins of the oracle's projection (Sec. 2.1, eq. (2) and the cone-effect
projection), Fried slopes (eq. (3)-(4)), tip/tilt projection (Sec. 4.3,
eq. (17)) and pupil geometry."""
import os

import numpy as np
import pytest

import oracle as O
from oracle import geometry as geo
from tests.tiny import tiny_config

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_pupil_counts_golden():
    for line in open(os.path.join(GOLD, "pupil_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, D, eps, cnt = line.split()
        assert int(geo.subaperture_mask(int(n), float(D), float(eps)).sum()) == int(cnt)


def _ramp_layers(sysm, a, b, c):
    out = []
    for L in sysm.layers:
        x = geo.layer_coords(L["n"], L["spacing"])
        out.append(a * x[:, None] + b * x[None, :] + c)
    return out


def test_bilinear_reproduces_affine_fields():
    cfg = tiny_config()
    S = O.System(cfg, [1.0] * len(cfg["wfs"]))
    a, b, c = 0.37, -1.3, 2.0
    for l, L in enumerate(S.layers):
        x = geo.layer_coords(L["n"], L["spacing"])
        phi = a * x[:, None] + b * x[None, :] + c
        for sen in S.sensors:
            s, ix0, tx, jy0, ty = sen["axes"][l]
            u = geo.project_layer(phi, ix0, tx, jy0, ty)
            hl = L["altitude"]
            X = s * sen["nodes"] + sen["theta"][0] * hl
            Y = s * sen["nodes"] + sen["theta"][1] * hl
            expect = a * X[:, None] + b * Y[None, :] + c
            assert np.max(np.abs(u - expect)) < 1e-12


def test_ground_layer_ngs_is_index_sampling():
    cfg = tiny_config()
    S = O.System(cfg, [1.0] * len(cfg["wfs"]))
    sen = S.sensors[2]                     # natural guide star, layer 0 at h = 0
    s, ix0, tx, jy0, ty = sen["axes"][0]
    assert s == 1.0 and np.all(tx == 0.0) and np.all(ty == 0.0)
    phi = np.random.default_rng(1).standard_normal((32, 32))
    u = geo.project_layer(phi, ix0, tx, jy0, ty)
    off = 16 - 4                           # node i sits at pixel i - n_sub/2 + N/2
    np.testing.assert_array_equal(u, phi[off:off + 9, off:off + 9])


def test_projection_adjoint_identity():
    cfg = tiny_config()
    S = O.System(cfg, [1.0] * len(cfg["wfs"]))
    rng = np.random.default_rng(5)
    for l in range(len(S.layers)):
        for sen in S.sensors:
            s, ix0, tx, jy0, ty = sen["axes"][l]
            x = rng.standard_normal((32, 32))
            y = rng.standard_normal((9, 9))
            lhs = np.sum(geo.project_layer(x, ix0, tx, jy0, ty) * y)
            rhs = np.sum(x * geo.project_layer_adjoint(y, ix0, tx, jy0, ty, 32))
            assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_fried_ramp_piston_waffle():
    n, D = 8, 4.0
    d = D / n
    mask = geo.subaperture_mask(n, D, 0.2)
    S = int(mask.sum())
    x = geo.node_coords(n, D)
    a, b = 0.8, -0.45
    u = a * x[:, None] + b * x[None, :] + 3.0
    s = geo.fried_slopes(u, mask)
    np.testing.assert_allclose(s[:S], a * d, rtol=1e-14)
    np.testing.assert_allclose(s[S:], b * d, rtol=1e-14)
    assert np.max(np.abs(geo.fried_slopes(np.full((9, 9), 2.5), mask))) == 0.0
    waffle = (-1.0) ** (np.arange(9)[:, None] + np.arange(9)[None, :])
    assert np.max(np.abs(geo.fried_slopes(waffle, mask))) < 1e-15


def test_fried_adjoint_identity():
    mask = geo.subaperture_mask(8, 4.0, 0.2)
    rng = np.random.default_rng(9)
    u = rng.standard_normal((9, 9))
    w = rng.standard_normal(2 * int(mask.sum()))
    lhs = geo.fried_slopes(u, mask) @ w
    rhs = np.sum(u * geo.fried_adjoint(w, mask))
    assert abs(lhs - rhs) < 1e-12


def test_cone_effect_scales_ramp_slopes():
    # a ramp on one layer at altitude h: LGS slopes = (1 - h/H) x NGS slopes
    cfg = tiny_config(tt=False)
    lgs_theta = cfg["wfs"][0]["theta"]
    cfg["wfs"][2]["theta"] = lgs_theta     # same direction for the NGS
    S = O.System(cfg, [1.0] * len(cfg["wfs"]))
    x = geo.layer_coords(32, 0.5)
    layers = [np.zeros((32, 32)), 0.6 * x[:, None] - 0.2 * x[None, :]]
    s = S.forward_layers(layers)
    s_lgs = S.slopes_of(s, 0)
    s_ngs = S.slopes_of(s, 2)
    h, H = cfg["layers"][1]["altitude"], cfg["wfs"][0]["H"]
    np.testing.assert_allclose(s_lgs, (1 - h / H) * s_ngs, rtol=1e-12)


def test_tip_tilt_projection():
    cfg = tiny_config()
    S = O.System(cfg, [1.0] * len(cfg["wfs"]))
    n = S.sensors[0]["S"]
    rng = np.random.default_rng(4)
    v = rng.standard_normal(2 * n)
    w = rng.standard_normal(2 * n)
    Tv = S._tt_remove(v, n)
    np.testing.assert_allclose(S._tt_remove(Tv, n), Tv, atol=1e-14)         # idempotent
    assert abs(Tv @ w - v @ S._tt_remove(w, n)) < 1e-12                       # symmetric
    # slopes of any layer ramp are pure tip/tilt for a laser guide star
    x = geo.layer_coords(32, 0.5)
    layers = [0.3 * x[:, None] + 0.1 * x[None, :], -0.2 * x[:, None] + 0.5 * x[None, :]]
    sl = S.slopes_of(S.forward_layers(layers), 0)
    assert np.max(np.abs(S._tt_remove(sl, n))) < 1e-13


def test_aggregated_sensor_averages_fine_slopes():
    cfg = tiny_config()
    S = O.System(cfg, [1.0] * len(cfg["wfs"]))
    sen = S.sensors[3]
    assert sen["S"] == 4
    x = geo.node_coords(8, 4.0)
    u = 0.5 * x[:, None] ** 2 - x[None, :]
    fine = geo.fried_slopes(u, sen["mask"])
    agg = S._measure(sen, u)
    Sf = int(sen["mask"].sum())
    sx = np.zeros((8, 8))
    sx[sen["mask"]] = fine[:Sf]
    cell0 = sen["mask"].copy()
    cell0[4:, :] = False
    cell0[:, 4:] = False
    assert abs(agg[0] - sx[cell0].mean()) < 1e-14
    w = np.random.default_rng(0).standard_normal(8)
    lhs = agg @ w
    rhs = np.sum(u * S._measure_adjoint(sen, w))
    assert abs(lhs - rhs) < 1e-12


def test_footprint_outside_grid_raises():
    cfg = tiny_config()
    cfg["wfs"][0]["theta"] = (40 * O.geometry.np.pi / 10800, 0.0)   # 40 arcmin: far off grid
    with pytest.raises(O.FootprintError):
        O.System(cfg, [1.0] * len(cfg["wfs"]))
