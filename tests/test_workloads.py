"""Checks of the synthetic inputs: von Karman screen statistics, seeding and
frozen flow."""
import math

import numpy as np

import workloads as WL


def test_screen_structure_function_follows_von_karman_law():
    # Small-separation expansion of the von Karman phase structure function:
    # D(r) = 6.88 (r/r0)^(5/3) [1 - 1.485 (r/L0)^(1/3) + 3.079 (r/L0)^2 - ...].
    # The FFT screen lacks sub-harmonics and frequencies beyond Nyquist, so it
    # may fall a little below the law; 1 and 2 m separations are checked.
    n, d, r0, L0 = 128, 0.5, 0.15, 25.0
    acc = {2: [], 4: []}
    for s in range(20):
        scr = WL.von_karman_screen(n, d, r0, L0, WL.rng_for(777, s, 0))
        for k in acc:
            acc[k].append(np.mean((scr - np.roll(scr, k, axis=0)) ** 2))
            acc[k].append(np.mean((scr - np.roll(scr, k, axis=1)) ** 2))
    for k, v in acc.items():
        r = k * d
        law = 6.88 * (r / r0) ** (5.0 / 3.0) * (1 - 1.485 * (r / L0) ** (1 / 3) + 3.079 * (r / L0) ** 2)
        ratio = np.mean(v) / law
        assert 0.85 < ratio < 1.1, (k, ratio)


def test_seeded_draws_are_reproducible_and_distinct():
    cfg = WL.config_c1()
    a = WL.layer_screens(cfg, 3)
    b = WL.layer_screens(cfg, 3)
    c = WL.layer_screens(cfg, 4)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.allclose(a[0], c[0])
    assert np.array_equal(WL.noise_draw(1, 2, 10), WL.noise_draw(1, 2, 10))


def test_frozen_flow_integer_shift_is_a_roll():
    scr = WL.von_karman_screen(32, 0.5, 0.15, 25.0, WL.rng_for(5, 0, 0))
    # 25 steps x 10 m/s x 2 ms = 0.5 m = one pixel along +x
    out = WL.frozen_flow_shift(scr, 0.5, 0.0, 25)
    assert np.max(np.abs(out - np.roll(scr, 1, axis=0))) < 1e-10


def test_configs_shapes():
    c2 = WL.config_c2()
    assert WL.n_unknowns(c2) == 372736
    assert [L["n"] for L in c2["layers"]] == [128, 160, 160, 192, 192, 224, 224, 256, 256]
    assert abs(sum(L["weight"] for L in c2["layers"]) - 1.0) < 1e-12
    w = [L["weight"] for L in c2["layers"]]
    assert all(w[i] >= w[i + 1] for i in range(len(w) - 1))
    assert len(WL.config_c4_classes()) == 8
    assert WL.n_unknowns(WL.config_c1()) == 12288
    t = WL.poisson_arrivals(5, 500.0, 2.0)
    assert 850 < len(t) < 1150 and np.all(np.diff(t) > 0)
