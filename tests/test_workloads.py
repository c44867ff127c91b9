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


def test_elongation_blocks_follow_eq16_and_invert():
    from workloads.elongation import elongation_blocks, elongated_noise
    cfg = WL.config_c2()
    cov, cinv = elongation_blocks(cfg, 0, sigma=0.2)
    assert cov.shape == (5112, 3)
    # C = sigma^2 (I + tau/f^2 beta beta^T): eigenvalues sigma^2 and
    # sigma^2 (1 + tau |beta|^2 / f^2) >= sigma^2, the larger along beta
    for q in (0, 100, 4000):
        C = np.array([[cov[q, 0], cov[q, 1]], [cov[q, 1], cov[q, 2]]])
        Ci = np.array([[cinv[q, 0], cinv[q, 1]], [cinv[q, 1], cinv[q, 2]]])
        assert np.allclose(C @ Ci, np.eye(2), atol=1e-10)
        ev = np.linalg.eigvalsh(C)
        assert abs(ev[0] - 0.04) < 1e-12 and ev[1] >= 0.04
    # the subaperture far from the launch point is the most elongated
    el = cov[:, 0] + cov[:, 2] - 2 * 0.04
    assert el.max() / el.min() > 10
    rng = np.random.default_rng(0)
    draws = np.stack([elongated_noise(cov[:3], rng) for _ in range(20000)])
    S = 3
    for q in range(3):
        emp = np.cov(draws[:, q], draws[:, S + q])
        assert np.allclose(emp, [[cov[q, 0], cov[q, 1]], [cov[q, 1], cov[q, 2]]], rtol=0.05, atol=2e-3)
