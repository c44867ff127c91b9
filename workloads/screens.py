"""Seeded random draws: von Karman phase screens, frozen-flow shifts, noise,
wind directions and Poisson arrival times.

Every draw comes from ``numpy.random.default_rng(SeedSequence([cfg_id, frame,
stream]))`` with stream 0 = screens, 1 = Cn2 profile, 2 = noise, 3 = wind,
4 = arrivals, so any frame of any configuration can be regenerated alone.
"""
import math

import numpy as np

STREAM_SCREENS, STREAM_CN2, STREAM_NOISE, STREAM_WIND, STREAM_ARRIVALS = range(5)


def rng_for(cfg_id, frame, stream):
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(frame), int(stream)]))


def von_karman_psd(f, r0, L0):
    """Phase power spectrum of von Karman turbulence (Sec. 3, von Karman
    modification of eq. (10)), in rad^2 m^2 at the wavelength r0 refers to."""
    return 0.023 * r0 ** (-5.0 / 3.0) * (f * f + L0 ** -2.0) ** (-11.0 / 6.0)


def von_karman_screen(n, spacing, r0, L0, rng):
    """Periodic n x n phase screen [x][y] in rad: white complex Gaussian
    shaped by sqrt(PSD) * df, real part, piston removed."""
    df = 1.0 / (n * spacing)
    fx = np.fft.fftfreq(n, d=spacing)
    f = np.sqrt(fx[:, None] ** 2 + fx[None, :] ** 2)
    amp = np.sqrt(von_karman_psd(f, r0, L0)) * df
    amp[0, 0] = 0.0
    c = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    scr = np.real(np.fft.ifft2(c * amp)) * (n * n)
    return scr - scr.mean()


def layer_screens(cfg, frame=0, seed_frame=None):
    """Truth layers of one frame: a list of n_l x n_l arrays.  Layer l gets
    Fried parameter r0 * w_l^(-3/5).  With ``seed_frame`` set, the screens of
    that frame are drawn and advanced by frozen flow to ``frame``."""
    base = frame if seed_frame is None else seed_frame
    rng = rng_for(cfg["cfg_id"], base, STREAM_SCREENS)
    out = []
    for L in cfg["layers"]:
        r0l = cfg["r0"] * L["weight"] ** (-3.0 / 5.0)
        out.append(von_karman_screen(L["n"], L["spacing"], r0l, cfg["L0"], rng))
    if seed_frame is not None and frame != seed_frame:
        dirs = wind_directions(cfg)
        out = [frozen_flow_shift(s, L["spacing"], dirs[i], (frame - seed_frame))
               for i, (s, L) in enumerate(zip(out, cfg["layers"]))]
    return out


def wind_directions(cfg):
    rng = rng_for(cfg["cfg_id"], 0, STREAM_WIND)
    return rng.uniform(0.0, 2.0 * math.pi, len(cfg["layers"]))


def frozen_flow_shift(screen, spacing, direction, steps, speed=10.0, dt=2e-3):
    """Shift a periodic screen by steps * speed * dt metres along ``direction``
    (Fourier phase ramp, so sub-pixel shifts are exact on the periodic grid)."""
    n = screen.shape[0]
    d = steps * speed * dt
    sx, sy = d * math.cos(direction), d * math.sin(direction)
    f = np.fft.fftfreq(n, d=spacing)
    ramp = np.exp(-2j * math.pi * (f[:, None] * sx + f[None, :] * sy))
    return np.real(np.fft.ifft2(np.fft.fft2(screen) * ramp))


def noise_draw(cfg_id, frame, n):
    """Standard normal draws for one frame's slopes (scaled by sigma later)."""
    return rng_for(cfg_id, frame, STREAM_NOISE).standard_normal(n)


def poisson_arrivals(cfg_id, rate_hz, duration_s):
    """Arrival times (s) of a Poisson stream."""
    rng = rng_for(cfg_id, 0, STREAM_ARRIVALS)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.asarray(out)
        out.append(t)
