"""Spot-elongation noise model of laser guide stars (input side).

A sodium-layer spot seen from subaperture r is elongated along r - r_launch
(the laser launch position) by about dh |r - r_launch| / H^2 radians, dh the
sodium layer thickness.  The paper's per-subaperture noise covariance is
C~ = sigma^2 (I + tau/f^2 beta beta^T) with beta that elongation vector and f
the non-elongated spot FWHM (Sec. 4.3, eq. (16)).  This module draws the
blocks and matching noise for the active subapertures of a sensor (centre in
the closed annulus, row-major order).
"""
import math

import numpy as np

ARCSEC = math.pi / 648000.0


def active_centres(n_sub, D, eps):
    c = (np.arange(n_sub) + 0.5 - n_sub / 2.0) * (D / n_sub)
    X, Y = np.meshgrid(c, c, indexing="ij")
    r2 = X ** 2 + Y ** 2
    act = (r2 <= (D / 2.0) ** 2) & (r2 >= (eps * D / 2.0) ** 2)
    return X[act], Y[act]


def elongation_blocks(cfg, m, sigma, tau=0.8, fwhm_arcsec=1.1, thickness=10e3):
    """(cov, cinv): arrays [S, 3] holding (a, b, c) of the symmetric 2x2
    covariance blocks of sensor m and of their inverses."""
    w = cfg["wfs"][m]
    D = cfg["diameter"]
    x, y = active_centres(w["n_sub"], D, cfg["obstruction"])
    th = np.hypot(*w["theta"])
    ux, uy = (w["theta"][0] / th, w["theta"][1] / th) if th > 0 else (1.0, 0.0)
    lx, ly = 0.5 * D * ux, 0.5 * D * uy                  # side launch at the pupil edge
    H = w["H"]
    bx = thickness * (x - lx) / H ** 2
    by = thickness * (y - ly) / H ** 2
    f = fwhm_arcsec * ARCSEC
    k = tau / f ** 2
    a = sigma ** 2 * (1.0 + k * bx * bx)
    b = sigma ** 2 * (k * bx * by)
    c = sigma ** 2 * (1.0 + k * by * by)
    det = a * c - b * b
    cov = np.stack([a, b, c], axis=1)
    cinv = np.stack([c / det, -b / det, a / det], axis=1)
    return cov, cinv


def elongated_noise(cov, rng):
    """One draw of x/y noise with the given 2x2 covariance blocks; returns the
    sensor's noise vector [x-slopes, y-slopes]."""
    a, b, c = cov[:, 0], cov[:, 1], cov[:, 2]
    l11 = np.sqrt(a)
    l21 = b / l11
    l22 = np.sqrt(np.maximum(c - l21 ** 2, 0.0))
    z1 = rng.standard_normal(len(a))
    z2 = rng.standard_normal(len(a))
    return np.concatenate([l11 * z1, l21 * z1 + l22 * z2])
