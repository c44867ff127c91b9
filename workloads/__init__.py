"""Seeded synthetic inputs for the wavelet-MCAO tomography solve.

This package holds the telescope/atmosphere configurations and the random
draws (turbulence screens, Cn2 profiles, noise, wind, arrival times).  It holds
none of the reconstruction method's arithmetic: no wavelet transform, no
projection, no slope operator.  Both the CPU oracle tests and the GPU path take
their inputs from here.
"""
from .configs import (ARCMIN, config_c1, config_c2, config_c2_dm3, config_c2_cg9,
                      config_c4_classes, config_by_name,
                      sigmas_from_clean, noisy_slopes,
                      ring_angles, n_unknowns)
from .screens import (von_karman_screen, layer_screens, frozen_flow_shift, wind_directions,
                      noise_draw, poisson_arrivals, rng_for)

__all__ = [
    "ARCMIN", "config_c1", "config_c2", "config_c2_dm3", "config_c2_cg9", "config_c4_classes", "config_by_name", "ring_angles",
    "n_unknowns", "sigmas_from_clean", "noisy_slopes", "von_karman_screen", "layer_screens", "frozen_flow_shift", "wind_directions",
    "noise_draw", "poisson_arrivals", "rng_for",
]
