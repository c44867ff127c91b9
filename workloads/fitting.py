"""Deformable mirrors and fitting directions of the E-ELT MCAO set-up.

The paper's system has three deformable mirrors conjugated to 0, 4 and
12.7 km, modelled as piecewise bilinear surfaces with about 9300 degrees of
freedom in total, and evaluates (and fits) on a 5 x 5 grid of directions over
a 2 arcmin square field (Sec. 5.1).  The mirror pitches below (0.5, 1 and
2 m) are a reading: grids just large enough to cover every fitting
direction's footprint, about 10,500 actuators.

``fitting_systems`` returns the two configuration dicts the fitting step
needs, sharing 25 "phase" sensors (one per direction, 84 x 84 pupil nodes):
the atmosphere (the tomography layers, to evaluate P phi) and the mirrors
(actuator grids as layers with no wavelet transform, to solve
(H^T H + alpha I) a = H^T P phi).
"""
import copy

from .configs import ARCMIN


def eelt_mirrors():
    return [{"altitude": 0.0, "pitch": 0.5, "n": 86},
            {"altitude": 4e3, "pitch": 1.0, "n": 48},
            {"altitude": 12.7e3, "pitch": 2.0, "n": 28}]


def fitting_directions(side_arcmin=2.0, k=5):
    step = side_arcmin / (k - 1)
    c = [(-side_arcmin / 2 + i * step) * ARCMIN for i in range(k)]
    return [(x, y) for x in c for y in c]


def phase_sensors(directions, n_sub=84):
    return [{"lgs": False, "theta": (float(t[0]), float(t[1])), "H": 90e3, "n_sub": n_sub,
             "tt_aggregate": 0, "remove_tt": False, "in_precond": True, "kind": "phase"}
            for t in directions]


def fitting_systems(tomo_cfg, mirrors=None, directions=None, alpha_fit=1e-3, n_iter=4,
                    n_sub=84):
    mirrors = eelt_mirrors() if mirrors is None else mirrors
    sensors = phase_sensors(fitting_directions() if directions is None else directions, n_sub)
    atm = copy.deepcopy(tomo_cfg)
    atm.update({"name": tomo_cfg["name"] + "-fit-atm", "wfs": copy.deepcopy(sensors)})
    dm = {"name": tomo_cfg["name"] + "-fit-dm", "cfg_id": tomo_cfg["cfg_id"] + 500,
          "diameter": tomo_cfg["diameter"], "obstruction": tomo_cfg["obstruction"],
          "layers": [{"altitude": m["altitude"], "weight": 1.0, "spacing": m["pitch"],
                      "n": m["n"]} for m in mirrors],
          "levels": 0, "wfs": copy.deepcopy(sensors),
          "alpha": alpha_fit, "r0": tomo_cfg["r0"], "L0": tomo_cfg["L0"],
          "n_iter": n_iter, "warm": True, "noise_frac": 0.0}
    return atm, dm


def mirror_wfs_system(tomo_cfg, mirrors=None):
    """The tomography's own sensors looking at the mirrors (A^ of the
    pseudo-open-loop control, Sec. 4.2): mirror grids as layers, no wavelet
    transform."""
    mirrors = eelt_mirrors() if mirrors is None else mirrors
    cfg = copy.deepcopy(tomo_cfg)
    cfg.update({"name": tomo_cfg["name"] + "-dm-wfs", "levels": 0,
                "layers": [{"altitude": m["altitude"], "weight": 1.0, "spacing": m["pitch"],
                            "n": m["n"]} for m in mirrors]})
    return cfg
