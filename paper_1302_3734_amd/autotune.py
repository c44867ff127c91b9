"""Tile-shape autotuner for the wavelet kernels.

For a telescope configuration, dtype and batch size it times the full
operator apply (W^-1, sensors, P^T + W) for every candidate (tile edge of the
tiled wavelet levels, LDS budget of the whole-band kernels) on the current
device with HIP events, and caches the fastest choice in a JSON file keyed by
(device architecture, layer sizes, sensor sizes, levels, dtype, batch).  The
LDS budget decides how many fine levels run as tiled launches and how many in
one LDS-resident block per layer.
"""
import json
import os
import statistics
import threading

import torch

from .plan import Plan

CANDIDATES = [(16, 2 * 1024), (16, 8 * 1024), (32, 2 * 1024), (32, 8 * 1024),
              (32, 32 * 1024), (64, 8 * 1024)]
_lock = threading.Lock()


def cache_path():
    return os.environ.get("WMCAO_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "wmcao", "tune.json"))


def _key(cfg, dtype, batch):
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    layers = ",".join(str(L["n"]) for L in cfg["layers"])
    wfs = ",".join(f"{w['n_sub']}{'a' if w.get('tt_aggregate') else ''}" for w in cfg["wfs"])
    return f"{arch}|L{layers}|W{wfs}|J{cfg['levels']}|{dtype}|B{batch}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_apply(plan, batch, reps=20):
    """Median time (ms) of one batched operator apply."""
    x = torch.randn(batch, plan.n, dtype=plan.torch_dtype, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        plan.apply_A(x, y)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.apply_A(x, y)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(cfg, sigmas, dtype="f32", batch=1, reps=20, force=False):
    """Fastest (tile, lds_budget) for this configuration; cached on disk."""
    key = _key(cfg, dtype, batch)
    with _lock:
        db = _load()
        if key in db and not force:
            return tuple(db[key]["best"])
    results = {}
    for tile, lds in CANDIDATES:
        if dtype == "f64" and tile == 64:
            continue
        plan = Plan(cfg, sigmas, dtype=dtype, max_batch=batch, tile=tile, lds_budget=lds)
        try:
            results[(tile, lds)] = time_apply(plan, batch, reps)
        finally:
            plan.close()
    best = min(results, key=results.get)
    with _lock:
        db = _load()
        db[key] = {"best": list(best),
                   "ms": {f"{t}/{l}": round(v, 5) for (t, l), v in results.items()}}
        _store(db)
    return best


def tuned_plan(cfg, sigmas, dtype="f32", max_batch=1, **kw):
    """A Plan built with the tuned tile edge and LDS budget."""
    tile, lds = tune(cfg, sigmas, dtype, max_batch)
    return Plan(cfg, sigmas, dtype=dtype, max_batch=max_batch, tile=tile, lds_budget=lds, **kw)
