"""Work-shape autotuner for a telescope configuration.

The plan options that only decide how the work is cut (not what is computed)
are tuned here: the tile edge of the tiled wavelet levels, the LDS budget of
the whole-band wavelet kernels (which decides how many fine levels run as
tiled launches), the node rows per projection and weighting work item, the
LDS budget of an adjoint-projection work item (which decides its footprint
rows), and the vector elements per PCG-update work item.  The operator
precision is not tuned: it decides the results.

The objective is the time of a whole warm-started PCG solve of `batch`
frames on the current device (HIP events around solves run back to back),
since the shapes interact:
smaller work items fill the GPU better at batch 1 and cost more per launch
at large batches.  The search is coordinate descent from the library
defaults: each option in turn takes the candidate that shortens the solve by
more than 1 %, the others held.  Results are cached in a JSON file keyed by
(device architecture, layer sizes, sensor sizes, levels, dtype, batch,
iterations).
"""
import json
import os
import statistics
import threading

import torch

from .plan import Plan

# option: candidates, the library default first
SPACE = {
    "tile": [32, 16, 64],
    "lds_budget": [8 * 1024, 2 * 1024, 32 * 1024],
    "proj_rows": [8, 4, 16, 32, 48],
    "adj_lds": [32 * 1024, 16 * 1024, 64 * 1024],
    "vec_chunk": [2048, 1024, 4096],
}
DEFAULTS = {k: v[0] for k, v in SPACE.items()}
_lock = threading.Lock()


def cache_path():
    return os.environ.get("WMCAO_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "wmcao", "tune.json"))


def _key(cfg, dtype, batch, n_iter, plan_kw):
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    layers = ",".join(str(L["n"]) for L in cfg["layers"])
    wfs = ",".join(f"{w['n_sub']}{'a' if w.get('tt_aggregate') else ''}" for w in cfg["wfs"])
    extra = ",".join(f"{k}={plan_kw[k]}" for k in sorted(plan_kw) if k != "cinv_blocks")
    return f"{arch}|L{layers}|W{wfs}|J{cfg['levels']}|{dtype}|B{batch}|it{n_iter}|{extra}"


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


def time_solve(plan, batch, n_iter=10, reps=7, rounds=3):
    """Time (ms) of one warm-started PCG solve of `batch` frames (seeded
    synthetic slopes and starts): `reps` solves back to back, as a stream of
    frames runs them, the median over `rounds`."""
    gen = torch.Generator(device="cuda").manual_seed(11)
    s = torch.randn(batch, plan.n_slopes, dtype=plan.torch_dtype, device="cuda", generator=gen) * 0.1
    x = torch.randn(batch, plan.n, dtype=plan.torch_dtype, device="cuda", generator=gen) * 0.01
    for _ in range(2):
        plan.solve(s, x, n_iter=n_iter, warm_start=True)
    torch.cuda.synchronize()
    times = []
    for _ in range(rounds):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            plan.solve(s, x, n_iter=n_iter, warm_start=True)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / reps)
    return statistics.median(times)


def _measure(cfg, sigmas, dtype, batch, n_iter, reps, opts, plan_kw):
    """(ms, None), or (None, reason) for a shape this configuration cannot take."""
    try:
        plan = Plan(cfg, sigmas, dtype=dtype, max_batch=batch, **opts, **plan_kw)
    except Exception as e:
        return None, str(e)[:200]
    try:
        return time_solve(plan, batch, n_iter, reps), None
    except Exception as e:
        return None, str(e)[:200]
    finally:
        plan.close()


def tune(cfg, sigmas, dtype="f32", batch=1, n_iter=10, reps=7, force=False, **plan_kw):
    """The fastest work shapes for this configuration, dtype and batch, as a
    dict of plan options (cached on disk)."""
    key = _key(cfg, dtype, batch, n_iter, plan_kw)
    with _lock:
        db = _load()
        if key in db and not force:
            return dict(db[key]["best"])
    cur = dict(DEFAULTS)
    t_default, err = _measure(cfg, sigmas, dtype, batch, n_iter, reps, cur, plan_kw)
    if t_default is None:
        raise RuntimeError(f"autotune: the default shapes fail for this configuration: {err}")
    best_t = t_default
    tried = {json.dumps(cur, sort_keys=True): round(t_default, 5)}
    for name, cands in SPACE.items():
        for v in cands:
            if v == cur[name]:
                continue
            trial = dict(cur, **{name: v})
            t, err = _measure(cfg, sigmas, dtype, batch, n_iter, reps, trial, plan_kw)
            tried[json.dumps(trial, sort_keys=True)] = round(t, 5) if t is not None else err
            if t is not None and t < 0.99 * best_t:
                cur, best_t = trial, t
    with _lock:
        db = _load()
        db[key] = {"best": cur, "ms": best_t, "default_ms": t_default, "tried": tried}
        _store(db)
    return dict(cur)


def record(cfg, dtype="f32", batch=1, n_iter=10, **plan_kw):
    """The cached tuning record (best shapes, their time, the defaults' time
    and every shape tried), or None."""
    return _load().get(_key(cfg, dtype, batch, n_iter, plan_kw))


def tuned_plan(cfg, sigmas, dtype="f32", max_batch=1, n_iter=10, **kw):
    """A Plan with the tuned work shapes for max_batch frames."""
    plan_kw = {k: v for k, v in kw.items() if k not in SPACE}
    best = tune(cfg, sigmas, dtype, max_batch, n_iter, **plan_kw)
    return Plan(cfg, sigmas, dtype=dtype, max_batch=max_batch, **best, **plan_kw)
