"""Tile autotuner: it times every candidate (tile edge, LDS budget) of the
wavelet kernels on the device, caches the fastest in a JSON file, and a plan
built with the choice still matches the FP64 oracle."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests.gpu_common import rel, require_gpu, say, setup, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_autotune_caches_and_tuned_plan_is_exact(tmp_path, monkeypatch):
    require_gpu()
    import torch
    from paper_1302_3734_amd import autotune
    monkeypatch.setenv("WMCAO_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = WL.config_c1()
    S, sig, s, _ = setup(cfg)
    best = autotune.tune(cfg, sig, dtype="f64", batch=2, reps=3)
    assert best in autotune.CANDIDATES
    db = json.loads((tmp_path / "tune.json").read_text())
    (entry,) = db.values()
    say(f"[autotune] best {best} of {entry['ms']}")
    assert tuple(entry["best"]) == best and len(entry["ms"]) >= 2
    assert autotune.tune(cfg, sig, dtype="f64", batch=2) == best    # cache hit
    plan = autotune.tuned_plan(cfg, sig, dtype="f64", max_batch=1)
    b = S.rhs(s)
    x_ref, _ = O.pcg(S.apply_A, b, 10, jacobi=S.jacobi_separable())
    x = to_np(plan.solve(to_dev(s[None], torch.float64), n_iter=10)).ravel()
    say(f"[autotune] e_x {rel(x, x_ref):.2e}")
    assert rel(x, x_ref) < 1e-11
    plan.close()
