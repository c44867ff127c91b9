"""Work-shape autotuner: it times candidate shapes (wavelet tile, whole-band
LDS budget, projection rows, adjoint LDS, vector chunk) on whole PCG solves,
caches the choice in a JSON file, and tuned plans still match the FP64 oracle:
the 8 m system in FP64 (1e-11) and the E-ELT system in FP32 (1e-5)."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests.gpu_common import record, rel, require_gpu, say, setup, slopes_for, solve_errors, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_autotune_caches_and_tuned_plan_is_exact(tmp_path, monkeypatch):
    require_gpu()
    import torch
    from paper_1302_3734_amd import autotune
    monkeypatch.setenv("WMCAO_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = WL.config_c1()
    S, sig, s, _ = setup(cfg)
    best = autotune.tune(cfg, sig, dtype="f64", batch=2, reps=3)
    assert set(best) == set(autotune.SPACE)
    assert all(best[k] in autotune.SPACE[k] for k in best)
    db = json.loads((tmp_path / "tune.json").read_text())
    (entry,) = db.values()
    say(f"[autotune] best {best}, {entry['ms']:.3f} ms against {entry['default_ms']:.3f} ms default; "
        f"{len(entry['tried'])} shapes tried")
    assert entry["best"] == best and len(entry["tried"]) >= 8
    assert autotune.tune(cfg, sig, dtype="f64", batch=2) == best    # cache hit
    plan = autotune.tuned_plan(cfg, sig, dtype="f64", max_batch=2)
    b = S.rhs(s)
    x_ref, _ = O.pcg(S.apply_A, b, 10, jacobi=S.jacobi_separable())
    x = to_np(plan.solve(to_dev(s[None], torch.float64), n_iter=10)).ravel()
    e = solve_errors(S, x, x_ref, b)
    say(f"[autotune] C1 FP64 tuned: e {e}")
    record("C1-tuned", "f64", e, (1e-11,) * 3)
    assert max(e) < 1e-11
    plan.close()


def test_tuned_eelt_fp32_plan_matches_oracle(tmp_path, monkeypatch):
    """The E-ELT FP32 plan tuned for 4 frames solves a warm-started frame
    within the fixed 1e-5 bar."""
    require_gpu()
    import torch
    from paper_1302_3734_amd import autotune
    monkeypatch.setenv("WMCAO_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = WL.config_c2()
    S, sig, s0, _ = setup(cfg, frame=0, seed_frame=0)
    J = S.jacobi_separable()
    x0, _ = O.pcg(S.apply_A, S.rhs(s0), 20, jacobi=J)
    s1 = slopes_for(S, cfg, sig, 1, seed_frame=0)
    x0_in = to_np(to_dev(x0, torch.float32)).ravel()
    s1_in = to_np(to_dev(s1, torch.float32)).ravel()
    b = S.rhs(s1_in)
    x_ref, _ = O.pcg(S.apply_A, b, 10, x0=x0_in, jacobi=J)
    plan = autotune.tuned_plan(cfg, sig, dtype="f32", max_batch=4)
    say(f"[autotune] E-ELT FP32 batch 4: {json.loads((tmp_path / 'tune.json').read_text())}")
    X = to_dev(np.repeat(x0_in[None], 4, 0), torch.float32)
    plan.solve(to_dev(np.repeat(s1_in[None], 4, 0), torch.float32), X, n_iter=10, warm_start=True)
    Xn = to_np(X).reshape(4, -1)
    for f in range(4):
        e = solve_errors(S, Xn[f], x_ref, b)
        record("C2-tuned", "f32", e, (1e-5,) * 3)
        assert max(e) < 1e-5, (f, e)
    assert all(np.array_equal(Xn[f], Xn[0]) for f in range(4))
    plan.close()
