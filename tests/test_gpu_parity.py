"""GPU parity of every operator stage against the FP64 oracle, through the C ABI.

Tolerances: the FP64 path must agree with the oracle to rounding level
(1e-12 relative for one operator application); the FP32 path to 1e-5, with
single-precision operators (op_precision 32) or FP64 operators (64)."""
import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests.gpu_common import maxrel, rel, require_gpu, say, setup, to_dev, to_np
from tests.tiny import tiny_config, tiny_edge_config, tiny_max_config, tiny_ragged_config

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _torch_dtype(dt):
    import torch
    return torch.float64 if dt == "f64" else torch.float32


CASES = [
    # (name, config builder, dtype, plan kwargs)
    ("tiny-f64", tiny_config, "f64", {}),
    ("tiny-f32", tiny_config, "f32", {}),
    ("ragged-tiled-f64", tiny_ragged_config, "f64", {"tile": 16, "lds_budget": 1024}),
    ("ragged-tiled-f32", tiny_ragged_config, "f32", {"tile": 16, "lds_budget": 512}),
    ("max-f64", tiny_max_config, "f64", {}),
    ("max-f32", tiny_max_config, "f32", {"tile": 16}),
    ("c1-f64", WL.config_c1, "f64", {}),
    ("c1-tiled-f64", WL.config_c1, "f64", {"tile": 32, "lds_budget": 2048}),
    ("c2-f64", WL.config_c2, "f64", {}),
    ("c2-f32", WL.config_c2, "f32", {}),
    ("c2-f64-lds160", WL.config_c2, "f64", {"lds_budget": 160 * 1024}),
    # 40..64-wide coarse blocks, rebuilt in each level-k0 synthesis tile
    ("c2-f32-lds32", WL.config_c2, "f32", {"lds_budget": 32 * 1024}),
    ("c2-f32-tile64", WL.config_c2, "f32", {"tile": 64}),
    # single-precision operators on the small systems too (their default is
    # FP64 operators), at several tiles and with ragged tails
    ("tiny-f32-op32", tiny_config, "f32", {"op_precision": 32}),
    ("ragged-tiled-f32-op32", tiny_ragged_config, "f32", {"tile": 16, "lds_budget": 512,
                                                          "op_precision": 32}),
    ("max-f32-op32", tiny_max_config, "f32", {"tile": 16, "op_precision": 32}),
    ("c1-f32", WL.config_c1, "f32", {}),
    ("c2-f32-op64", WL.config_c2, "f32", {"op_precision": 64}),
    # every work shape the autotuner may choose away from the defaults
    ("c2-f32-rows16", WL.config_c2, "f32", {"proj_rows": 16, "adj_lds": 64 * 1024}),
    ("c2-f64-rows4", WL.config_c2, "f64", {"proj_rows": 4, "adj_lds": 16 * 1024, "vec_chunk": 4096}),
    ("max-f64-rows16", tiny_max_config, "f64", {"proj_rows": 16, "vec_chunk": 1024}),
    ("c2-f32-rows32", WL.config_c2, "f32", {"proj_rows": 32, "adj_lds": 64 * 1024}),
    ("c2-f64-rows48", WL.config_c2, "f64", {"proj_rows": 48}),
    ("max-f64-rows48", tiny_max_config, "f64", {"proj_rows": 48}),
    # footprints at the layer edges, read through windows that wrap around them
    ("edge-tiled-f64", tiny_edge_config, "f64", {"tile": 16, "lds_budget": 512}),
    ("edge-tiled-f32-op32", tiny_edge_config, "f32", {"tile": 16, "lds_budget": 256, "op_precision": 32}),
]

_cache = {}


def _get(name, builder):
    if name not in _cache:
        cfg = builder()
        _cache.clear()
        _cache[name] = (cfg,) + setup(cfg)
    return _cache[name]


@pytest.mark.parametrize("name,builder,dt,kw", CASES, ids=[c[0] for c in CASES])
def test_operator_stages(name, builder, dt, kw):
    require_gpu()
    from paper_1302_3734_amd import Plan
    key = name.split("-")[0]
    cfg, S, sig, s, truth = _get(key, builder)
    tol = TOL[dt]
    tdt = _torch_dtype(dt)
    say(f"[{name}] plan")
    plan = Plan(cfg, sig, dtype=dt, max_batch=2, **kw)
    assert plan.n == S.n and plan.n_slopes == S.n_slopes
    assert list(plan.slope_offsets) == list(S.slope_off)
    rng = np.random.default_rng(1)
    c = rng.standard_normal((2, S.n))

    say(f"[{name}] W^-1")
    lay = to_np(plan.coeffs_to_layers(to_dev(c, tdt))).reshape(2, -1)
    for f in range(2):
        ref = S.join(S.to_layers(c[f]))
        assert maxrel(lay[f], ref) < tol, (f, maxrel(lay[f], ref))

    say(f"[{name}] W")
    pix = rng.standard_normal((2, S.n))
    co = to_np(plan.layers_to_coeffs(to_dev(pix, tdt))).reshape(2, -1)
    for f in range(2):
        ref = S.to_coeffs(S.split(pix[f]))
        assert maxrel(co[f], ref) < tol

    say(f"[{name}] W W^-1 = I")
    rt = to_np(plan.layers_to_coeffs(plan.coeffs_to_layers(to_dev(c, tdt)))).reshape(2, -1)
    assert maxrel(rt, c) < (1e-12 if dt == "f64" else 1e-5)

    say(f"[{name}] forward")
    layers = S.join(truth)
    fw = to_np(plan.forward_layers(to_dev(layers[None, :], tdt))).ravel()
    assert maxrel(fw, S.forward_layers(truth)) < tol

    say(f"[{name}] rhs")
    b = to_np(plan.rhs(to_dev(s[None, :], tdt))).ravel()
    b_ref = S.rhs(s)
    assert rel(b, b_ref) < tol and maxrel(b, b_ref) < 10 * tol

    say(f"[{name}] apply_A")
    y = to_np(plan.apply_A(to_dev(c, tdt))).reshape(2, -1)
    for f in range(2):
        ref = S.apply_A(c[f])
        assert rel(y[f], ref) < tol, (f, rel(y[f], ref))
        assert maxrel(y[f], ref) < 10 * tol

    say(f"[{name}] jacobi")
    J = to_np(plan.precond_diag())
    J_ref = S.jacobi_separable()
    assert np.max(np.abs(J - J_ref) / J_ref) < 1e-12
    plan.close()
    say(f"[{name}] ok")


def test_adjoint_identities_on_device():
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    cfg = tiny_ragged_config()
    S, sig, s, truth = setup(cfg)
    plan = Plan(cfg, sig, dtype="f64", max_batch=1, tile=16, lds_budget=1024)
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.standard_normal((1, S.n)), device="cuda")
    y = torch.tensor(rng.standard_normal((1, S.n)), device="cuda")
    w = torch.tensor(rng.standard_normal((1, S.n_slopes)), device="cuda")
    # <W^-1 x, y> = <x, W y>
    lhs = float((plan.coeffs_to_layers(x) * y).sum())
    rhs = float((x * plan.layers_to_coeffs(y)).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # A symmetric: <x, A y> = <A x, y>
    lhs = float((x * plan.apply_A(y)).sum())
    rhs = float((plan.apply_A(x) * y).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # rhs is the adjoint of the forward model composed with the noise weight
    # on sensors without tip/tilt removal: check <rhs(w), x> = <C^-1 w, G P W^-1 x>
    lhs = float((plan.rhs(w) * x).sum())
    fwd = plan.forward_layers(plan.coeffs_to_layers(x))
    rhs = float(np.dot(S.weight(w.cpu().numpy().ravel()), fwd.cpu().numpy().ravel()))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    plan.close()
