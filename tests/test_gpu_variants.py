"""GPU parity of the paper's variants against the FP64 oracle, through the C
ABI: laser spot elongation (Sec. 4.3, eq. (16)) with tau = 0.8 through the 2x2
noise blocks; the accelerated 3-layers-at-DM-altitudes PCG with 4 iterations
(Sec. 5.3); the 9-layer plain CG with 10 iterations (Sec. 5.2)."""
import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests.gpu_common import rel, require_gpu, say, setup, slopes_for, to_dev, to_np

pytestmark = pytest.mark.gpu


def _blocks(cfg, sig):
    from workloads.elongation import elongation_blocks
    cinv = []
    for m, w in enumerate(cfg["wfs"]):
        cinv.append(elongation_blocks(cfg, m, sig[m], tau=0.8)[1] if w["lgs"] else None)
    return cinv


def test_elongation_blocks_apply_and_solve():
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    cfg = WL.config_c2()
    S0, sig, s, _ = setup(cfg)
    cinv = _blocks(cfg, sig)
    S = O.System(cfg, sig, cinv_blocks=cinv)
    plan = Plan(cfg, sig, dtype="f64", max_batch=1, cinv_blocks=cinv)
    J = to_np(plan.precond_diag())
    J_ref = S.jacobi_separable()
    assert np.max(np.abs(J - J_ref) / J_ref) < 1e-12
    c = np.random.default_rng(2).standard_normal(S.n)
    y = to_np(plan.apply_A(to_dev(c[None], torch.float64))).ravel()
    assert rel(y, S.apply_A(c)) < 1e-12
    b = S.rhs(s)
    x_ref, _ = O.pcg(S.apply_A, b, 8, jacobi=J_ref)
    x = to_np(plan.solve(to_dev(s[None], torch.float64), n_iter=8)).ravel()
    say(f"[elongation] e_x {rel(x, x_ref):.2e}")
    assert rel(x, x_ref) < 1e-11
    plan.close()


@pytest.mark.parametrize("name", ["C2-dm3", "C2-cg9"])
def test_paper_variants_fp64(name):
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    cfg = WL.config_by_name(name)
    precond = cfg.get("precond", True)
    S, sig, s0, _ = setup(cfg, frame=0, seed_frame=0)
    J = S.jacobi_separable() if precond else None
    x0, _ = O.pcg(S.apply_A, S.rhs(s0), 20, jacobi=J)
    s1 = slopes_for(S, cfg, sig, 1, seed_frame=0)
    b = S.rhs(s1)
    x_ref, _ = O.pcg(S.apply_A, b, cfg["n_iter"], x0=x0, jacobi=J)
    plan = Plan(cfg, sig, dtype="f64", max_batch=1, precond=precond)
    xt = to_dev(x0[None], torch.float64)
    plan.solve(to_dev(s1[None], torch.float64), xt, n_iter=cfg["n_iter"], warm_start=True)
    e = rel(to_np(xt).ravel(), x_ref)
    say(f"[{name}] e_x {e:.2e}")
    assert e < 1e-11
    plan.close()
