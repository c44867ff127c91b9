"""The allocation-free solve (wmcao_solve_noalloc): the same PCG solve as
wmcao_solve with every scratch buffer in the library's fixed device array,
called through the C ABI.  Its results equal wmcao_solve's bit for bit, on two
calls in a row (the second with fewer frames, so the array still holds the
first call's contents), and a batch beyond the array's size is rejected on the
host before any launch."""
import ctypes as C

import numpy as np
import pytest

import workloads as WL
from tests.gpu_common import require_gpu, say, setup, slopes_for, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(plan, slopes, x, batch, n_iter, warm, resid=None, status=None):
    from paper_1302_3734_amd import _abi
    from paper_1302_3734_amd.plan import _stream_ptr
    lib = _abi.lib()
    return lib.wmcao_solve_noalloc(plan.handle, C.c_void_p(slopes.data_ptr()),
                                   C.c_void_p(x.data_ptr()), batch, n_iter, int(warm),
                                   C.c_void_p(resid.data_ptr() if resid is not None else 0),
                                   C.c_void_p(status.data_ptr() if status is not None else 0),
                                   _stream_ptr())


@pytest.mark.parametrize("name,dt,batches,kw", [("C1", "f32", (16, 5), {}), ("C1", "f64", (8, 3), {}),
                                                 ("C2", "f32", (2, 1), {}),
                                                 # projection and weighting items of different sizes
                                                 ("C2", "f32", (2, 1), {"proj_rows": 16})],
                         ids=["C1-f32", "C1-f64", "C2-f32", "C2-f32-rows16"])
def test_noalloc_solve_equals_solve(name, dt, batches, kw):
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    cfg = WL.config_by_name(name)
    S, sig, s0, _ = setup(cfg, frame=0, seed_frame=0)
    tdt = torch.float32 if dt == "f32" else torch.float64
    B = batches[0]
    sl = to_dev(np.stack([slopes_for(S, cfg, sig, 1 + f, seed_frame=0) for f in range(B)]), tdt)
    plan = Plan(cfg, sig, dtype=dt, max_batch=B, **kw)
    gen = torch.Generator(device="cuda").manual_seed(3)
    x0 = torch.randn(B, plan.n, dtype=tdt, device="cuda", generator=gen) * 0.01
    n_it = 6
    for call, b in enumerate(batches):
        say(f"[noalloc] {name} {dt} call {call}: {b} frames")
        ref = x0[:b].clone()
        res_ref = torch.zeros(b, n_it + 1, dtype=torch.float64, device="cuda")
        plan.solve(sl[:b].contiguous(), ref, n_iter=n_it, warm_start=True, resid=res_ref)
        x = x0[:b].clone()
        res = torch.zeros(b, n_it + 1, dtype=torch.float64, device="cuda")
        st = torch.full((b,), 99, dtype=torch.int32, device="cuda")
        rc = _noalloc(plan, sl[:b].contiguous(), x, b, n_it, True, res, st)
        assert rc == 0, rc
        torch.cuda.synchronize()
        assert torch.equal(x, ref), (name, dt, call)
        assert torch.equal(res, res_ref), (name, dt, call)
        assert int(st.max()) == 0 and int(st.min()) == 0
        # cold start, no optional outputs
        xc = torch.full_like(x, 3.0)
        assert _noalloc(plan, sl[:b].contiguous(), xc, b, n_it, False) == 0
        refc = plan.solve(sl[:b].contiguous(), n_iter=n_it)
        torch.cuda.synchronize()
        assert torch.equal(xc, refc)
    plan.close()


def test_noalloc_rejects_batches_beyond_its_scratch():
    """Eight E-ELT frames need more than the fixed scratch: rejected with
    WMCAO_ERR_SIZE, and the output is untouched."""
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan, _abi
    cfg = WL.config_c2()
    sig = [0.2] * 6 + [0.02, 0.006, 0.004]
    plan = Plan(cfg, sig, dtype="f32", max_batch=8)
    sl = torch.zeros(8, plan.n_slopes, dtype=torch.float32, device="cuda")
    x = torch.full((8, plan.n), 0.5, dtype=torch.float32, device="cuda")
    rc = _noalloc(plan, sl, x, 8, 4, True)
    assert rc == -2, rc                                  # WMCAO_ERR_SIZE
    assert "scratch" in _abi.lib().wmcao_last_error().decode()
    torch.cuda.synchronize()
    assert torch.all(x == 0.5)
    plan.close()
