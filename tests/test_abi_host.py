"""The C-ABI library loads, exports every function its header declares, and
rejects invalid plans on the host before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1302_3734_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "wmcao.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(wmcao_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_abi.EXPORTED)


def test_strerror_and_last_error():
    L = _abi.lib()
    assert L.wmcao_strerror(0) == b"ok"
    assert b"footprint" in L.wmcao_strerror(-3) or b"outside" in L.wmcao_strerror(-3)
    assert isinstance(L.wmcao_last_error(), bytes)


def _args(n=64, levels=4, order=3, n_sub=16, agg=0, dtype=0, tile=0, sigma=0.1, streams=0, **opt):
    Ls = (_abi.Layer * 1)(_abi.Layer(0.0, 1.0, 0.5, n))
    Ws = (_abi.Wfs * 1)(_abi.Wfs(0, 0.0, 0.0, 90e3, n_sub, agg, -1, -1, sigma, None, 0))
    pupil = _abi.Pupil(8.0, 0.0)
    opts = _abi.Options(1.0, 0.15, 25.0, dtype, 1, 0, 1, tile, 0, streams)
    opts.op_fp64_stages = -1
    for k, v in opt.items():
        setattr(opts, k, v)
    return pupil, Ls, Ws, _abi.Wavelet(0, order), levels, opts


@pytest.mark.parametrize("kw,code", [
    ({"n": 60}, -2),                 # 60 not divisible by 2^4
    ({"n": 32, "levels": 4}, -2),    # coarsest transform length 4 < 6
    ({"order": 4}, -4),              # only db3 is built
    ({"n_sub": 200}, -4),            # sensor too large
    ({"agg": 3}, -1),                # 3 does not divide 16
    ({"dtype": 7}, -1),
    ({"tile": 48}, -1),
    ({"sigma": 0.0}, -1),
    ({"streams": 5}, -1),            # one to four concurrent parts
    ({"streams": -1}, -1),
    ({"op_precision": 16}, -1),      # operators are FP32 or FP64
    ({"dtype": 1, "op_precision": 32}, -1),
    ({"op_fp64_stages": 9}, -1),     # a mask of 1, 2 and 4
    ({"proj_rows": 3}, -1),           # 4 .. 48 node rows
    ({"proj_rows": 64}, -1),
    ({"vec_chunk": 3000}, -1),
    ({"adj_lds": 1024}, -1),
])
def test_invalid_plans_rejected_on_host(kw, code):
    L = _abi.lib()
    pupil, Ls, Ws, wav, levels, opts = _args(**kw)
    h = C.c_void_p()
    rc = L.wmcao_plan(C.byref(pupil), Ls, 1, Ws, 1, wav, levels, C.byref(opts), C.byref(h))
    assert rc == code, (rc, L.wmcao_last_error())
    assert not h.value
    assert L.wmcao_last_error()


def test_layer_and_sensor_limits_rejected_on_host():
    """17 layers or 33 sensors exceed the plan's tables (16 and 32)."""
    L = _abi.lib()
    pupil, _, Ws, wav, levels, opts = _args()
    h = C.c_void_p()
    Ls17 = (_abi.Layer * 17)(*[_abi.Layer(500.0 * k, 1.0 / 17, 0.5, 64) for k in range(17)])
    assert L.wmcao_plan(C.byref(pupil), Ls17, 17, Ws, 1, wav, levels, C.byref(opts), C.byref(h)) == -1
    assert not h.value
    pupil, Ls, _, wav, levels, opts = _args()
    Ws33 = (_abi.Wfs * 33)(*[_abi.Wfs(0, 0.0, 0.0, 90e3, 16, 0, -1, -1, 0.1, None, 0) for _ in range(33)])
    assert L.wmcao_plan(C.byref(pupil), Ls, 1, Ws33, 33, wav, levels, C.byref(opts), C.byref(h)) == -1
    assert not h.value


def test_null_arguments_rejected():
    L = _abi.lib()
    assert L.wmcao_solve(None, None, None, 1, 1, 0, None, None, None) == -1
    assert L.wmcao_apply_A(None, None, None, 1, None) == -1
    assert L.wmcao_serve_launch(None, None, None, 1, None, None, 0, None, None, 1, None) == -1
    assert L.wmcao_sizes(None, None, None, None, None) == -1
    L.wmcao_plan_destroy(None)


def test_every_autotuner_candidate_passes_option_checks():
    """Each work shape the autotuner may try is one the plan accepts: option
    checks run on the host before the device is touched, so without a GPU a
    valid plan stops at the device (no HIP device), never at an option."""
    from paper_1302_3734_amd import autotune
    L = _abi.lib()
    for name, cands in autotune.SPACE.items():
        for v in cands:
            pupil, Ls, Ws, wav, levels, opts = _args(**{name: v})
            h = C.c_void_p()
            rc = L.wmcao_plan(C.byref(pupil), Ls, 1, Ws, 1, wav, levels, C.byref(opts), C.byref(h))
            if rc == 0:
                L.wmcao_plan_destroy(h)
            assert rc != -1, (name, v, L.wmcao_last_error())
