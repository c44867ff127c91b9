"""Served stream with continuous batching: every frame's result equals the same
frame solved alone (same warm start, same slopes), bitwise; every request
completes; latencies are recorded."""
import time

import numpy as np
import pytest

import workloads as WL
from tests.gpu_common import require_gpu, say, setup, slopes_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lanes", [2, 1], ids=["lane-per-config", "one-packed-lane"])
def test_served_mix_equals_alone(lanes):
    """lanes=1 packs both configurations into one lane, so launches capture
    new multi-plan graphs while frames are in flight."""
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    from paper_1302_3734_amd.serve import Server
    c1 = WL.config_c1()
    c8 = [c for c in WL.config_c4_classes() if c["name"] == "C4-8m-lgs"][0]
    cfgs, pools = {}, {}
    for cfg in (c1, c8):
        S, sig, s, _ = setup(cfg)
        cfgs[cfg["name"]] = (cfg, sig)
        pools[cfg["name"]] = [torch.tensor(slopes_for(S, cfg, sig, f), dtype=torch.float32,
                                           device="cuda") for f in range(6)]
    streams = {"a": "C1", "b": "C1", "c": "C4-8m-lgs"}
    srv = Server(cfgs, streams, dtype="f32", n_iter=6, hip_streams=lanes, keep_inputs=True)
    futs = []
    say("[serve] submitting")
    for f in range(6):
        for st, c in streams.items():
            futs.append((st, c, f, srv.submit(st, pools[c][(f + ord(st)) % 6])))
        time.sleep(0.0005 * (f % 3))
    results = [(st, c, f, fu.result(timeout=60)) for st, c, f, fu in futs]
    srv.close()
    lat = srv.latencies_ms()
    say(f"[serve] {len(lat)} frames, {srv.launches} launches, "
        f"frames/launch {np.mean(srv.frames_in_launch):.2f}, p50 {np.median(lat):.3f} ms")
    assert len(lat) == len(futs)
    assert max(srv.frames_in_launch) >= 2          # frames were packed together
    alone = {c: Plan(cfg, sig, dtype="f32", max_batch=1) for c, (cfg, sig) in cfgs.items()}
    for st, c, f, (x, x0) in results:
        xs = x0.clone()
        alone[c].solve(pools[c][(f + ord(st)) % 6].reshape(1, -1), xs, n_iter=6, warm_start=True)
        torch.cuda.synchronize()
        assert torch.equal(xs, x), (st, f)
    for p in alone.values():
        p.close()


def test_served_slots_equal_alone():
    """Two lanes per configuration (slots=2, one launch each in flight): a
    frame that arrives while its predecessor is being solved starts at once
    on the free lane from the newest result already complete.  Both lanes of
    every configuration are used, every request completes, and every frame
    equals the same frame solved alone from the warm start it was given,
    bitwise."""
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    from paper_1302_3734_amd.serve import Server
    c1 = WL.config_c1()
    c8 = [c for c in WL.config_c4_classes() if c["name"] == "C4-8m-lgs"][0]
    cfgs, pools = {}, {}
    for cfg in (c1, c8):
        S, sig, s, _ = setup(cfg)
        cfgs[cfg["name"]] = (cfg, sig)
        pools[cfg["name"]] = [torch.tensor(slopes_for(S, cfg, sig, f), dtype=torch.float32,
                                           device="cuda") for f in range(6)]
    streams = {"a": "C1", "b": "C4-8m-lgs"}
    srv = Server(cfgs, streams, dtype="f32", n_iter=6, keep_inputs=True, slots=2, depth=1,
                 max_frames=2)
    futs = []
    say("[serve-slots] submitting")
    for f in range(12):
        for st, c in streams.items():
            futs.append((st, c, f, srv.submit(st, pools[c][f % 6])))
        time.sleep(0.0002 * (f % 4))
    results = [(st, c, f, fu.result(timeout=60)) for st, c, f, fu in futs]
    srv.close()
    say(f"[serve-slots] {len(results)} frames, launches per lane {srv.lane_launches}")
    assert len(srv.records) == len(futs)
    assert min(srv.lane_launches) > 0, srv.lane_launches
    alone = {c: Plan(cfg, sig, dtype="f32", max_batch=1) for c, (cfg, sig) in cfgs.items()}
    for st, c, f, (x, x0) in results:
        xs = x0.clone()
        alone[c].solve(pools[c][f % 6].reshape(1, -1), xs, n_iter=6, warm_start=True)
        torch.cuda.synchronize()
        assert torch.equal(xs, x), (st, f)
    for p in alone.values():
        p.close()


def test_failed_launch_resolves_its_futures():
    """A launch that raises hands the error to its frames' futures; later
    frames are still served.  A frame of the wrong size is refused at
    submission."""
    require_gpu()
    import torch
    from paper_1302_3734_amd.serve import Server
    cfg = WL.config_c1()
    S, sig, s, _ = setup(cfg)
    sl = torch.tensor(s, dtype=torch.float32, device="cuda")

    class Boom(RuntimeError):
        pass

    srv = Server({"C1": (cfg, sig)}, {"a": "C1"}, dtype="f32", n_iter=4, depth=1, max_frames=1)
    with pytest.raises(ValueError):
        srv.submit("a", sl[:-1])
    launch = srv._launch
    calls = []

    def flaky(lane, groups):
        calls.append(lane)
        if len(calls) == 2:
            raise Boom("injected")
        return launch(lane, groups)

    srv._launch = flaky
    futs = []
    for _ in range(4):
        futs.append(srv.submit("a", sl))
        futs[-1].exception(timeout=60)   # one frame at a time: the second launch is the failing one
    srv.close()
    outcomes = [type(f.exception()) for f in futs]
    assert outcomes == [type(None), Boom, type(None), type(None)], outcomes
    assert srv.failed == 1 and len(srv.records) == 3


def test_budget_queues_frames():
    """A budget that fits one frame at a time serialises the streams but
    every request still completes."""
    require_gpu()
    import torch
    from paper_1302_3734_amd.serve import Server
    cfg = WL.config_c1()
    S, sig, s, _ = setup(cfg)
    sl = torch.tensor(s, dtype=torch.float32, device="cuda")
    srv = Server({"C1": (cfg, sig)}, {"a": "C1", "b": "C1"}, dtype="f32", n_iter=4,
                 hbm_budget=1)
    srv.hbm_budget = srv.frame_bytes["C1"]           # room for exactly one frame
    futs = [srv.submit(st, sl) for st in ("a", "b") for _ in range(3)]
    for fu in futs:
        fu.result(timeout=60)
    srv.close()
    assert max(srv.frames_in_launch) == 1 and len(srv.records) == 6


def test_served_c5_geometries_equal_alone_and_match_oracle():
    """The served stream's four telescope configurations (8 m and 16 m
    NGS-only, 39 m and 42 m LGS-only), one telescope stream each, with the two
    E-ELT-class configurations sharing one lane: every served frame equals
    the same frame solved alone from the same warm start, bitwise, and the
    newest frame of every stream matches the FP64 oracle's PCG from that warm
    start (FP32 bar)."""
    require_gpu()
    import torch
    from paper_1302_3734_amd import Plan
    from paper_1302_3734_amd.serve import Server
    from tests import oracle_jobs
    from tests.gpu_common import oracle_pool_map, record
    names = ["C4-8m-ngs", "C4-16m-ngs", "C4-39m-lgs", "C4-42m-lgs"]
    cfgs, pools = {}, {}
    n_frames = 4
    for nm in names:
        cfg = WL.config_by_name(nm)
        S, sig, s, _ = setup(cfg, frame=0, seed_frame=0)
        cfgs[nm] = (cfg, sig)
        sl = oracle_pool_map(oracle_jobs.slopes, [(nm, sig, f, 0) for f in range(1, n_frames + 1)])
        pools[nm] = [torch.tensor(v, dtype=torch.float32, device="cuda") for v in sl]
    streams = {nm: nm for nm in names}
    lanes = {"C4-8m-ngs": 0, "C4-16m-ngs": 1, "C4-39m-lgs": 2, "C4-42m-lgs": 2}
    srv = Server(cfgs, streams, dtype="f32", n_iter=10, keep_inputs=True, lane_map=lanes, max_frames=4)
    futs = []
    say("[serve-c5] submitting")
    for f in range(n_frames):
        for nm in names:
            futs.append((nm, f, srv.submit(nm, pools[nm][f])))
        time.sleep(0.001)
    results = [(nm, f, fu.result(timeout=120)) for nm, f, fu in futs]
    srv.close()
    say(f"[serve-c5] {len(results)} frames, {srv.launches} launches")
    alone = {nm: Plan(cfg, sig, dtype="f32", max_batch=1) for nm, (cfg, sig) in cfgs.items()}
    jobs = []
    for nm, f, (x, x0) in results:
        xs = x0.clone()
        alone[nm].solve(pools[nm][f].reshape(1, -1), xs, n_iter=10, warm_start=True)
        torch.cuda.synchronize()
        assert torch.equal(xs, x), (nm, f)
        if f == n_frames - 1:
            jobs.append((nm, cfgs[nm][1], pools[nm][f].double().cpu().numpy(),
                         x0.double().cpu().numpy().ravel(), x.double().cpu().numpy().ravel(), 10, "f32"))
    for p in alone.values():
        p.close()
    say("[serve-c5] oracle references")
    res = oracle_pool_map(oracle_jobs.check, jobs)
    for job, (e, bars) in zip(jobs, res):
        say(f"[serve-c5] {job[0]}: e {e} bars {bars}")
        record("served-" + job[0], "f32", e, bars)
        assert all(a < c for a, c in zip(e, bars)), (job[0], e, bars)
