#!/usr/bin/env python3
"""Benchmark of the wavelet-MCAO PCG solve at E-ELT scale on one MI355X.

Workload: the 42 m E-ELT configuration (6 sodium LGS with 84x84 Fried sensors
and cone effect, 3 tip/tilt NGS, 9 layers of 128..256 pixels, db3 with 5
levels, modified Jacobi PCG, 10 iterations, warm restart).  One step solves a
batch of B frames (B independent telescope streams, each warm-started from its
previous reconstruction) in FP32 with FP64 inner products and scalars; the
plan runs the batch as two concurrent halves on two HIP streams (its default
for batches this large; --streams 1 keeps one stream).  Inputs
are synthetic: seeded von Karman screens with frozen flow, slopes from the
library's forward model plus Gaussian noise at SNR 20.

Prints one JSON line: frames/s, p99 frame latency, the dominant kernel's
achieved HBM bandwidth against the MI355X peak (per-kernel times measured on
one stream, where a launch's event time is its own), the per-frame FP64 solve
as a comparison, and the CPU oracle on a bounded sample.
"""
import argparse
import gc
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_eelt_b32.txt")
TRAFFIC_FILE_B128 = os.path.join(ROOT, "profiles", "hbm_traffic_eelt_b128.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1302_3734_amd", "csrc", "wmcao_kernels.hip")
N_FRAMES_ROT = 4            # distinct frozen-flow frames per stream in rotation


# ----------------------------------------------------------------- CPU leg ----
def _cpu_worker(args):
    """Oracle on frames of one stream: rhs + 10 warm PCG iterations timed."""
    stream, frames, n_iter = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)                     # one core per worker process
    import oracle as O
    cfg = WL.config_c2()
    S0 = O.System(cfg, [1.0] * len(cfg["wfs"]))
    base = 1000 * stream
    truth0 = WL.layer_screens(cfg, base, seed_frame=base)
    sig = WL.sigmas_from_clean(cfg, S0.forward_layers(truth0), S0.slope_off)
    S = O.System(cfg, sig)
    J = S.jacobi_separable()
    spent = 0.0
    done = 0
    for t in range(1, frames + 1):
        prev = WL.layer_screens(cfg, base + t - 1, seed_frame=base)
        cur = WL.layer_screens(cfg, base + t, seed_frame=base)
        x0 = S.to_coeffs(prev)
        s = WL.noisy_slopes(S.forward_layers(cur), sig, S.slope_off,
                            WL.noise_draw(cfg["cfg_id"], base + t, S.n_slopes))
        t0 = time.perf_counter()
        b = S.rhs(s)
        O.pcg(S.apply_A, b, n_iter, x0=x0, jacobi=J)
        spent += time.perf_counter() - t0
        done += 1
    return done, spent


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workers, frames_per_worker, n_iter, single_frames=3):
    """The FP64 oracle on the host: one process with one thread, then one
    single-threaded process per core, each solving frames of its own stream."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(1) as pool:
        d1, s1 = pool.map(_cpu_worker, [(0, single_frames, n_iter)])[0]
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_cpu_worker, [(w, frames_per_worker, n_iter) for w in range(workers)])
    wall = time.perf_counter() - t0
    rate = sum(d / s for d, s in res)
    frames = sum(d for d, _ in res)
    return {"value": rate, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": d1 / s1, "unit": "frames/s", "cores": 1,
                              "sample": f"{d1} frames, one process, one thread"},
            "sample": f"{workers} single-threaded processes x {frames_per_worker} frames of the "
                      f"E-ELT workload ({frames} frames), FP64 NumPy oracle, right side + "
                      f"{n_iter} warm PCG iterations timed per frame; plan, Jacobi and input "
                      f"synthesis excluded; wall {wall:.1f} s"}


# ----------------------------------------------------------------- GPU leg ----
def pctl(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


SERVED = ["C4-8m-ngs", "C4-16m-ngs", "C4-39m-lgs", "C4-42m-lgs"]
# one lane per configuration: measured faster than packing the two E-ELT-class
# configurations into one lane (their launches overlap on two lanes)
SERVED_LANES = {"C4-8m-ngs": 0, "C4-16m-ngs": 1, "C4-39m-lgs": 2, "C4-42m-lgs": 3}
# two lanes per configuration, one launch in flight on each: measured p99
# 3.0-3.1 ms against 3.2-5.4 ms for one lane each with two in flight (and
# 3 lanes per configuration no better)
SERVED_SLOTS, SERVED_DEPTH = 2, 1


def served_stream(duration_s, rate_hz, n_iter, dtype="f32", plain=False, tuned=True,
                  slots=SERVED_SLOTS, depth=SERVED_DEPTH):
    """Poisson arrivals over four telescope configurations (8 m and 16 m
    NGS-only, 39 m and 42 m LGS-only), one stream each at rate_hz/4, served
    with continuous batching (`slots` lanes per configuration with `depth`
    launches in flight each, or with slots = 1 one lane per configuration;
    backlogs batched); frozen-flow frames from a pool of 8 per stream.  The
    same server runs in FP32 or FP64.  With plain, the arrivals are served the
    plain way instead: one frame per launch, one launch at a time (FP64).
    Returns latency percentiles and throughput."""
    import torch
    from paper_1302_3734_amd import Plan
    from paper_1302_3734_amd.serve import Server
    names = SERVED
    cfgs, pools = {}, {}
    for nm in names:
        cfg = WL.config_by_name(nm)
        fwd = Plan(cfg, [1.0] * len(cfg["wfs"]), dtype="f64", max_batch=1)
        so = fwd.slope_offsets
        lay = []
        for t in range(8):
            v = np.concatenate([a.ravel() for a in WL.layer_screens(cfg, t, seed_frame=0)])
            lay.append(fwd.forward_layers(torch.tensor(v, device="cuda")[None])[0])
        sig = WL.sigmas_from_clean(cfg, lay[0].cpu().numpy(), so)
        sv = torch.tensor(np.concatenate([np.full(so[m + 1] - so[m], sig[m])
                                          for m in range(len(sig))]), device="cuda")
        pools[nm] = [(lay[t] + sv * torch.tensor(WL.noise_draw(cfg["cfg_id"], t, fwd.n_slopes),
                                                 device="cuda")) for t in range(8)]
        if dtype == "f32":
            pools[nm] = [v.float() for v in pools[nm]]
        cfgs[nm] = (cfg, sig)
        fwd.close()
    if plain:
        srv = Server(cfgs, {nm: nm for nm in names}, dtype=dtype, n_iter=n_iter, hip_streams=1,
                     pack=False, depth=1, max_frames=1, tuned=tuned)
    elif slots != 1:
        srv = Server(cfgs, {nm: nm for nm in names}, dtype=dtype, n_iter=n_iter, slots=slots,
                     depth=depth, max_frames=4, tuned=tuned)
    else:
        srv = Server(cfgs, {nm: nm for nm in names}, dtype=dtype, n_iter=n_iter,
                     lane_map=SERVED_LANES, pack=True, depth=depth, max_frames=4, tuned=tuned)
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)       # hand the interpreter lock to the server threads promptly
    # no cyclic garbage collection while frames are served: its passes over the
    # growing records would stall the server threads for milliseconds
    gc.collect()
    gc.disable()
    arrivals = sorted((t, nm) for k, nm in enumerate(names)
                      for t in WL.poisson_arrivals(500 + k, rate_hz / len(names), duration_s))
    torch.cuda.synchronize()
    futs = []
    cnt = {nm: 0 for nm in names}
    t0 = time.perf_counter()
    for t, nm in arrivals:
        wait = t - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)          # releases the interpreter lock to the server threads
        futs.append(srv.submit(nm, pools[nm][cnt[nm] % 8]))
        cnt[nm] += 1
    for f in futs:
        f.result(timeout=120)
    elapsed = time.perf_counter() - t0
    gc.enable()
    sys.setswitchinterval(switch)
    srv.close()
    lat = srv.latencies_ms()
    wait, run = srv.waits_ms()
    per_cfg = {}
    for nm in names:
        lv = [1e3 * (r[3] - r[2]) for r in srv.records if r[0] == nm]
        per_cfg[nm] = {"p50_ms": round(pctl(lv, 0.5), 4), "p99_ms": round(pctl(lv, 0.99), 4)}
    lanes = (f"lanes per configuration {slots}" if slots != 1 else f"lanes {SERVED_LANES}")
    mode = ("plain FP64, one frame per launch, one launch at a time" if plain else
            f"{dtype.upper()} continuous batching: {lanes}, depth {depth}, up to 4 "
            f"frames per telescope stream per launch")
    return {"mode": mode, "configs": names, "rate_hz": rate_hz, "duration_s": duration_s,
            "frames": len(lat), "frames_per_s": round(len(lat) / elapsed, 1),
            "p50_frame_latency_ms": round(pctl(lat, 0.5), 4),
            "p99_frame_latency_ms": round(pctl(lat, 0.99), 4),
            "p99_queue_wait_ms": round(pctl(wait, 0.99), 4),
            "p50_launch_to_result_ms": round(pctl(run, 0.5), 4),
            "p99_launch_to_result_ms": round(pctl(run, 0.99), 4),
            "launches": srv.launches, "launches_per_lane": srv.lane_launches,
            "mean_frames_per_launch": round(float(np.mean(srv.frames_in_launch)), 3),
            "per_config": per_cfg, "work_shapes": srv.work_shapes}


# Stages of one operator apply and of the PCG updates, the library kernels
# (timing kinds) that carry them, and the elements each pass must move by the
# survey's algorithmic count (n unknowns, Q sensor nodes): W^-1 reads and
# writes n; the projection chain reads n and writes the Q node fields; P^T
# reads Q and writes n; W + alpha D reads the n-pixel P^T image and p, and
# writes n (the right side's pass: 2n); the updates move 7n (x, r and the
# inner products) + 4n (p) per iteration, and the initial residual 5n.
STAGES = [
    ("W^-1", ("idwt_coarse", "idwt_tile")),
    ("P, Gamma, C^-1, Gamma^T", ("project", "weights")),
    ("P^T", ("adjoint",)),
    ("W + alpha D", ("fdwt_tile", "fdwt_coarse")),
    ("PCG updates", ("init", "update_r", "update_p", "replace_r")),
]


def stage_elements(n, Q, steps, iters):
    """Algorithmic elements moved by each stage over `steps` warm solves of
    `iters` iterations (per frame): each solve is one right side, one apply
    for the warm start's residual and one apply per iteration."""
    applies, rhs = steps * (1 + iters), steps
    return {"W^-1": applies * 2 * n,
            "P, Gamma, C^-1, Gamma^T": applies * (n + Q),
            "P^T": (applies + rhs) * (Q + n),
            "W + alpha D": applies * 3 * n + rhs * 2 * n,
            "PCG updates": steps * (iters * 11 * n + 5 * n)}


def stage_table(prof, n, Q, steps, iters, B, traffic_file, esz=4):
    """Per-stage times, launches and achieved GB/s by the algorithmic bytes of
    `steps` solves of B frames (profile_read output of those steps), and the
    per-kernel averages."""
    elems = stage_elements(n, Q, steps, iters)
    stages = {}
    for name, ks in STAGES:
        ms = sum(prof[k][0] for k in ks)
        launches = sum(prof[k][1] for k in ks)
        if not launches:
            continue
        abytes = elems[name] * esz * B                      # over the profiled window
        design = sum(prof[k][2] for k in ks)
        stages[name] = {"kernels": list(ks), "ms": round(ms, 4), "launches": launches,
                        "avg_launch_us": round(1e3 * ms / launches, 3),
                        "bytes_per_launch": round(abytes / launches),
                        "achieved_gbs": round(abytes / (ms / 1e3) / 1e9, 1),
                        "frac": round(abytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "design_bytes_per_launch": round(design / launches),
                        "traffic_per_launch": measured_traffic(prof, ks, traffic_file)}
    tot_ms = sum(v[0] for v in prof.values())
    kernels = {k: {"avg_us": round(1e3 * v[0] / v[1], 3), "launches": v[1],
                   "share": round(v[0] / tot_ms, 4)}
               for k, v in prof.items() if v[1]}
    return stages, kernels


def measured_traffic(prof, kernels, traffic_file=None):
    """HBM bytes per launch of a group of library kernels from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE per dispatch, each scaled by its
    copy-kernel calibration factor), weighted by the launches of each kernel
    in `prof`; None if there is no summary, a kernel is missing from it or the
    kernel source has changed since the counters were taken."""
    import hashlib
    try:
        lines = open(traffic_file or TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    meta, rows = {}, {}
    for ln in lines:
        if ln.startswith("#") and ":" in ln:
            k, v = ln[1:].split(":", 1)
            meta[k.strip()] = v.strip()
        elif ln and not ln.startswith("#"):
            f = ln.split()
            if len(f) >= 3 and f[0].startswith("k_"):
                rows[f[0]] = (float(f[1]), float(f[2]))
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if meta.get("kernel source sha256") != src:
        return None
    ff = float(meta.get("fetch calibration factor", "nan"))
    fw = float(meta.get("write calibration factor", "nan"))
    tot, cnt = 0.0, 0
    for k in kernels:
        launches = prof[k][1]
        if not launches:
            continue
        if "k_" + k not in rows:
            return None
        fetch, write = rows["k_" + k]
        tot += 1024.0 * (fetch * ff + write * fw) * launches
        cnt += launches
    if not cnt or not math.isfinite(tot):
        return None
    return round(tot / cnt)


def n_nodes(cfg):
    return sum((w["n_sub"] + 1) ** 2 for w in cfg["wfs"])


def _synthetic_slopes(cfg, plan, frames, seeds=None, sig=None):
    """Seeded screens through the library's forward model plus noise at the
    configuration's level: [len(frames), n_slopes] FP64 on the device.  With
    seeds, frame frames[i] is advanced by frozen flow from frame seeds[i];
    otherwise every frame has screens of its own.  sig: noise levels (default:
    from the first frame's clean slopes)."""
    import torch
    out = []
    so = plan.slope_offsets
    sv = None
    if sig is not None:
        sv = torch.tensor(np.concatenate([np.full(so[m + 1] - so[m], sig[m])
                                          for m in range(len(sig))]), device="cuda")
    for i, t in enumerate(frames):
        sd = None if seeds is None else seeds[i]
        v = np.concatenate([a.ravel() for a in WL.layer_screens(cfg, t, seed_frame=sd)])
        clean = plan.forward_layers(torch.tensor(v, device="cuda")[None])[0]
        if sig is None:
            sig = WL.sigmas_from_clean(cfg, clean.cpu().numpy(), so)
            sv = torch.tensor(np.concatenate([np.full(so[m + 1] - so[m], sig[m])
                                              for m in range(len(sig))]), device="cuda")
        noise = torch.tensor(WL.noise_draw(cfg["cfg_id"], t, plan.n_slopes), device="cuda")
        out.append(clean + sv * noise)
    return torch.stack(out), sig


def batched_small(n_frames=128, n_iter=10, reps=20, tuned=True):
    """C3: independent 8 m frames (own seeded screens and noise) in one FP32
    batched solve replayed as a HIP graph, with the work shapes the
    autotuner picks for this batch."""
    import torch
    from paper_1302_3734_amd import Plan, autotune
    cfg = WL.config_c1()
    fwd = Plan(cfg, [1.0] * len(cfg["wfs"]), dtype="f64", max_batch=1)
    sl, sig = _synthetic_slopes(cfg, fwd, range(n_frames))
    fwd.close()
    shapes = autotune.tune(cfg, sig, "f32", n_frames, n_iter) if tuned else dict(autotune.DEFAULTS)
    plan = Plan(cfg, sig, dtype="f32", max_batch=n_frames, **shapes)
    s32 = sl.float().contiguous()
    x = torch.zeros(n_frames, plan.n, dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(3):
            plan.solve(s32, x, n_iter=n_iter, graph=True, stream=st)
    st.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        with torch.cuda.stream(st):
            plan.solve(s32, x, n_iter=n_iter, graph=True, stream=st)
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    plan.close()
    ms = statistics.median(ts)
    return {"workload": "8 m, 3 NGS 16x16, 3 layers 64 px, db3 4 levels, 10 its from zero",
            "frames_per_launch": n_frames, "ms_per_launch": round(ms, 4),
            "frames_per_s": round(n_frames / ms * 1e3, 1), "mode": "FP32, hipGraph replay",
            "work_shapes": shapes}


def mixed_batch(n_frames=64, n_iter=10, reps=10):
    """C4: frames drawn uniformly from eight telescope classes, all packed into
    one multi-plan solve (warm start) replayed as a HIP graph."""
    import torch
    from paper_1302_3734_amd import Plan, solve_multi
    classes = WL.config_c4_classes()
    pick = np.random.default_rng(np.random.SeedSequence([4, 0, 4])).integers(0, len(classes), n_frames)
    counts = [int((pick == k).sum()) for k in range(len(classes))]
    plans, slopes, coeffs = [], [], []
    for k, cfg in enumerate(classes):
        if counts[k] == 0:
            continue
        fwd = Plan(cfg, [1.0] * len(cfg["wfs"]), dtype="f64", max_batch=1)
        sl, sig = _synthetic_slopes(cfg, fwd, range(counts[k]))
        fwd.close()
        p = Plan(cfg, sig, dtype="f32", max_batch=counts[k])
        plans.append(p)
        slopes.append(sl.float().contiguous())
        coeffs.append(torch.zeros(counts[k], p.n, dtype=torch.float32, device="cuda"))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(3):
            solve_multi(plans, slopes, coeffs, n_iter=n_iter, warm_start=True, graph=True)
    st.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        with torch.cuda.stream(st):
            solve_multi(plans, slopes, coeffs, n_iter=n_iter, warm_start=True, graph=True)
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    for p in plans:
        p.close()
    ms = statistics.median(ts)
    return {"workload": "8 classes {8, 16, 39, 42 m} x {LGS-only, NGS-only}, FP32, 10 warm its",
            "frames_per_launch": n_frames, "counts": counts, "ms_per_launch": round(ms, 4),
            "frames_per_s": round(n_frames / ms * 1e3, 1), "mode": "one packed launch, hipGraph replay"}


def onaxis_wavefront(cfg, layers_vec, n_sub=84):
    """On-axis wavefront at the pupil nodes of an 84x84 grid (rad at 500 nm)
    and the mask of nodes inside the annular pupil.  At zero field angle the
    0.5 m nodes coincide with 0.5 m layer pixels of every layer, so the
    wavefront is a plain sum of layer samples."""
    D, eps = cfg["diameter"], cfg["obstruction"]
    d = D / n_sub
    c = (np.arange(n_sub) + 0.5 - n_sub / 2.0) * d
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    act = (r2 <= (D / 2) ** 2) & (r2 >= (eps * D / 2) ** 2)
    nodes = np.zeros((n_sub + 1, n_sub + 1), bool)
    for di in (0, 1):
        for dj in (0, 1):
            nodes[di:di + n_sub, dj:dj + n_sub] |= act
    vec = np.asarray(layers_vec, dtype=np.float64)
    w = np.zeros((n_sub + 1, n_sub + 1))
    off = 0
    for L in cfg["layers"]:
        N = L["n"]
        lay = vec[off:off + N * N].reshape(N, N)
        o = N // 2 - n_sub // 2
        w += lay[o:o + n_sub + 1, o:o + n_sub + 1]
        off += N * N
    return w, nodes


def onaxis_residual(cfg, layers_vec, truth_vec, truth_cfg=None):
    """On-axis wavefront residual (rad RMS at 500 nm, piston removed) over the
    pupil nodes, and its Marechal Strehl in K band (2.2 um).  The truth may
    live on another layer set (truth_cfg)."""
    w, nodes = onaxis_wavefront(cfg, layers_vec)
    wt, _ = onaxis_wavefront(truth_cfg or cfg, truth_vec)
    v = (w - wt)[nodes]
    v = v - v.mean()
    rms = float(np.sqrt(np.mean(v ** 2)))
    return rms, float(np.exp(-(rms * 0.5 / 2.2) ** 2))


def large_batch(cfg, sig, slopes32, shapes, n_iter=10, frames=128, steps=8):
    """Measurement only: `frames` E-ELT frames per FP32 solve (about 1.5 GB
    live, far beyond the 256 MB Infinity Cache), one stream, so that HBM
    bandwidth figures rest on traffic that cannot stay in the cache.  The
    inputs repeat the batch-32 frames.  Returns frames/s and the per-stage
    table."""
    import torch
    from paper_1302_3734_amd import Plan
    nrot, b0 = slopes32.shape[0], slopes32.shape[1]
    sl = [slopes32[t].repeat((frames + b0 - 1) // b0, 1)[:frames].contiguous() for t in range(nrot)]
    plan = Plan(cfg, sig, dtype="f32", max_batch=frames, streams=1, **shapes)
    X = torch.zeros(frames, plan.n, dtype=torch.float32, device="cuda")
    plan.solve(sl[0], X, n_iter=30)
    for i in range(2):
        plan.solve(sl[1 + i % (nrot - 1)], X, n_iter=n_iter, warm_start=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        plan.solve(sl[1 + i % (nrot - 1)], X, n_iter=n_iter, warm_start=True)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    plan.profile(True)
    for i in range(3):
        plan.solve(sl[1 + i % (nrot - 1)], X, n_iter=n_iter, warm_start=True)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    stages, kernels = stage_table(prof, plan.n, n_nodes(cfg), 3, n_iter, frames, TRAFFIC_FILE_B128)
    plan.close()
    return {"workload": f"{frames} E-ELT frames per solve, FP32, 10 warm its, one stream "
                        "(measurement only)",
            "ms_per_solve": round(ms, 4), "frames_per_s": round(frames / ms * 1e3, 1),
            "work_shapes": shapes, "stages": stages, "kernels": kernels}


def control_loop(cfg, sig, slopes, steps=20, warmup=3):
    """The paper's closed loop at E-ELT scale (Sec. 4.2, Alg. 4.1): one
    pseudo-open-loop control step per frame (open-loop slopes through the
    mirror-to-slope map, tomography by 10 warm PCG iterations, W^-1, fitting
    of the three mirrors over 25 directions by 4 warm CG iterations, the
    integrator), single frames as they arrive, FP32 and FP64.  Times per step
    from HIP events; the loop starts from zero commands and is fed the
    benchmark's frozen-flow slopes of one telescope stream."""
    import torch
    from paper_1302_3734_amd.fitting import PolcController
    from workloads.fitting import fitting_systems, mirror_wfs_system
    atm, dm = fitting_systems(cfg)
    dmw = mirror_wfs_system(cfg)
    out = {"workload": "E-ELT POLC step: open-loop slopes, tomography 10 warm its, W^-1, "
                       "fitting of 3 mirrors (~10,500 actuators) over 25 directions, 4 warm its",
           "actuators": None}
    for dt, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        ctl = PolcController(cfg, sig, dmw, atm, dm, dtype=dt, gain=0.4, n_iter=10)
        out["actuators"] = ctl.fitter.n_act
        s = slopes.to(tdt)
        for t in range(warmup):
            ctl.step(s[t % s.shape[0]][None].contiguous())
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for t in range(steps):
            ev[t][0].record()
            ctl.step(s[(warmup + t) % s.shape[0]][None].contiguous())
            ev[t][1].record()
        torch.cuda.synchronize()
        lat = sorted(a.elapsed_time(b) for a, b in ev)
        out[dt] = {"p50_ms_per_step": round(statistics.median(lat), 4),
                   "p99_ms_per_step": round(pctl(lat, 0.99), 4)}
        ctl.close()
    return out


def iteration_sweep(frames=(1, 11, 21, 31), iters=(1, 2, 3, 4, 6, 8, 10, 15, 20)):
    """Speed/quality trade-off of the paper's three solvers on the same E-ELT
    frames (Sec. 5.2-5.3; a synthetic stand-in for its iteration study): nine
    layers with Jacobi PCG, nine layers with plain CG, three layers at the
    mirror altitudes with Jacobi PCG.  Each solves in FP64 for several
    iteration counts, from zero and warm-started from the same variant's
    30-iteration reconstruction of the previous frame (the paper's warm
    restart); the on-axis residual and K-band Strehl against the nine truth
    screens are averaged over the frames.  Time: one frame, hipGraph replay,
    at the variant's own iteration count."""
    import torch
    from paper_1302_3734_amd import Plan
    base = WL.config_c2()
    fwd = Plan(base, [1.0] * len(base["wfs"]), dtype="f64", max_batch=1)
    # one frozen-flow sequence per frame: frame t follows frame t - 1 of the
    # sequence seeded at t - 1
    seeds = [t - 1 for t in frames]
    sl, sig = _synthetic_slopes(base, fwd, frames, seeds)
    prev, _ = _synthetic_slopes(base, fwd, seeds, seeds, sig)
    fwd.close()
    truths = [np.concatenate([a.ravel() for a in WL.layer_screens(base, t, seed_frame=t - 1)])
              for t in frames]
    out = {"frames": list(frames), "iterations": list(iters)}
    for name in ("C2", "C2-cg9", "C2-dm3"):
        cfg = WL.config_by_name(name)
        plan = Plan(cfg, sig, dtype="f64", max_batch=len(frames), tile=16,
                    precond=bool(cfg.get("precond", True)))
        x_prev = torch.zeros(len(frames), plan.n, dtype=torch.float64, device="cuda")
        plan.solve(prev, x_prev, n_iter=30)
        res = {"cold": ([], []), "warm": ([], [])}
        for k in iters:
            for mode in ("cold", "warm"):
                x = x_prev.clone() if mode == "warm" else torch.zeros_like(x_prev)
                plan.solve(sl, x, n_iter=k, warm_start=mode == "warm")
                lay = plan.coeffs_to_layers(x).cpu().numpy().reshape(len(frames), -1)
                r = [onaxis_residual(cfg, lay[i], truths[i], base) for i in range(len(frames))]
                res[mode][0].append(round(float(np.mean([a for a, _ in r])), 5))
                res[mode][1].append(round(float(np.mean([b for _, b in r])), 5))
        its = int(cfg["n_iter"])
        x1 = torch.zeros(1, plan.n, dtype=torch.float64, device="cuda")
        s1 = sl[:1].contiguous()
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for _ in range(3):
                plan.solve(s1, x1, n_iter=its, graph=True, stream=st)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            for _ in range(20):
                plan.solve(s1, x1, n_iter=its, graph=True, stream=st)
            b.record(st)
        st.synchronize()
        out[name] = {"layers": len(cfg["layers"]), "preconditioner": bool(cfg.get("precond", True)),
                     "paper_iterations": its, "ms_per_frame_fp64": round(a.elapsed_time(b) / 20, 4),
                     "onaxis_rms_rad_cold": res["cold"][0], "strehl_K_cold": res["cold"][1],
                     "onaxis_rms_rad_warm": res["warm"][0], "strehl_K_warm": res["warm"][1]}
        plan.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=32, help="frames per step")
    ap.add_argument("--iters", type=int, default=10, help="PCG iterations per frame")
    ap.add_argument("--tile", type=int, default=0, help="wavelet tile edge (0: autotuned)")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default work shapes instead of autotuned ones")
    ap.add_argument("--streams", type=int, default=0,
                    help="concurrent parts of a solve: 1..4, 0 library default (2)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the per-frame FP64 comparison")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--cpu-frames", type=int, default=2)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workloads (same as --extra none)")
    ap.add_argument("--extra", default="c2x128,c3,c4,polc,sweep",
                    help="comma list of extra workloads: c2x128 (128 E-ELT frames per solve), c3 "
                         "(128 8 m frames), c4 (mixed sizes), polc (closed-loop control steps), "
                         "sweep (iteration study), or none")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a 256 MiB device copy (byte-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(frames would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)

    # CPU oracle first, before anything initialises the GPU (forked workers).
    cpu = None
    if not args.no_cpu:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(workers, args.cpu_frames, args.iters)
        print(f"[bench] cpu oracle {cpu['value']:.3f} frames/s on {workers} cores", flush=True)

    import torch
    from paper_1302_3734_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = WL.config_c2()
    B, K, Wm, IT = args.batch, args.steps, args.warmup, args.iters

    # ---- synthetic inputs: screens on the host, slopes by the forward model --
    fwd = Plan(cfg, [1.0] * len(cfg["wfs"]), dtype="f64", max_batch=1)
    n, ns, so = fwd.n, fwd.n_slopes, fwd.slope_offsets
    truth0 = WL.layer_screens(cfg, 0, seed_frame=0)
    t0 = torch.tensor(np.concatenate([a.ravel() for a in truth0]), device="cuda")[None]
    clean0 = fwd.forward_layers(t0).cpu().numpy().ravel()
    sig = WL.sigmas_from_clean(cfg, clean0, so)
    sigvec = torch.tensor(np.concatenate([np.full(so[m + 1] - so[m], sig[m])
                                          for m in range(len(sig))]), device="cuda")
    print(f"[bench] sigma {['%.3g' % s for s in sig]}", flush=True)

    truths = {}                                  # (stream, t) -> concatenated layers (host)
    slopes64 = torch.empty(N_FRAMES_ROT + 1, B, ns, dtype=torch.float64, device="cuda")
    for k in range(B):
        base = 1000 * k
        for t in range(N_FRAMES_ROT + 1):
            lay = WL.layer_screens(cfg, base + t, seed_frame=base)
            v = np.concatenate([a.ravel() for a in lay])
            if k == 0:
                truths[t] = v
            s = fwd.forward_layers(torch.tensor(v, device="cuda")[None])[0]
            xi = torch.tensor(WL.noise_draw(cfg["cfg_id"], base + t, ns), device="cuda")
            slopes64[t, k] = s + sigvec * xi
    fwd.close()
    slopes32 = slopes64.float().contiguous()
    print("[bench] inputs ready", flush=True)

    # ---- work shapes: autotuned for this device, configuration and batch -----
    from paper_1302_3734_amd import autotune

    def shapes(dtype, batch):
        """Work shapes tuned for the library's default plan (two concurrent
        parts where large enough); --streams runs use the same shapes."""
        sh = dict(autotune.DEFAULTS) if args.no_tune else autotune.tune(cfg, sig, dtype, batch, IT)
        if args.tile:
            sh["tile"] = args.tile
        return sh

    t_tune = time.perf_counter()
    shapes32 = shapes("f32", B)
    print(f"[bench] work shapes for {B} frames: {shapes32} ({time.perf_counter() - t_tune:.1f} s)",
          flush=True)

    # ---- batched FP32 plan --------------------------------------------------
    p32 = Plan(cfg, sig, dtype="f32", max_batch=B, streams=args.streams, **shapes32)
    X = torch.zeros(B, n, dtype=torch.float32, device="cuda")
    p32.solve(slopes32[0], X, n_iter=30)           # frame 0 of every stream from zero
    torch.cuda.synchronize()

    def step(i):
        t = 1 + (i % N_FRAMES_ROT)
        p32.solve(slopes32[t], X, n_iter=IT, warm_start=True)

    for i in range(Wm):
        step(i)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for i in range(K):
        ev[i][0].record()
        step(Wm + i)
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    lat = sorted(a.elapsed_time(b) for a, b in ev)
    p50 = statistics.median(lat)
    p99 = pctl(lat, 0.99)
    fps = B * K / wall
    ms_step = 1e3 * wall / K
    print(f"[bench] fp32 batch {B}: {fps:.1f} frames/s, {ms_step:.3f} ms/step, p99 {p99:.3f} ms",
          flush=True)

    # ---- did the timed steps run two concurrent halves? ---------------------
    p32.profile(True)
    step(Wm + K)
    torch.cuda.synchronize()
    tot2 = p32.profile_read()
    p32.profile(False)
    halves = tot2["update_r"][1] > IT   # a split step updates each half separately

    # ---- per-kernel timing with HIP events on the launch stream ------------
    # On one stream (the same kernels over the whole batch of B frames), so a
    # launch's event time is its own: with two concurrent halves it would also
    # hold the other half's kernels.
    p1 = p32 if not halves else Plan(cfg, sig, dtype="f32", max_batch=B, streams=1, **shapes32)

    def step1(i):
        t = 1 + (i % N_FRAMES_ROT)
        p1.solve(slopes32[t], X, n_iter=IT, warm_start=True)

    step1(Wm + K + 1)
    prof_steps = 5
    p1.profile(True)
    for i in range(prof_steps):
        step1(Wm + K + 2 + i)
    torch.cuda.synchronize()
    prof = p1.profile_read()
    p1.profile(False)
    if p1 is not p32:
        p1.close()
    stages, kernels = stage_table(prof, n, n_nodes(cfg), prof_steps, IT, B, TRAFFIC_FILE)
    dom = max((nm for nm in stages if nm != "PCG updates"), key=lambda nm: stages[nm]["ms"])
    D = stages[dom]
    print(f"[bench] dominant operator stage {dom}: {D['avg_launch_us']:.1f} us/launch, "
          f"{D['achieved_gbs']:.0f} GB/s by algorithmic bytes (one stream; timed steps "
          f"{'two concurrent halves' if halves else 'one stream'})", flush=True)
    for nm, v in stages.items():
        print(f"[bench]   stage {nm:26s} {v['ms'] / prof_steps:8.3f} ms/step  x{v['launches']:4d}  "
              f"{v['achieved_gbs']:7.1f} GB/s  frac {v['frac']:.3f}", flush=True)
    for k, v in kernels.items():
        print(f"[bench]   {k:12s} {v['avg_us']:9.1f} us  x{v['launches']:4d}  "
              f"{100 * v['share']:5.1f}%", flush=True)

    # ---- reconstruction check and the per-frame FP64 comparison -------------
    result = {}
    if not args.no_fp64:
        def per_frame(plan, frames_all, dt):
            """Back-to-back single-frame warm solves of stream 0 (hipGraph
            replay): frames/s and p99 latency."""
            x1 = torch.zeros(1, n, dtype=dt, device="cuda")
            plan.solve(frames_all[0, :1].contiguous(), x1, n_iter=30)
            torch.cuda.synchronize()
            stream = torch.cuda.Stream()
            lat, nf = [], 100
            frames = [frames_all[1 + (i % N_FRAMES_ROT), :1].contiguous() for i in range(nf)]
            buf = torch.empty_like(frames[0])
            with torch.cuda.stream(stream):
                for i in range(nf):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    buf.copy_(frames[i])
                    e0.record(stream)
                    plan.solve(buf, x1, n_iter=IT, warm_start=True, graph=True, stream=stream)
                    e1.record(stream)
                    lat.append((e0, e1))
            stream.synchronize()
            ls = sorted(a.elapsed_time(b) for a, b in lat[2:])
            return 1e3 / statistics.mean(ls), pctl(ls, 0.99)

        def burst(plan, frames_all, dt, nb):
            """nb frames of different streams arriving at once, solved one
            after another (batch 1): each frame's latency is the time from the
            burst to its own result."""
            x1 = torch.zeros(1, n, dtype=dt, device="cuda")
            stream = torch.cuda.Stream()
            frames = [frames_all[1 + (i % N_FRAMES_ROT), :1].contiguous() for i in range(nb)]
            buf = torch.empty_like(frames[0])
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ends = []
                for i in range(nb):
                    buf.copy_(frames[i])
                    plan.solve(buf, x1, n_iter=IT, warm_start=True, graph=True, stream=stream)
                    e = torch.cuda.Event(enable_timing=True)
                    e.record(stream)
                    ends.append(e)
            stream.synchronize()
            ls = sorted(e0.elapsed_time(e) for e in ends)
            return pctl(ls, 0.5), pctl(ls, 0.99), ls[-1]

        shapes1_64 = shapes("f64", 1)
        shapes1_32 = shapes("f32", 1)
        p64 = Plan(cfg, sig, dtype="f64", max_batch=1, **shapes1_64)
        fps64, p99_64 = per_frame(p64, slopes64, torch.float64)
        b50, b99, bmax = burst(p64, slopes64, torch.float64, B)
        q32 = Plan(cfg, sig, dtype="f32", max_batch=1, **shapes1_32)
        fps32, p99_32 = per_frame(q32, slopes32, torch.float32)
        q32.close()
        # equal reconstruction: FP32 and FP64 solves of stream 0 frame 1, both
        # warm-started from the same FP64 frame-0 reconstruction
        xa = torch.zeros(1, n, dtype=torch.float64, device="cuda")
        p64.solve(slopes64[0, :1].contiguous(), xa, n_iter=30)
        xb = xa.float()
        p64.solve(slopes64[1, :1].contiguous(), xa, n_iter=IT, warm_start=True)
        p32.solve(slopes32[1, :1].contiguous(), xb, n_iter=IT, warm_start=True)
        la = p64.coeffs_to_layers(xa).cpu().numpy().ravel()
        lb = p32.coeffs_to_layers(xb).double().cpu().numpy().ravel()
        tr = truths[1]
        rms_a, strehl_a = onaxis_residual(cfg, la, tr)
        rms_b, strehl_b = onaxis_residual(cfg, lb, tr)
        rms_0, _ = onaxis_residual(cfg, np.zeros_like(tr), tr)
        result["fp64_per_frame"] = {"frames_per_s": round(fps64, 2),
                                    "p99_frame_latency_ms": round(p99_64, 4),
                                    "mode": "batch 1, hipGraph replay", "work_shapes": shapes1_64}
        result["fp32_per_frame"] = {"frames_per_s": round(fps32, 2),
                                    "p99_frame_latency_ms": round(p99_32, 4),
                                    "mode": "batch 1, hipGraph replay", "work_shapes": shapes1_32}
        print(f"[bench] per frame: FP64 {fps64:.1f} frames/s p99 {p99_64:.3f} ms; "
              f"FP32 {fps32:.1f} frames/s p99 {p99_32:.3f} ms", flush=True)
        result["burst"] = {
            "frames": B,
            "plain_fp64_p50_latency_ms": round(b50, 4), "plain_fp64_p99_latency_ms": round(b99, 4),
            "plain_fp64_frames_per_s": round(1e3 * B / bmax, 2),
            "batched_fp32_p99_latency_ms": round(p99, 4), "batched_fp32_frames_per_s": round(fps, 2),
            "mode": "B frames at once: FP64 solved one by one (batch 1, graph) vs FP32 one batched step"}
        print(f"[bench] burst of {B}: plain FP64 p99 {b99:.3f} ms; batched FP32 p99 {p99:.3f} ms",
              flush=True)
        result["reconstruction"] = {
            "frame": "stream 0, frame 1, both warm-started from the FP64 30-iteration frame 0",
            "fp32_vs_fp64_coeff_rel_diff": float(
                np.linalg.norm(xb.double().cpu().numpy() - xa.cpu().numpy())
                / np.linalg.norm(xa.cpu().numpy())),
            "onaxis_uncorrected_rms_rad": round(rms_0, 4),
            "onaxis_residual_rms_rad_fp64": round(rms_a, 5),
            "onaxis_residual_rms_rad_fp32": round(rms_b, 5),
            "strehl_K_fp64": round(strehl_a, 5), "strehl_K_fp32": round(strehl_b, 5),
            "strehl_rel_diff": abs(strehl_a - strehl_b) / strehl_a}
        p64.close()

    extras = set() if args.no_extra else set(args.extra.split(",")) - {"none"}
    if "c2x128" in extras:
        result["c2_batch128"] = large_batch(cfg, sig, slopes32, shapes("f32", 128))
        r128 = result["c2_batch128"]
        print(f"[bench] c2 x128: {r128['ms_per_solve']:.3f} ms per solve, "
              f"{r128['frames_per_s']:.0f} frames/s; stage fracs "
              f"{ {k: v['frac'] for k, v in r128['stages'].items()} }", flush=True)
    if "c3" in extras:
        result["c3_batched"] = batched_small(tuned=not args.no_tune)
        print(f"[bench] c3 {result['c3_batched']}", flush=True)
    if "c4" in extras:
        result["c4_mixed"] = mixed_batch()
        print(f"[bench] c4 {result['c4_mixed']}", flush=True)
    if "polc" in extras:
        result["control_loop"] = control_loop(cfg, sig, slopes32[1:, 0])
        print(f"[bench] control loop {result['control_loop']}", flush=True)
    if "sweep" in extras:
        result["iteration_sweep"] = iteration_sweep()
        sw = result["iteration_sweep"]
        for name in ("C2", "C2-cg9", "C2-dm3"):
            v = sw[name]
            print(f"[bench] sweep {name}: {v['layers']} layers, {v['paper_iterations']} its "
                  f"{v['ms_per_frame_fp64']:.3f} ms/frame; Strehl_K warm by its {v['strehl_K_warm']}; "
                  f"cold {v['strehl_K_cold']}", flush=True)

    if args.serve_seconds > 0:
        tuned = not args.no_tune
        result["served"] = served_stream(args.serve_seconds, args.serve_rate, IT, "f32", tuned=tuned)
        print(f"[bench] served {result['served']}", flush=True)
        if not args.no_fp64:
            result["served_fp64"] = served_stream(args.serve_seconds, args.serve_rate, IT, "f64",
                                                  tuned=tuned)
            print(f"[bench] served FP64 (same server) {result['served_fp64']}", flush=True)
            result["served_plain_fp64"] = served_stream(min(2.0, args.serve_seconds),
                                                        args.serve_rate, IT, "f64", plain=True,
                                                        tuned=tuned)
            print(f"[bench] served plain FP64 {result['served_plain_fp64']}", flush=True)

    out = {
        "metric": "PCG frames/s and p99 frame latency at E-ELT scale; operator HBM GB/s vs peak",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "E-ELT 42 m, 6 LGS 84x84 + 3 TT NGS, 9 layers 128-256 px, "
                               "db3 5 levels, Jacobi PCG 10 its warm",
                   "frames_per_step": B, "pcg_iters": IT, "n_unknowns": n, "n_slopes": ns,
                   "concurrent_halves": bool(halves),
                   "precision": "FP32 vectors and operator storage; W^-1 and P^T in FP32, "
                                "W and every inner product and step scalar in FP64",
                   "work_shapes": shapes32, "work_shapes_source": "defaults" if args.no_tune
                   else "autotuned on this device"},
        "p50_frame_latency_ms": round(p50, 4),
        "p99_frame_latency_ms": round(p99, 4),
        "roofline": {"bound": "hbm", "kernel": dom, "kernels": D["kernels"],
                     "achieved": D["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": D["frac"], "traffic": D["traffic_per_launch"],
                     "traffic_unit": "bytes per launch",
                     "avg_launch_us": D["avg_launch_us"],
                     "algorithmic_bytes_per_launch": D["bytes_per_launch"],
                     "design_bytes_per_launch": D["design_bytes_per_launch"],
                     "bytes_rule": ("survey's algorithmic count per stage pass: W^-1 2n, "
                                    "P chain n+Q, P^T Q+n, W + alpha D 3n (right side 2n), "
                                    "updates 11n per iteration; x 4 B x frames, divided by "
                                    "the stage's launches"),
                     "measured_on": ("one stream, the same kernels over the whole batch (the "
                                     "timed steps run it as two concurrent halves, where a "
                                     "launch's event time would also hold the other half's "
                                     "kernels)") if halves else "the timed configuration"},
        "stages": stages,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    out.update(result)
    if args.calib_copy:
        src_t = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    p32.close()


if __name__ == "__main__":
    main()
