#!/usr/bin/env python3
"""Benchmark of the wavelet-MCAO PCG solve at E-ELT scale on one MI355X.

Workload: the 42 m E-ELT configuration (6 sodium LGS with 84x84 Fried sensors
and cone effect, 3 tip/tilt NGS, 9 layers of 128..256 pixels, db3 with 5
levels, modified Jacobi PCG, 10 iterations, warm restart).  One step solves a
batch of B frames (B independent telescope streams, each warm-started from its
previous reconstruction) in FP32 with FP64 inner products and scalars.  Inputs
are synthetic: seeded von Karman screens with frozen flow, slopes from the
library's forward model plus Gaussian noise at SNR 20.

Prints one JSON line: frames/s, p99 frame latency, the dominant kernel's
achieved HBM bandwidth against the MI355X peak, the per-frame FP64 solve as a
comparison, and the CPU oracle on a bounded sample.
"""
import argparse
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
N_FRAMES_ROT = 4            # distinct frozen-flow frames per stream in rotation


# ----------------------------------------------------------------- CPU leg ----
def _cpu_worker(args):
    """Oracle on frames of one stream: rhs + 10 warm PCG iterations timed."""
    stream, frames, n_iter = args
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


def cpu_baseline(workers, frames_per_worker, n_iter):
    import multiprocessing as mp
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_cpu_worker, [(w, frames_per_worker, n_iter) for w in range(workers)])
    wall = time.perf_counter() - t0
    rate = sum(d / s for d, s in res)
    frames = sum(d for d, _ in res)
    return {"value": rate, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} processes x {frames_per_worker} frames of the E-ELT workload "
                      f"({frames} frames), FP64 NumPy oracle, right side + {n_iter} warm PCG "
                      f"iterations timed per frame; plan, Jacobi and input synthesis excluded; "
                      f"wall {wall:.1f} s"}


# ----------------------------------------------------------------- GPU leg ----
def algorithmic_bytes(plan_info, kernel, esz, frames, epi_apply=True):
    """Bytes one launch of ``kernel`` must move for ``frames`` frames (see the
    per-kernel table in the design notes): n unknowns, Q node values."""
    n, Q = plan_info["n"], plan_info["n_nodes"]
    lay = plan_info["layers"]                      # list of (N, k0)
    if kernel == "update_p":                       # read x, p, r, J; write x, p
        per = 6 * n
    elif kernel == "update_r":                     # read r, q, J; write r
        per = 4 * n
    elif kernel == "idwt_tile":                    # level-1 launch: read LL1 + details, write pixels
        per = 2 * sum(N * N for N, k0 in lay if k0 >= 1)
    elif kernel == "fdwt_tile":                    # nodes in; p details in; LL1 + details out
        per = Q + (1.75 if epi_apply else 1.0) * sum(N * N for N, k0 in lay if k0 >= 1)
    elif kernel == "idwt_coarse":
        per = 2 * sum((N >> k0) ** 2 for N, k0 in lay)
    elif kernel == "fdwt_coarse":
        per = 3 * sum((N >> k0) ** 2 for N, k0 in lay)
    elif kernel == "sensor":                       # pixels of every layer in, node fields out
        per = n + Q
    else:
        per = 4 * n
    return per * esz * frames


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=32, help="frames per step")
    ap.add_argument("--iters", type=int, default=10, help="PCG iterations per frame")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the per-frame FP64 comparison")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--cpu-frames", type=int, default=2)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
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

    # ---- batched FP32 plan --------------------------------------------------
    p32 = Plan(cfg, sig, dtype="f32", max_batch=B, tile=args.tile)
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
    p99 = lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]
    fps = B * K / wall
    ms_step = 1e3 * wall / K
    print(f"[bench] fp32 batch {B}: {fps:.1f} frames/s, {ms_step:.3f} ms/step, p99 {p99:.3f} ms",
          flush=True)

    # ---- per-kernel timing with HIP events on the launch stream ------------
    p32.profile(True)
    for i in range(5):
        step(Wm + K + i)
    torch.cuda.synchronize()
    prof = p32.profile_read()
    p32.profile(False)
    dom = max(prof, key=lambda k: prof[k][0])
    dms, dcnt = prof[dom]
    plan_info = {"n": n, "n_nodes": 9 * 85 * 85,
                 "layers": [(L["n"], 0 if (L["n"] ** 2) * 4 <= 65536 else 1) for L in cfg["layers"]]}
    abytes = algorithmic_bytes(plan_info, dom, 4, B)
    avg_s = dms / max(dcnt, 1) / 1e3
    achieved = abytes / avg_s / 1e9
    kernels = {k: {"avg_us": round(1e3 * v[0] / v[1], 3), "launches": v[1],
                   "share": round(v[0] / sum(x[0] for x in prof.values()), 4)}
               for k, v in prof.items() if v[1]}
    print(f"[bench] dominant kernel {dom}: {1e6 * avg_s:.1f} us/launch, {achieved:.0f} GB/s",
          flush=True)

    # ---- reconstruction check and the per-frame FP64 comparison -------------
    result = {}
    if not args.no_fp64:
        p64 = Plan(cfg, sig, dtype="f64", max_batch=1)
        x64 = torch.zeros(1, n, dtype=torch.float64, device="cuda")
        p64.solve(slopes64[0, :1].contiguous(), x64, n_iter=30)
        xs32 = torch.zeros(1, n, dtype=torch.float32, device="cuda")
        p32.solve(slopes32[0, :1].contiguous(), xs32, n_iter=30)
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
        lat64 = []
        nf = 40
        frames64 = [slopes64[1 + (i % N_FRAMES_ROT), :1].contiguous() for i in range(nf)]
        buf = torch.empty_like(frames64[0])
        with torch.cuda.stream(stream):
            for i in range(nf):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                buf.copy_(frames64[i])
                e0.record(stream)
                p64.solve(buf, x64, n_iter=IT, warm_start=True, graph=True, stream=stream)
                e1.record(stream)
                lat64.append((e0, e1))
        stream.synchronize()
        l64 = sorted(a.elapsed_time(b) for a, b in lat64[2:])
        fps64 = 1e3 / statistics.mean(l64)
        p99_64 = l64[min(len(l64) - 1, int(math.ceil(0.99 * len(l64))) - 1)]
        # equal reconstruction: FP32 and FP64 solves of stream 0 frame 1 from
        # the same frame-0 reconstructions
        xa = torch.zeros(1, n, dtype=torch.float64, device="cuda")
        p64.solve(slopes64[0, :1].contiguous(), xa, n_iter=30)
        p64.solve(slopes64[1, :1].contiguous(), xa, n_iter=IT, warm_start=True)
        xb = torch.zeros(1, n, dtype=torch.float32, device="cuda")
        p32.solve(slopes32[0, :1].contiguous(), xb, n_iter=30)
        p32.solve(slopes32[1, :1].contiguous(), xb, n_iter=IT, warm_start=True)
        la = p64.coeffs_to_layers(xa).cpu().numpy().ravel()
        lb = p32.coeffs_to_layers(xb).double().cpu().numpy().ravel()
        tr = truths[1]
        err_a = float(np.linalg.norm(la - tr) / np.linalg.norm(tr))
        err_b = float(np.linalg.norm(lb - tr) / np.linalg.norm(tr))
        result["fp64_per_frame"] = {"frames_per_s": round(fps64, 2),
                                    "p99_frame_latency_ms": round(p99_64, 4),
                                    "mode": "batch 1, hipGraph replay"}
        result["reconstruction"] = {
            "fp32_vs_fp64_coeff_rel_diff": float(
                np.linalg.norm(xb.double().cpu().numpy() - xa.cpu().numpy())
                / np.linalg.norm(xa.cpu().numpy())),
            "truth_rel_err_fp64": err_a, "truth_rel_err_fp32": err_b,
            "truth_err_rel_diff": abs(err_a - err_b) / err_a}
        p64.close()

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
                   "frames_per_step": B, "pcg_iters": IT, "n_unknowns": n, "n_slopes": ns},
        "p50_frame_latency_ms": round(p50, 4),
        "p99_frame_latency_ms": round(p99, 4),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "avg_launch_us": round(1e6 * avg_s, 3),
                     "algorithmic_bytes_per_launch": int(abytes)},
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    out.update(result)
    print(json.dumps(out), flush=True)
    p32.close()


if __name__ == "__main__":
    main()
