"""Continuous-batching request loop for streams of wavelet-MCAO frames.

Telescope streams submit slope frames as they arrive.  Every stream belongs
to a configuration whose plan (tables, Jacobi diagonal, scratch) stays
resident on the device together with the stream's warm-start coefficients
(the previous frame's reconstruction, Sec. 5.1).  A worker thread admits the
oldest pending frame of every stream that has no frame on the GPU, as long as
the bytes reserved by frames in flight stay within an HBM budget, and packs
all admitted frames of all configurations into one multi-plan PCG launch
(``wmcao_solve_multi``, captured as a HIP graph per combination of
configurations and frame counts and replayed from fixed staging buffers).
Launches alternate over several HIP streams (default priority) with one plan
instance per (configuration, HIP stream), so a batch admitted while another
is on the GPU runs alongside it.  A completion thread
stamps each frame when its launch's event completes; latency is arrival to
completion.  Because every frame's reductions are private and ordered, a
frame's result does not depend on the batch it was packed into.
"""
import collections
import threading
import time
from concurrent.futures import Future

import torch

from .plan import Plan, solve_multi


class _Stream:
    def __init__(self, name, cfg_name, n, dtype):
        self.name = name
        self.cfg = cfg_name
        self.x = torch.zeros(1, n, dtype=dtype, device="cuda")   # warm-start state
        self.queue = collections.deque()
        self.busy = False
        self.frames_done = 0


class _Frame:
    __slots__ = ("stream", "slopes", "ready", "t_arrival", "t_launch", "t_done", "future", "index",
                 "x0")

    def __init__(self, stream, slopes, index):
        self.stream = stream
        self.slopes = slopes
        self.ready = torch.cuda.Event()
        self.ready.record()              # the slopes are complete on the caller's stream
        self.t_arrival = time.perf_counter()
        self.t_launch = None
        self.t_done = None
        self.future = Future()
        self.index = index
        self.x0 = None


class Server:
    """Serve PCG solves for telescope streams with continuous batching.

    configs: {name: (cfg dict, sigmas)}; streams: {stream name: config name}.
    hbm_budget: bytes that frames in flight may reserve (default: half of the
    free device memory at start).  keep_inputs: keep each frame's warm start
    (for invariance checks).  graphs: replay captured launches.  tile: tile
    edge of the wavelet kernels (0 = library default; 16 favours latency).
    pack: put frames of several configurations into one launch (throughput);
    otherwise each configuration's frames go to a launch of their own, which
    runs alongside the others on its own HIP stream (latency)."""

    def __init__(self, configs, streams, dtype="f32", n_iter=10, hip_streams=2,
                 hbm_budget=None, keep_inputs=False, graphs=True, tile=0, pack=True):
        self.dtype = dtype
        self.n_iter = int(n_iter)
        self.keep_inputs = keep_inputs
        self.graphs = graphs
        self.pack = pack
        self.hip_streams = [torch.cuda.Stream() for _ in range(hip_streams)]
        count = collections.Counter(streams.values())
        # one plan per (configuration, HIP stream), batch = streams of that config
        self.plans = {c: [Plan(cfg, sig, dtype=dtype, max_batch=count[c], tile=tile)
                          for _ in range(hip_streams)]
                      for c, (cfg, sig) in configs.items() if count[c]}
        self.n = {c: p[0].n for c, p in self.plans.items()}
        self.n_slopes = {c: p[0].n_slopes for c, p in self.plans.items()}
        tdt = self.plans[next(iter(self.plans))][0].torch_dtype
        self.torch_dtype = tdt
        self.streams = {s: _Stream(s, c, self.n[c], tdt) for s, c in streams.items()}
        # fixed staging buffers per (configuration, HIP stream): graph replays
        # read the slopes and warm starts from, and leave the results in, them
        self.stage = {c: [(torch.zeros(count[c], self.n_slopes[c], dtype=tdt, device="cuda"),
                           torch.zeros(count[c], self.n[c], dtype=tdt, device="cuda"))
                          for _ in range(hip_streams)] for c in self.plans}
        if graphs:
            # capture the one-configuration launches up front, so that no frame
            # waits for a graph to be recorded
            for c, ps in self.plans.items():
                for hs, plan in enumerate(ps):
                    Sb, Xb = self.stage[c][hs]
                    with torch.cuda.stream(self.hip_streams[hs]):
                        for k in range(1, count[c] + 1):
                            solve_multi([plan], [Sb[:k]], [Xb[:k]], n_iter=self.n_iter,
                                        warm_start=True, graph=True)
            torch.cuda.synchronize()
        esz = torch.empty(0, dtype=tdt).element_size()
        # bytes a frame in flight reserves: slopes + state + the plan scratch of one frame
        self.frame_bytes = {c: esz * (self.n_slopes[c] + 7 * self.n[c]) for c in self.plans}
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = free // 2
        self.hbm_budget = int(hbm_budget)
        self.reserved = 0
        self.cv = threading.Condition()
        self.inflight = collections.deque()
        self.next_hs = 0
        self.hs_busy = [False] * hip_streams
        self.running = True
        self.records = []
        self.launches = 0
        self.frames_in_launch = []
        self.worker = threading.Thread(target=self._loop, daemon=True)
        self.completer = threading.Thread(target=self._complete, daemon=True)
        self.worker.start()
        self.completer.start()

    # ---- client side ---------------------------------------------------------
    def submit(self, stream, slopes):
        """Queue one frame (device tensor of the plan dtype, n_slopes values);
        returns a Future resolving to the reconstruction coefficients."""
        st = self.streams[stream]
        if slopes.dtype != self.torch_dtype or not slopes.is_cuda:
            slopes = slopes.to(device="cuda", dtype=self.torch_dtype)
        slopes = slopes.reshape(1, -1).contiguous()
        with self.cv:
            fr = _Frame(st, slopes, st.frames_done + len(st.queue))
            st.queue.append(fr)
            self.cv.notify_all()
        return fr.future

    def close(self):
        with self.cv:
            self.running = False
            self.cv.notify_all()
        self.worker.join()
        self.completer.join()
        for ps in self.plans.values():
            for p in ps:
                p.close()

    # ---- worker --------------------------------------------------------------
    def _admit(self):
        """Frames to launch now: the oldest pending frame of every idle stream,
        within the HBM budget, grouped per configuration (one configuration per
        launch unless packing)."""
        groups = collections.OrderedDict()
        for st in self.streams.values():
            if st.busy or not st.queue:
                continue
            if not self.pack and groups and st.cfg not in groups:
                continue
            need = self.frame_bytes[st.cfg]
            if self.reserved + need > self.hbm_budget:
                continue
            self.reserved += need
            st.busy = True
            groups.setdefault(st.cfg, []).append(st.queue.popleft())
        return groups

    def _loop(self):
        while True:
            with self.cv:
                while True:
                    free_hs = [i for i, b in enumerate(self.hs_busy) if not b]
                    groups = self._admit() if free_hs else {}
                    if groups:
                        break
                    if not self.running and not any(s.queue for s in self.streams.values()) \
                            and not any(self.hs_busy):
                        self.cv.notify_all()
                        return
                    self.cv.wait(timeout=0.05)
                hs = free_hs[0]
                self.hs_busy[hs] = True
            self._launch(hs, groups)

    def _launch(self, hs, groups):
        stream = self.hip_streams[hs]
        t_launch = time.perf_counter()
        for frs in groups.values():
            for f in frs:
                f.t_launch = t_launch
        plans, slopes, coeffs, frames = [], [], [], []
        with torch.cuda.stream(stream):
            for frs in groups.values():
                for f in frs:
                    stream.wait_event(f.ready)
            for cfg, frs in groups.items():
                plan = self.plans[cfg][hs]
                if self.graphs:
                    Sb, Xb = self.stage[cfg][hs]
                    S, X = Sb[:len(frs)], Xb[:len(frs)]
                    for k, f in enumerate(frs):
                        S[k].copy_(f.slopes[0])
                        X[k].copy_(f.stream.x[0])
                else:
                    S = torch.cat([f.slopes for f in frs]) if len(frs) > 1 else frs[0].slopes
                    X = torch.cat([f.stream.x for f in frs]) if len(frs) > 1 else frs[0].stream.x
                if self.keep_inputs:
                    for f in frs:
                        f.x0 = f.stream.x.clone()
                plans.append(plan)
                slopes.append(S)
                coeffs.append(X)
                frames.append(frs)
            solve_multi(plans, slopes, coeffs, n_iter=self.n_iter, warm_start=True,
                        graph=self.graphs)
            results = []
            for X, frs in zip(coeffs, frames):
                for k, f in enumerate(frs):
                    if X is not f.stream.x:
                        f.stream.x.copy_(X[k:k + 1])
                    results.append((f, f.stream.x.clone()))
            ev = torch.cuda.Event()
            ev.record(stream)
        self.launches += 1
        self.frames_in_launch.append(len(results))
        with self.cv:
            self.inflight.append((ev, hs, results))
            self.cv.notify_all()

    def _complete(self):
        while True:
            with self.cv:
                while not self.inflight:
                    if not self.running and not any(s.queue for s in self.streams.values()) \
                            and not any(self.hs_busy):
                        return
                    self.cv.wait(timeout=0.05)
                pending = list(self.inflight)
            done = None
            for item in pending:
                if item[0].query():
                    done = item
                    break
            if done is None:
                time.sleep(2e-5)
                continue
            t = time.perf_counter()
            ev, hs, results = done
            with self.cv:
                self.inflight.remove(done)
                self.hs_busy[hs] = False
                for f, _ in results:
                    f.t_done = t
                    f.stream.busy = False
                    f.stream.frames_done += 1
                    self.reserved -= self.frame_bytes[f.stream.cfg]
                    self.records.append((f.stream.name, f.index, f.t_arrival, t, f.t_launch))
                self.cv.notify_all()
            for f, x in results:
                f.future.set_result((x, f.x0))

    # ---- statistics ------------------------------------------------------------
    def latencies_ms(self):
        return [1e3 * (r[3] - r[2]) for r in self.records]

    def waits_ms(self):
        """Arrival to launch (queueing) and launch to completion, per frame."""
        return ([1e3 * (r[4] - r[2]) for r in self.records],
                [1e3 * (r[3] - r[4]) for r in self.records])
