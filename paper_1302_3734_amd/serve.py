"""Continuous-batching request loop for streams of wavelet-MCAO frames.

Telescope streams submit slope frames as they arrive.  Every stream belongs
to a configuration whose plan (tables, Jacobi diagonal, scratch) stays
resident on the device together with the stream's warm-start coefficients
(the previous frame's reconstruction, Sec. 5.1).

Each configuration is bound to one or more HIP streams ("lanes"; default
priority) with a plan and staging buffers of their own on each, and every
launch of that configuration goes to one of its lanes, so the host enqueues a
launch as soon as its frames are admitted, without waiting for the previous
launch to finish.  A worker thread admits, per lane, the pending frames of
every telescope stream (oldest first, at most `max_frames` per stream) while
the bytes reserved by frames in flight stay within an HBM budget and the lane
holds fewer than `depth` launches, and batches them into one multi-plan PCG
launch (``wmcao_solve_multi``, replayed as a captured HIP graph from fixed
staging buffers).  The frames of one stream in one launch all start from the
stream's newest reconstruction that the launch can use without waiting: the
result of the newest frame launched on the same lane (stream order on the
device delivers it), or a newer one already complete on another lane.  With
one lane per configuration each frame thus starts from its predecessor's
result when frames arrive one by one, and a backlog is solved as one batch
rather than one frame after another; with several lanes (`slots`) a frame
that arrives while its predecessor is still being solved starts at once on a
free lane, from the newest result already complete.  Lanes run side by side
on the device, so frames overlap.  A completion thread stamps each frame when its
launch's event completes; latency is arrival to completion.  Because every
frame's reductions are private and ordered, a frame's result does not depend
on the batch it was packed into.  Result tensors are allocated on the lane's
HIP stream and complete before their futures resolve.
"""
import collections
import ctypes as C
import threading
import time
from concurrent.futures import Future

import torch

from . import _abi
from .plan import Plan, solve_multi


GRAPH_CACHE = 64   # captures the library keeps (wmcao_solve_multi_graph)


class _Stream:
    def __init__(self, name, cfg_name, n, dtype, lanes):
        self.name = name
        self.cfg = cfg_name
        # warm-start state per lane: the newest result produced there (written
        # in that lane's stream order) and its frame index
        self.x = {lane: torch.zeros(1, n, dtype=dtype, device="cuda") for lane in lanes}
        self.x_index = {lane: -1 for lane in lanes}
        self.done = (-1, None)                                    # newest completed (index, result)
        self.queue = collections.deque()                          # frames not yet launched
        self.submitted = 0


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
    hip_streams: number of lanes (default: one per configuration); configuration
    i uses lane i mod hip_streams, unless lane_map ({config name: lane index})
    assigns the lanes.  slots (an int, or {config name: int}) above 1: every
    configuration gets that many lanes of its own instead (hip_streams,
    lane_map and pack are then unused), so that up to that many launches of
    one configuration run at once.  wait: how
    completions are found, "block" (a thread per lane waits on its oldest
    launch's event without holding the interpreter lock) or "poll" (one thread
    queries every lane's oldest event in turn, never while a launch may be
    capturing a graph: used whenever a lane packs two configurations or the
    lanes' launches outnumber the library's 64 kept captures, since a launch
    may then capture while frames are in flight).  hbm_budget: bytes that frames in flight may
    reserve (default: half of the free device memory at start).  depth: launches
    a lane may hold in flight.  max_frames: frames of one telescope stream in
    one launch.  keep_inputs: keep each frame's warm start (for
    invariance checks).  graphs: replay captured launches.  tile: tile edge of
    the wavelet kernels (0 = library default; 16 favours latency).  pack: when
    a lane serves several configurations, put their frames into one launch;
    otherwise one configuration per launch, in turn.  tuned: each
    configuration's plan takes the work shapes the autotuner finds for
    single-frame solves on this device (tile is then ignored).

    A caller with a latency target keeps Python's cyclic garbage collector
    off while it serves (gc.disable()): its passes over the objects of many
    frames in flight stall the worker and completion threads for milliseconds
    (served p99 at 2000 frames/s measured 6-13 ms with it, 3.0-3.1 ms
    without)."""

    def __init__(self, configs, streams, dtype="f32", n_iter=10, hip_streams=None,
                 hbm_budget=None, keep_inputs=False, graphs=True, tile=0, pack=True, depth=2,
                 max_frames=8, lane_map=None, tuned=False, slots=1, wait="block"):
        self.dtype = dtype
        self.n_iter = int(n_iter)
        self.keep_inputs = keep_inputs
        self.graphs = graphs
        self.pack = pack
        self.depth = max(1, int(depth))
        self.max_frames = max(1, int(max_frames))
        # frames of a configuration in one launch: max_frames per telescope stream
        count = {c: k * self.max_frames for c, k in collections.Counter(streams.values()).items()}
        names = [c for c in configs if count.get(c)]
        per_cfg = slots if isinstance(slots, dict) else {c: slots for c in names}
        self.slots = {c: max(1, int(per_cfg.get(c, 1))) for c in names}
        if any(k > 1 for k in self.slots.values()):
            self.cfg_lanes, n_lanes = {}, 0
            for c in names:
                self.cfg_lanes[c] = list(range(n_lanes, n_lanes + self.slots[c]))
                n_lanes += self.slots[c]
        elif lane_map:
            n_lanes = max(int(lane_map[c]) for c in names) + 1
            self.cfg_lanes = {c: [int(lane_map[c])] for c in names}
        else:
            n_lanes = min(len(names), int(hip_streams) if hip_streams else len(names))
            self.cfg_lanes = {c: [i % n_lanes] for i, c in enumerate(names)}
        self.lanes = [torch.cuda.Stream() for _ in range(n_lanes)]
        self.lane_cfgs = [[c for c in names if i in self.cfg_lanes[c]] for i in range(n_lanes)]
        # a plan per configuration and lane (its launches are ordered on that
        # lane), batch = the telescope streams of the configuration times
        # max_frames.  The lanes are the concurrency: plans that also split
        # large batches onto a second stream of their own made served frames
        # slower (p50 1.2 to 3.0 ms at 2000 frames/s), so the plans here use
        # one stream each.
        shapes = {c: {"tile": tile} for c in names}
        if tuned:
            from . import autotune
            shapes = {c: autotune.tune(configs[c][0], configs[c][1], dtype, 1, self.n_iter, streams=1)
                      for c in names}
        self.work_shapes = shapes
        # a plan (scratch) and fixed staging buffers per configuration and
        # lane: graph replays read the slopes and warm starts from, and leave
        # the results in, the staging buffers
        self.plans = {(c, lane): Plan(configs[c][0], configs[c][1], dtype=dtype, max_batch=count[c],
                                      streams=1, **shapes[c])
                      for c in names for lane in self.cfg_lanes[c]}
        first = {c: self.plans[(c, self.cfg_lanes[c][0])] for c in names}
        self.n = {c: p.n for c, p in first.items()}
        self.n_slopes = {c: p.n_slopes for c, p in first.items()}
        tdt = first[names[0]].torch_dtype
        self.torch_dtype = tdt
        self.streams = {s: _Stream(s, c, self.n[c], tdt, self.cfg_lanes[c]) for s, c in streams.items()}
        self.cfg_streams = {c: [st for st in self.streams.values() if st.cfg == c] for c in names}
        self.stage = {(c, lane): (torch.zeros(count[c], self.n_slopes[c], dtype=tdt, device="cuda"),
                                  torch.zeros(count[c], self.n[c], dtype=tdt, device="cuda"))
                      for c, lane in self.plans}
        if graphs:
            # capture the one-configuration launches up front, so that no frame
            # waits for a graph to be recorded; on a lane that packs two
            # configurations, every combination of frame counts too
            for (c, lane), plan in self.plans.items():
                Sb, Xb = self.stage[(c, lane)]
                with torch.cuda.stream(self.lanes[lane]):
                    for k in range(1, count[c] + 1):
                        solve_multi([plan], [Sb[:k]], [Xb[:k]], n_iter=self.n_iter,
                                    warm_start=True, graph=True)
            for lane, cs in enumerate(self.lane_cfgs):
                if not pack or len(cs) != 2:
                    continue
                (c0, c1), pl = cs, [self.plans[(c, lane)] for c in cs]
                st0, st1 = self.stage[(c0, lane)], self.stage[(c1, lane)]
                with torch.cuda.stream(self.lanes[lane]):
                    for k0 in range(1, count[c0] + 1):
                        for k1 in range(1, count[c1] + 1):
                            solve_multi(pl, [st0[0][:k0], st1[0][:k1]], [st0[1][:k0], st1[1][:k1]],
                                        n_iter=self.n_iter, warm_start=True, graph=True)
            torch.cuda.synchronize()
        esz = torch.empty(0, dtype=tdt).element_size()
        # bytes a frame in flight reserves: slopes + state + the plan scratch of one frame
        self.frame_bytes = {c: esz * (self.n_slopes[c] + 7 * self.n[c]) for c in names}
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = free // 2
        self.hbm_budget = int(hbm_budget)
        self.reserved = 0
        # one lock; the worker waits on cv (frames or free capacity), each lane's
        # completion thread on its own condition, the polling thread on any_cv,
        # so that a notification wakes only the thread that has work
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.lane_cv = [threading.Condition(self.lock) for _ in self.lanes]
        self.any_cv = threading.Condition(self.lock)
        # a launch may capture a new HIP graph on its lane; events recorded on
        # that lane must not be queried meanwhile, so launching and polling
        # take turns
        self.hip_lock = threading.Lock()
        self.inflight = [collections.deque() for _ in self.lanes]   # per lane, in launch order
        self.turn = [0] * n_lanes                                   # next configuration (no packing)
        self.running = True
        self.records = []
        self.launches = 0
        self.failed = 0                    # frames whose launch raised (their futures hold the error)
        self.lane_launches = [0] * n_lanes
        self.frames_in_launch = []
        self.worker = threading.Thread(target=self._loop, daemon=True)
        # blocking waits need every graph captured above and kept: lanes of one
        # configuration each, and no more captures than the library keeps (64)
        n_graphs = sum(count[c] for c, _ in self.plans)
        kept = n_graphs <= GRAPH_CACHE and all(len(cs) == 1 for cs in self.lane_cfgs)
        self.wait = wait if (not graphs or kept) else "poll"
        if self.wait == "block":
            self.completers = [threading.Thread(target=self._complete_lane, args=(lane,), daemon=True)
                               for lane in range(n_lanes)]
        else:
            self.completers = [threading.Thread(target=self._complete, daemon=True)]
        self.worker.start()
        for th in self.completers:
            th.start()

    # ---- client side ---------------------------------------------------------
    def submit(self, stream, slopes):
        """Queue one frame (device tensor of the plan dtype, n_slopes values);
        returns a Future resolving to (reconstruction coefficients, warm start
        or None)."""
        st = self.streams[stream]
        if slopes.numel() != self.n_slopes[st.cfg]:
            raise ValueError(f"stream {stream!r}: {slopes.numel()} slopes, the configuration "
                             f"has {self.n_slopes[st.cfg]}")
        if slopes.dtype != self.torch_dtype or not slopes.is_cuda:
            slopes = slopes.to(device="cuda", dtype=self.torch_dtype)
        slopes = slopes.reshape(1, -1).contiguous()
        with self.cv:
            fr = _Frame(st, slopes, st.submitted)
            st.submitted += 1
            st.queue.append(fr)
            self.cv.notify()
        return fr.future

    def close(self):
        with self.cv:
            self.running = False
            self._wake_all()
        self.worker.join()
        for th in self.completers:
            th.join()
        for p in self.plans.values():
            p.close()

    # ---- worker --------------------------------------------------------------
    def _admit_lane(self, lane):
        """Frames for one launch on a lane: the oldest pending frame of every
        telescope stream of the lane's configurations (one configuration, in
        turn, unless packing), within the HBM budget."""
        cfgs = self.lane_cfgs[lane]
        if not self.pack and len(cfgs) > 1:
            order = cfgs[self.turn[lane]:] + cfgs[:self.turn[lane]]
            for c in order:
                if any(st.queue for st in self.cfg_streams[c]):
                    cfgs = [c]
                    self.turn[lane] = (self.lane_cfgs[lane].index(c) + 1) % len(self.lane_cfgs[lane])
                    break
        groups = collections.OrderedDict()
        for c in cfgs:
            need = self.frame_bytes[c]
            for st in self.cfg_streams[c]:
                frs = []
                while st.queue and len(frs) < self.max_frames and \
                        self.reserved + need <= self.hbm_budget:
                    self.reserved += need
                    frs.append(st.queue.popleft())
                if frs:
                    groups.setdefault(c, []).append((st, frs))
        return groups

    @staticmethod
    def _warm_start(st, lane, stream):
        """The newest result of stream st that a launch on `lane` may read at
        once: the lane's own (stream order), or a newer complete one."""
        idx, x = st.done
        if x is not None and idx > st.x_index[lane]:
            x.record_stream(stream)   # read on this lane: keep its memory until then
            return x
        return st.x[lane]

    def _wake_all(self):
        """Wake every thread (call with the lock held)."""
        self.cv.notify_all()
        self.any_cv.notify_all()
        for c in self.lane_cv:
            c.notify_all()

    def _idle(self):
        return not any(st.queue for st in self.streams.values()) and not any(self.inflight)

    def _loop(self):
        pending = [0] * len(self.lanes)   # launches admitted but not yet in flight
        while True:
            with self.cv:
                while True:
                    work = []
                    for lane in range(len(self.lanes)):
                        if len(self.inflight[lane]) + pending[lane] >= self.depth:
                            continue
                        groups = self._admit_lane(lane)
                        if groups:
                            work.append((lane, groups))
                            pending[lane] += 1
                    if work:
                        break
                    if not self.running and self._idle():
                        self._wake_all()
                        return
                    self.cv.wait(timeout=0.05)
            for lane, groups in work:
                try:
                    self._launch(lane, groups)
                except Exception as e:   # the launch's frames fail; the server goes on
                    self._fail(groups, e)
                pending[lane] -= 1

    def _fail(self, groups, exc):
        """Resolve the futures of frames whose launch raised with that error."""
        t = time.perf_counter()
        frames = [f for per_stream in groups.values() for _, frs in per_stream for f in frs]
        with self.cv:
            for f in frames:
                f.t_done = t
                self.reserved -= self.frame_bytes[f.stream.cfg]
                self.failed += 1
            self.cv.notify()
        for f in frames:
            f.future.set_exception(exc)

    def _launch(self, lane, groups):
        if self.graphs and len(groups) == 1:
            ev, results = self._launch_one(lane, *next(iter(groups.items())))
        else:
            ev, results = self._launch_packed(lane, groups)
        with self.cv:
            self.launches += 1
            self.lane_launches[lane] += 1
            self.frames_in_launch.append(len(results))
            self.inflight[lane].append((ev, results))
            self.lane_cv[lane].notify()
            self.any_cv.notify()

    def _launch_one(self, lane, cfg, per_stream):
        """A launch of one configuration: its staging copies, the captured
        solve and the copies of the results out (every frame's, and each
        telescope stream's newest into its warm-start state) in one library
        call (wmcao_serve_launch)."""
        stream = self.lanes[lane]
        t_launch = time.perf_counter()
        Sb, Xb = self.stage[(cfg, lane)]
        sp, wp, orow, optr, results, states = [], [], [], [], [], []
        with torch.cuda.stream(stream):
            k = 0
            for st, frs in per_stream:
                x_src = self._warm_start(st, lane, stream)
                x0 = x_src.clone() if self.keep_inputs else None
                res = torch.empty(len(frs), self.n[cfg], dtype=self.torch_dtype, device="cuda")
                for i, f in enumerate(frs):
                    f.t_launch = t_launch
                    f.x0 = x0
                    stream.wait_event(f.ready)
                    f.slopes.record_stream(stream)   # read on the lane after the caller's work
                    sp.append(f.slopes.data_ptr())
                    wp.append(x_src.data_ptr())
                    orow.append(k + i)
                    optr.append(res[i].data_ptr())
                    results.append((f, res[i:i + 1]))
                orow.append(k + len(frs) - 1)        # the newest frame's result: the lane's state
                optr.append(st.x[lane].data_ptr())
                states.append((st, frs[-1].index))
                k += len(frs)
            vp = C.c_void_p
            with self.hip_lock:
                _abi.check(_abi.lib().wmcao_serve_launch(
                    self.plans[(cfg, lane)].handle, vp(Sb.data_ptr()), vp(Xb.data_ptr()), k,
                    (vp * k)(*sp), (vp * k)(*wp), len(orow), (C.c_int * len(orow))(*orow),
                    (vp * len(optr))(*optr), self.n_iter, vp(stream.cuda_stream)), "wmcao_serve_launch")
            ev = torch.cuda.Event()
            ev.record(stream)
        for st, idx in states:
            st.x_index[lane] = idx
        return ev, results

    def _launch_packed(self, lane, groups):
        stream = self.lanes[lane]
        t_launch = time.perf_counter()
        plans, slopes, coeffs, spans = [], [], [], []
        with torch.cuda.stream(stream):
            for per_stream in groups.values():
                for st, frs in per_stream:
                    for f in frs:
                        f.t_launch = t_launch
                        stream.wait_event(f.ready)
                        f.slopes.record_stream(stream)   # read on the lane after the caller's work
            for cfg, per_stream in groups.items():
                Sb, Xb = self.stage[(cfg, lane)]
                k = 0
                for st, frs in per_stream:
                    m = len(frs)
                    for i, f in enumerate(frs):
                        Sb[k + i].copy_(f.slopes[0])
                    # the stream's newest reconstruction this lane can use for all its frames
                    x_src = self._warm_start(st, lane, stream)
                    Xb[k:k + m].copy_(x_src.expand(m, -1))
                    if self.keep_inputs:
                        x0 = x_src.clone()
                        for f in frs:
                            f.x0 = x0
                    spans.append((cfg, st, frs, k))
                    k += m
                plans.append(self.plans[(cfg, lane)])
                slopes.append(Sb[:k])
                coeffs.append(Xb[:k])
            with self.hip_lock:
                solve_multi(plans, slopes, coeffs, n_iter=self.n_iter, warm_start=True,
                            graph=self.graphs)
            results = []
            for cfg, st, frs, k in spans:
                Xb = self.stage[(cfg, lane)][1]
                m = len(frs)
                st.x[lane].copy_(Xb[k + m - 1:k + m])   # the newest frame's result
                st.x_index[lane] = frs[-1].index
                res = Xb[k:k + m].clone()
                for i, f in enumerate(frs):
                    results.append((f, res[i:i + 1]))
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, results

    def _complete(self):
        while True:
            with self.any_cv:
                while not any(self.inflight):
                    if not self.running and self._idle() and not self.worker.is_alive():
                        return
                    self.any_cv.wait(timeout=0.05)
                heads = [(lane, q[0]) for lane, q in enumerate(self.inflight) if q]
            with self.hip_lock:
                done = [(lane, item) for lane, item in heads if item[0].query()]
            if not done:
                time.sleep(2e-5)
                continue
            self._finish(done)

    def _complete_lane(self, lane):
        q = self.inflight[lane]
        while True:
            with self.lane_cv[lane]:
                while not q:
                    if not self.running and self._idle() and not self.worker.is_alive():
                        return
                    self.lane_cv[lane].wait(timeout=0.05)
                item = q[0]
            # recorded after its launch, outside any capture (no lane of this
            # mode captures once serving has started)
            item[0].synchronize()
            self._finish([(lane, item)])

    def _finish(self, done):
        t = time.perf_counter()
        with self.cv:
            for lane, (ev, results) in done:
                self.inflight[lane].popleft()
                for f, x in results:
                    f.t_done = t
                    self.reserved -= self.frame_bytes[f.stream.cfg]
                    self.records.append((f.stream.name, f.index, f.t_arrival, t, f.t_launch))
                    if f.index > f.stream.done[0]:
                        f.stream.done = (f.index, x)
            self.cv.notify()
        for lane, (ev, results) in done:
            for f, x in results:
                f.future.set_result((x, f.x0))

    # ---- statistics ------------------------------------------------------------
    def latencies_ms(self):
        return [1e3 * (r[3] - r[2]) for r in self.records]

    def waits_ms(self):
        """Arrival to launch (queueing) and launch to completion, per frame."""
        return ([1e3 * (r[4] - r[2]) for r in self.records],
                [1e3 * (r[3] - r[4]) for r in self.records])
