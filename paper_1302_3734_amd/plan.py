"""Python binding of the wavelet-MCAO solver: a Plan over the C ABI.

PyTorch provides device memory and the current HIP stream; every step of the
solve runs in the library's HIP kernels.  The binding only converts a
configuration dict into the ABI structs and passes tensor pointers.

Configuration dict keys (the same shape as the synthetic workload configs):
``diameter``, ``obstruction``, ``levels``, ``alpha``, ``r0``, ``L0``,
``layers`` (list of {altitude, weight, spacing, n}) and ``wfs`` (list of
{lgs, theta, H, n_sub, tt_aggregate, remove_tt, in_precond}).
"""
import ctypes as C

import torch

from . import _abi

_DT = {"f32": (_abi.WMCAO_F32, torch.float32), "f64": (_abi.WMCAO_F64, torch.float64)}


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Plan:
    """A solver plan for one telescope configuration on the current device."""

    def __init__(self, cfg, sigmas, dtype="f64", max_batch=1, cinv_blocks=None,
                 precond=True, resid_replace_every=0, tile=0, lds_budget=0, streams=0,
                 op_precision=0, op_fp64_stages=-1, proj_rows=0, vec_chunk=0, adj_lds=0):
        lib = _abi.lib()
        code, self.torch_dtype = _DT[dtype]
        self.dtype = dtype
        self.cfg = cfg
        self.max_batch = int(max_batch)
        layers = cfg["layers"]
        wfs = cfg["wfs"]
        Ls = (_abi.Layer * len(layers))()
        for i, L in enumerate(layers):
            Ls[i] = _abi.Layer(L["altitude"], L["weight"], L["spacing"], L["n"])
        Ws = (_abi.Wfs * len(wfs))()
        self._keep = []
        for m, w in enumerate(wfs):
            blk = None
            if cinv_blocks is not None and cinv_blocks[m] is not None:
                arr = (C.c_double * (len(cinv_blocks[m]) * 3))()
                flat = [float(v) for row in cinv_blocks[m] for v in row]
                for i, v in enumerate(flat):
                    arr[i] = v
                self._keep.append(arr)
                blk = C.cast(arr, C.POINTER(C.c_double))
            Ws[m] = _abi.Wfs(int(w["lgs"]), w["theta"][0], w["theta"][1], w.get("H", 90e3),
                             int(w["n_sub"]), int(w.get("tt_aggregate", 0)),
                             int(w.get("remove_tt", -1)), int(w.get("in_precond", -1)),
                             float(sigmas[m]) if sigmas is not None else 0.0, blk,
                             1 if w.get("kind", "sh") == "phase" else 0)
        pupil = _abi.Pupil(cfg["diameter"], cfg["obstruction"])
        opts = _abi.Options(cfg["alpha"], cfg["r0"], cfg["L0"], code, self.max_batch,
                            int(resid_replace_every), 1 if precond else 0, int(tile),
                            int(lds_budget), int(streams), int(op_precision),
                            int(op_fp64_stages), int(proj_rows), int(vec_chunk), int(adj_lds))
        h = C.c_void_p()
        rc = lib.wmcao_plan(C.byref(pupil), Ls, len(layers), Ws, len(wfs), _abi.Wavelet(0, 3),
                            int(cfg["levels"]), C.byref(opts), C.byref(h))
        _abi.check(rc, "wmcao_plan")
        self._h = h
        n = C.c_int64()
        ns = C.c_int64()
        lo = (C.c_int64 * (len(layers) + 1))()
        so = (C.c_int64 * (len(wfs) + 1))()
        _abi.check(lib.wmcao_sizes(h, C.byref(n), C.byref(ns), lo, so), "wmcao_sizes")
        self.n = n.value
        self.n_slopes = ns.value
        self.layer_offsets = list(lo)
        self.slope_offsets = list(so)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _abi.lib().wmcao_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers ---------------------------------------------------------
    def _check_vec(self, t, size, name):
        if not (t.is_cuda and t.dtype == self.torch_dtype and t.is_contiguous()):
            raise TypeError(f"{name}: contiguous {self.torch_dtype} CUDA tensor expected")
        if t.numel() % size:
            raise ValueError(f"{name}: size must be a multiple of {size}")
        b = t.numel() // size
        if not 1 <= b <= self.max_batch:
            raise ValueError(f"{name}: batch {b} outside 1..{self.max_batch}")
        return b

    def _new(self, batch, size):
        return torch.empty(batch, size, dtype=self.torch_dtype, device="cuda")

    def _call(self, fn, x, in_size, out_size, name, out=None):
        b = self._check_vec(x, in_size, name)
        y = self._new(b, out_size) if out is None else out
        self._check_vec(y, out_size, name + " out")
        _abi.check(fn(self._h, _ptr(x), _ptr(y), b, _stream_ptr()), name)
        return y

    # ---- ABI calls ---------------------------------------------------------
    def coeffs_to_layers(self, coeffs, out=None):
        return self._call(_abi.lib().wmcao_coeffs_to_layers, coeffs, self.n, self.n,
                          "wmcao_coeffs_to_layers", out)

    def layers_to_coeffs(self, layers, out=None):
        return self._call(_abi.lib().wmcao_layers_to_coeffs, layers, self.n, self.n,
                          "wmcao_layers_to_coeffs", out)

    def forward_layers(self, layers, out=None):
        return self._call(_abi.lib().wmcao_forward_layers, layers, self.n, self.n_slopes,
                          "wmcao_forward_layers", out)

    def rhs(self, slopes, out=None):
        return self._call(_abi.lib().wmcao_rhs, slopes, self.n_slopes, self.n, "wmcao_rhs", out)

    def apply_A(self, x, out=None):
        return self._call(_abi.lib().wmcao_apply_A, x, self.n, self.n, "wmcao_apply_A", out)

    def precond_diag(self):
        j = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _abi.check(_abi.lib().wmcao_precond_diag(self._h, _ptr(j), _stream_ptr()),
                   "wmcao_precond_diag")
        return j

    def profile(self, enable=True):
        """Start (or stop) per-kernel event timing of later calls on this plan."""
        _abi.check(_abi.lib().wmcao_profile_enable(self._h, int(bool(enable))), "wmcao_profile_enable")

    def profile_read(self):
        """{kernel name: (total ms, launches, algorithmic bytes)} since the last
        profile(True)."""
        out = {}
        for k, name in enumerate(_abi.KERNELS):
            ms = C.c_double()
            n = C.c_int()
            by = C.c_double()
            _abi.check(_abi.lib().wmcao_profile_read(self._h, k, C.byref(ms), C.byref(n),
                                                     C.byref(by)), "wmcao_profile_read")
            out[name] = (ms.value, n.value, by.value)
        return out

    def solve(self, slopes, coeffs=None, n_iter=10, warm_start=False, resid=None, status=None,
              graph=False, stream=None):
        """PCG solve; ``coeffs`` is updated in place (x0 in if warm_start)."""
        b = self._check_vec(slopes, self.n_slopes, "slopes")
        if coeffs is None:
            coeffs = self._new(b, self.n)
        self._check_vec(coeffs, self.n, "coeffs")
        if coeffs.numel() // self.n != b:
            raise ValueError("slopes and coeffs batch differ")
        rp = C.c_void_p(0)
        sp = C.c_void_p(0)
        if resid is not None:
            assert resid.dtype == torch.float64 and resid.numel() == b * (n_iter + 1)
            rp = _ptr(resid)
        if status is not None:
            assert status.dtype == torch.int32 and status.numel() == b
            sp = _ptr(status)
        fn = _abi.lib().wmcao_solve_graph if graph else _abi.lib().wmcao_solve
        _abi.check(fn(self._h, _ptr(slopes), _ptr(coeffs), b, int(n_iter), int(bool(warm_start)),
                      rp, sp, _stream_ptr(stream)), "wmcao_solve")
        return coeffs


def solve_multi(plans, slopes, coeffs, n_iter=10, warm_start=False, graph=False):
    """One packed PCG solve over frames of several plans (mixed sizes).  With
    graph=True the launches are captured once per argument set and replayed
    (the buffers must then stay allocated while the plans live)."""
    k = len(plans)
    H = (C.c_void_p * k)(*[p.handle.value for p in plans])
    S = (C.c_void_p * k)()
    X = (C.c_void_p * k)()
    N = (C.c_int * k)()
    for i, p in enumerate(plans):
        b = p._check_vec(slopes[i], p.n_slopes, "slopes")
        if p._check_vec(coeffs[i], p.n, "coeffs") != b:
            raise ValueError("slopes and coeffs batch differ")
        S[i] = slopes[i].data_ptr()
        X[i] = coeffs[i].data_ptr()
        N[i] = b
    name = "wmcao_solve_multi_graph" if graph else "wmcao_solve_multi"
    _abi.check(getattr(_abi.lib(), name)(H, S, X, N, k, int(n_iter), int(bool(warm_start)),
                                         _stream_ptr()), name)
    return coeffs
