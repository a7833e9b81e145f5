"""paper_2408_00494_amd -- belief-space stochastic MPPI (BSS-MPPI) on MI355X.

Python front end of libbssmppi.  PyTorch supplies device memory (through the library's allocator
hook) and streams; the binding only marshals arguments to the C ABI, and every step of a solve
runs in the library's HIP kernels.

    from paper_2408_00494_amd import Solver, workloads
    prob, x0, v = workloads.config_small()
    s = Solver(prob)
    u0, info = s.solve(x0)
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import BssError, check, params_from_problem

__all__ = ["Solver", "Batch", "Server", "BssError", "backoff", "validate", "dev_philox", "dev_normals", "dev_disturbance", "solve_noalloc", "noalloc_scratch_bytes",
           "dev_model_step", "dev_model_step8", "dev_sdf", "dev_score", "dev_update", "dev_repair"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def validate(problem: dict) -> None:
    p = params_from_problem(problem)
    check(_lib.lib().bss_validate(C.byref(p)))


def backoff(problem: dict) -> float:
    p = params_from_problem(problem)
    nu = C.c_double()
    check(_lib.lib().bss_backoff(C.byref(p), C.byref(nu)))
    return nu.value


class Solver:
    """One BSS-MPPI controller instance (a library context) on the current CUDA/HIP device.

    Device buffers come from PyTorch's caching allocator; work goes on ``stream`` (default: the
    current stream at construction)."""

    def __init__(self, problem: dict, stream=None, lanes: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (torch.cuda.is_available() is False)")
        self.problem = dict(problem)
        self.K, self.M, self.T = int(problem["K"]), int(problem["M"]), int(problem["T"])
        self._n_con = int(problem.get("n_con", 0))
        self._params = params_from_problem(dict(problem, lanes=lanes))
        self._device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._blocks = {}

        def _alloc(nbytes, _user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self._device)
            self._blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _release(ptr, _user):
            self._blocks.pop(int(ptr), None)

        self._alloc_cb = BssAllocator_alloc(_alloc)
        self._release_cb = BssAllocator_release(_release)
        self._allocator = _lib.BssAllocator(self._alloc_cb, self._release_cb, None)
        ctx = C.c_void_p()
        check(_lib.lib().bss_create(C.byref(self._params), C.byref(self._allocator),
                                    _stream_ptr(self._stream), C.byref(ctx)))
        self._ctx = ctx

    # ---- lifetime -----------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.lib().bss_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- solves ---------------------------------------------------------------------------------
    def solve(self, x0, Sigma0=None):
        """Synchronous solve from host inputs.  Returns (u0 as numpy [2], info dict)."""
        x = np.ascontiguousarray(x0, dtype=np.float64)
        S0 = None if Sigma0 is None else np.ascontiguousarray(Sigma0, dtype=np.float64)
        u0 = np.zeros(2)
        info = _lib.BssInfo()
        dp = C.POINTER(C.c_double)
        st = _lib.lib().bss_solve(self._ctx, x.ctypes.data_as(dp),
                                  None if S0 is None else S0.ctypes.data_as(C.c_void_p),
                                  u0.ctypes.data_as(dp), C.byref(info))
        check(st)
        return u0, _info_dict(info)

    def solve_async(self, x0_dev, Sigma0_dev=None):
        """Enqueue a solve from device tensors (float64 [6] and [6, 6] or None)."""
        check(_lib.lib().bss_solve_async(self._ctx, _ptr(x0_dev), _ptr(Sigma0_dev)))

    def step_shift(self):
        check(_lib.lib().bss_step_shift(self._ctx))

    def info(self):
        info = _lib.BssInfo()
        check(_lib.lib().bss_get_info(self._ctx, C.byref(info)))
        return _info_dict(info)

    # ---- state --------------------------------------------------------------------------------
    def get_controls(self):
        v = np.zeros((self.T, 2))
        check(_lib.lib().bss_get_controls(self._ctx, v.ctypes.data_as(C.c_void_p)))
        return v

    def set_controls(self, v):
        vv = np.ascontiguousarray(v, dtype=np.float64).reshape(self.T, 2)
        check(_lib.lib().bss_set_controls(self._ctx, vv.ctypes.data_as(C.c_void_p)))

    @property
    def solve_index(self):
        s = C.c_uint32()
        check(_lib.lib().bss_get_solve_index(self._ctx, C.byref(s)))
        return s.value

    @solve_index.setter
    def solve_index(self, s):
        check(_lib.lib().bss_set_solve_index(self._ctx, int(s)))

    def set_lanes(self, lanes: int):
        check(_lib.lib().bss_set_lanes(self._ctx, int(lanes)))

    def set_shape(self, lanes: int = 0, ppl: int = 0, split: int = -1):
        """Force lanes per sample and/or particles per lane (0 = automatic; ppl wins) and the
        noise split (-1 automatic, 0 off, 1 on)."""
        check(_lib.lib().bss_set_shape(self._ctx, int(lanes), int(ppl), int(split)))

    def set_outputs(self, controls: bool = True, beliefs: bool = True):
        """Turn the optional per-solve outputs on or off: the copy of the sampled controls, and
        the belief records (without them the records may stay on chip; results are the same)."""
        flags = ((_lib.BSS_OUT_CONTROLS if controls else 0) |
                 (_lib.BSS_OUT_BELIEFS if beliefs else 0))
        check(_lib.lib().bss_set_outputs(self._ctx, flags))

    def buffers(self):
        """Torch views of the context's device buffers: v (current mean sequence, before any
        pending warm-start shift), u, mom, S, stats, and con_var (a_i^T Sigma a_i of the half-space
        constraints, [K][T+1][n_con]) when there are any.  Query again after each solve (the mean
        sequence alternates between two buffers)."""
        torch = _torch()
        b = _lib.BssBuffers()
        check(_lib.lib().bss_get_buffers(self._ctx, C.byref(b)))
        (base_ptr, blk), = self._blocks.items()
        K, T = self.K, self.T

        def view(ptr, nbytes, dtype, shape):
            off = ptr - base_ptr
            return blk[off:off + nbytes].view(dtype).reshape(shape)
        out = {
            "v": view(b.v, T * 2 * 8, torch.float64, (T, 2)),
            "u": view(b.u, K * T * 2 * 4, torch.float32, (K, T, 2)),
            "mom": view(b.mom, K * (T + 1) * 9 * 8, torch.float64, (K, T + 1, 9)),
            "S": view(b.S, K * 8, torch.float64, (K,)),
            "stats": view(b.stats, 8 * 8, torch.float64, (8,)),
            "v_shift": b.v_shift,
        }
        if b.con_var:
            n = self._n_con
            out["con_var"] = view(b.con_var, K * (T + 1) * n * 8, torch.float64, (K, T + 1, n))
        return out

    # ---- timing -------------------------------------------------------------------------------
    def timing(self, enable: bool):
        check(_lib.lib().bss_timing_enable(self._ctx, 1 if enable else 0))

    def timing_read(self):
        """(total rollout-kernel ms, number of solves) since the last read."""
        ms = C.c_double()
        n = C.c_int32()
        check(_lib.lib().bss_timing_read(self._ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Batch:
    """Many Solvers solved together: one rollout launch and one merge launch per batched solve
    (optionally replayed from a captured HIP graph).  Member i reads its state estimate from row i
    of the batch's state array (``set_states`` / ``copy_states_from``); results land in each
    member's buffers.  The members get their advanced state back in ``close``."""

    def __init__(self, solvers, ppl: int = 0, shift_after: bool = True):
        self.solvers = list(solvers)
        self.n = len(self.solvers)
        arr = (C.c_void_p * self.n)(*[s._ctx.value for s in self.solvers])
        b = C.c_void_p()
        check(_lib.lib().bss_batch_create(arr, self.n, int(ppl), 1 if shift_after else 0,
                                          C.byref(b)))
        self._b = b
        ptr = C.c_void_p()
        check(_lib.lib().bss_batch_states(self._b, C.byref(ptr)))
        self.states_ptr = ptr.value

    def set_states(self, x0):
        x = np.ascontiguousarray(x0, dtype=np.float64).reshape(self.n, 6)
        check(_lib.lib().bss_batch_set_states(self._b, x.ctypes.data_as(C.c_void_p)))

    def copy_states_from(self, x0_dev):
        """Enqueue a device-to-device copy of x0_dev (float64 [n, 6], contiguous) into the state
        array on the batch's stream."""
        check(_lib.lib().bss_batch_copy_states(self._b, _ptr(x0_dev.contiguous())))

    def solve(self):
        check(_lib.lib().bss_batch_solve(self._b))

    def capture(self):
        check(_lib.lib().bss_batch_capture(self._b))

    def tune(self):
        p = C.c_int32()
        check(_lib.lib().bss_batch_tune(self._b, C.byref(p)))
        return p.value

    def set_grid(self, persistent: bool):
        """Plain (False) or persistent work-queue (True) solve grid; before capture."""
        check(_lib.lib().bss_batch_set_grid(self._b, 1 if persistent else 0))

    def set_member_ppl(self, ppl):
        """Each member's own particles per lane (1, 2, 4 or 8), in one launch; before capture."""
        if len(ppl) != self.n:
            raise ValueError(f"need {self.n} values, got {len(ppl)}")
        arr = (C.c_int32 * self.n)(*[int(p) for p in ppl])
        check(_lib.lib().bss_batch_set_member_ppl(self._b, arr))

    def member_shape(self, i):
        """(lanes per sample, particles per lane) of member i in the current layout."""
        lanes, p = C.c_int32(), C.c_int32()
        check(_lib.lib().bss_batch_member_shape(self._b, int(i), C.byref(lanes), C.byref(p)))
        return lanes.value, p.value

    def layout(self):
        nb, p, sp = C.c_int32(), C.c_int32(), C.c_int32()
        check(_lib.lib().bss_batch_info(self._b, C.byref(nb), C.byref(p), C.byref(sp)))
        return {"nblocks": nb.value, "ppl": p.value, "split": bool(sp.value & 1),
                "persistent": bool(sp.value & 2),
                "member_ppl": [self.member_shape(i)[1] for i in range(self.n)]}

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            _lib.lib().bss_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving runtime: vehicles with device-resident warm starts whose solve requests (own K, M
    and delta each) are batched as they arrive over ``n_streams`` concurrent slots, admitted by an
    HBM scratch budget.  ``vehicles`` is a list of problem dicts (their K, M are ignored)."""

    def __init__(self, vehicles, T, K_max, M_max, ppl=4, n_streams=2, max_batch=256,
                 hbm_budget=32 << 30):
        self.n = len(vehicles)
        self.T = int(T)
        cfg = _lib.BssServerConfig(self.n, self.T, int(K_max), int(M_max), int(ppl),
                                   int(n_streams), int(max_batch), int(hbm_budget))
        arr = (_lib.BssParams * self.n)(*[params_from_problem(dict(p, K=K_max, M=M_max, T=T))
                                          for p in vehicles])
        srv = C.c_void_p()
        check(_lib.lib().bss_server_create(C.byref(cfg), arr, C.byref(srv)))
        self._s = srv

    def submit(self, vehicle, K, M, delta, x0):
        x = np.ascontiguousarray(x0, dtype=np.float64)
        rid = C.c_int64()
        check(_lib.lib().bss_server_submit(self._s, int(vehicle), int(K), int(M), float(delta),
                                           x.ctypes.data_as(C.c_void_p), C.byref(rid)))
        return rid.value

    def pump(self):
        n = C.c_int32()
        check(_lib.lib().bss_server_pump(self._s, C.byref(n)))
        return n.value

    def poll(self, max_n=1024):
        buf = (_lib.BssCompletion * max_n)()
        got = _lib.lib().bss_server_poll(self._s, buf, max_n)
        return [{"req": c.req, "vehicle": c.vehicle, "status": c.status,
                 "u0": np.array(c.u0[:]), "t_done": c.t_done} for c in buf[:got]]

    def drain(self):
        check(_lib.lib().bss_server_drain(self._s))

    def get_controls(self, vehicle):
        v = np.zeros((self.T, 2))
        check(_lib.lib().bss_server_get_controls(self._s, int(vehicle),
                                                 v.ctypes.data_as(C.c_void_p)))
        return v

    def set_controls(self, vehicle, v):
        vv = np.ascontiguousarray(v, dtype=np.float64).reshape(self.T, 2)
        check(_lib.lib().bss_server_set_controls(self._s, int(vehicle),
                                                 vv.ctypes.data_as(C.c_void_p)))

    def vehicle_state(self, vehicle):
        si, pend = C.c_uint32(), C.c_int64()
        check(_lib.lib().bss_server_vehicle_state(self._s, int(vehicle), C.byref(si),
                                                  C.byref(pend)))
        return si.value, pend.value

    def replay(self, t_arrival, vehicle, K, M, delta, x0):
        """Real-time replay of a request trace; returns (latency_s, u0 [n,2], status)."""
        t = np.ascontiguousarray(t_arrival, dtype=np.float64)
        n = t.shape[0]
        veh = np.ascontiguousarray(vehicle, dtype=np.int32)
        KK = np.ascontiguousarray(K, dtype=np.int32)
        MM = np.ascontiguousarray(M, dtype=np.int32)
        dd = np.ascontiguousarray(delta, dtype=np.float64)
        xx = np.ascontiguousarray(x0, dtype=np.float64).reshape(n, 6)
        lat = np.zeros(n)
        u0 = np.zeros((n, 2))
        st = np.zeros(n, dtype=np.int32)
        vp = C.c_void_p
        check(_lib.lib().bss_server_replay(
            self._s, n, t.ctypes.data_as(vp), veh.ctypes.data_as(vp), KK.ctypes.data_as(vp),
            MM.ctypes.data_as(vp), dd.ctypes.data_as(vp), xx.ctypes.data_as(vp),
            lat.ctypes.data_as(vp), u0.ctypes.data_as(vp), st.ctypes.data_as(vp)))
        return lat, u0, st

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            _lib.lib().bss_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BssAllocator_alloc = _lib.BssAllocator._fields_[0][1]
BssAllocator_release = _lib.BssAllocator._fields_[1][1]


def _info_dict(info):
    return {"S_min": info.S_min, "Z": info.Z, "ess": info.ess, "n_finite": info.n_finite,
            "lanes": info.lanes, "ppl": info.ppl, "split": bool(info.split),
            "dcbf_violations": info.dcbf_violations, "kernel_ms": info.kernel_ms,
            "records_on_chip": bool(info.records_on_chip)}


# ---- stand-alone kernels (device tensors in/out, current stream) --------------------------------
def dev_philox(seed: int, ctr):
    torch = _torch()
    out = torch.empty_like(ctr)
    check(_lib.lib().bss_dev_philox(int(seed), _ptr(ctr), _ptr(out), ctr.shape[0], _stream_ptr()))
    return out


def dev_normals(seed: int, ctr):
    torch = _torch()
    z = torch.empty((ctr.shape[0], 4), dtype=torch.float32, device=ctr.device)
    check(_lib.lib().bss_dev_normals(int(seed), _ptr(ctr), _ptr(z), ctr.shape[0], _stream_ptr()))
    return z


def solve_noalloc(problem: dict, s: int, x0, v_in, v_out, stats, Sigma0=None, stream=None):
    """One solve through bss_solve_noalloc (no device allocation: the library's static scratch):
    device tensors x0 [6], v_in [T][2], v_out [T][2], stats [8] (float64), Sigma0 [36] or None;
    enqueued on `stream` (default: torch's current stream)."""
    p = params_from_problem(problem)
    check(_lib.lib().bss_solve_noalloc(C.byref(p), int(s), _ptr(x0), _ptr(Sigma0), _ptr(v_in),
                                       _ptr(v_out), _ptr(stats), _stream_ptr(stream)))


def noalloc_scratch_bytes(problem: dict) -> int:
    """Scratch bytes bss_solve_noalloc needs for the problem (0 if it is invalid)."""
    p = params_from_problem(problem)
    return int(_lib.lib().bss_noalloc_scratch_bytes(C.byref(p)))


def dev_disturbance(seed: int, s: int, K: int, M: int, T: int, lanes: int, ppl: int,
                    crn: bool = False, device="cuda"):
    """Disturbance normals of a solve through the solve kernel's own noise path: returns
    (w [K][T][M][3] float32, words [K][T][3 ceil(M/4)][4] uint32 as int32 bits)."""
    torch = _torch()
    nblk = 3 * ((M + 3) // 4)
    w = torch.empty((K, T, M, 3), dtype=torch.float32, device=device)
    words = torch.empty((K, T, nblk, 4), dtype=torch.int32, device=device)
    check(_lib.lib().bss_dev_disturbance(int(seed), int(s), int(K), int(M), int(T),
                                         1 if crn else 0, int(lanes), int(ppl), _ptr(w),
                                         _ptr(words), _stream_ptr()))
    return w, words


def dev_model_step(problem: dict, x, u):
    torch = _torch()
    p = params_from_problem(problem)
    xn = torch.empty_like(x)
    check(_lib.lib().bss_dev_model_step(C.byref(p), _ptr(x), _ptr(u), _ptr(xn), x.shape[0],
                                        _stream_ptr()))
    return xn


def dev_model_step8(problem: dict, x, u):
    """One noise-free single-precision period of the 8-state vehicle: x [n, 8], u [n, 2]
    (float32 device tensors) -> xn [n, 8]."""
    torch = _torch()
    p = params_from_problem(problem)
    xn = torch.empty_like(x)
    check(_lib.lib().bss_dev_model_step8(C.byref(p), _ptr(x), _ptr(u), _ptr(xn), x.shape[0],
                                         _stream_ptr()))
    return xn


def dev_sdf(a: float, b: float, pts):
    torch = _torch()
    out = torch.empty((pts.shape[0], 3), dtype=torch.float64, device=pts.device)
    check(_lib.lib().bss_dev_sdf(float(a), float(b), _ptr(pts), _ptr(out), pts.shape[0],
                                 _stream_ptr()))
    return out


def dev_score(problem: dict, mom, u, v):
    torch = _torch()
    p = params_from_problem(problem)
    S = torch.empty((problem["K"],), dtype=torch.float64, device=mom.device)
    check(_lib.lib().bss_dev_score(C.byref(p), _ptr(mom), _ptr(u), _ptr(v), _ptr(S),
                                   _stream_ptr()))
    return S


def dev_update(problem: dict, S, u, v):
    """Returns (v+, stats) from device tensors S [K] f64, u [K,T,2] f32, v [T,2] f64."""
    torch = _torch()
    p = params_from_problem(problem)
    nbytes = _lib.lib().bss_dev_update_workspace(int(problem["K"]), int(problem["T"]))
    ws = torch.zeros((nbytes,), dtype=torch.uint8, device=S.device)
    vv = v.clone()
    stats = torch.zeros((8,), dtype=torch.float64, device=S.device)
    check(_lib.lib().bss_dev_update(C.byref(p), _ptr(S), _ptr(u), _ptr(vv), _ptr(stats),
                                    _ptr(ws), _stream_ptr()))
    return vv, stats


def dev_repair(problem: dict, mom, u):
    torch = _torch()
    p = params_from_problem(problem)
    out = torch.empty_like(u)
    check(_lib.lib().bss_dev_repair(C.byref(p), _ptr(mom), _ptr(u), _ptr(out), u.shape[0],
                                    _stream_ptr()))
    return out
