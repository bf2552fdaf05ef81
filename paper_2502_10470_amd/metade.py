"""Python binding of libmetade.so (argument marshalling only).

The functions named ``metade_*`` mirror the C entry points of
``include/metade.h`` one to one.  :class:`Batch` is a convenience wrapper that
takes a seeded workload description, allocates the caller-owned device
buffers with PyTorch and passes plain device pointers and the current HIP
stream to the library.  Every step of the method runs in the library's HIP
kernels; there is no CPU fallback -- without the built library or a GPU the
binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmetade.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4
FP32, BF16_REFINE = 0, 1
EVOLVER_DE, EVOLVER_PSO, EVOLVER_CSO, EVOLVER_NES = 0, 1, 2, 3
FN = {"rastrigin": 1, "rosenbrock": 2, "ackley": 3, "elliptic": 4, "schwefel": 5, "hybrid": 6,
      "lqr_mlp": 7}

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32


class MetadeProblem(ctypes.Structure):
    _fields_ = [
        ("kind", _u32), ("D", _u32), ("bias", ctypes.c_float), ("cond", ctypes.c_float),
        ("o", _vp), ("R", _vp), ("perm", _vp), ("split", _u32 * 3),
        ("obs", _u32), ("act", _u32), ("hidden1", _u32), ("hidden2", _u32), ("steps", _u32),
        ("n_rollouts", _u32), ("ctrl_weight", ctypes.c_float),
        ("A", _vp), ("B", _vp), ("x0", _vp),
    ]


class MetadeConfig(ctypes.Structure):
    _fields_ = [
        ("n_runs", _u32), ("N", _vp), ("problem", _vp), ("stream_id", _vp),
        ("n_problems", _u32), ("problems", _vp), ("seed", ctypes.c_uint64),
        ("lb", ctypes.c_float), ("ub", ctypes.c_float), ("n_cs", _u32), ("precision", _u32),
        ("pop", _vp), ("fit", _vp), ("best_y", _vp), ("best_x", _vp), ("stream", _vp),
        ("evolver", _u32), ("graph", _u32),
    ]


class MetadeTuning(ctypes.Structure):
    _fields_ = [("lane_parts", ctypes.c_uint32), ("mfma_rows", ctypes.c_uint32)]


class MetadeError(RuntimeError):
    pass


_lib = None

_SIGS = {
    "metade_query_sizes": [ctypes.POINTER(MetadeConfig)] + [ctypes.POINTER(ctypes.c_size_t)] * 5,
    "metade_init": [ctypes.POINTER(MetadeConfig), ctypes.POINTER(_vp)],
    "metade_reset": [_vp],
    "metade_set_theta": [_vp, _vp],
    "metade_inner_step": [_vp, _u32],
    "metade_inner_step_static": [_vp, _u32],
    "metade_trace_sizes": [_vp] + [ctypes.POINTER(ctypes.c_size_t)] * 3,
    "metade_inner_step_trace": [_vp, _vp, _vp, _vp],
    "metade_outer_reset": [_vp],
    "metade_outer_step": [_vp, _u32, _u32],
    "metade_get_outer": [_vp, _vp, _vp, _vp, _vp],
    "metade_set_outer": [_vp, _vp, _vp, _u32],
    "metade_run": [_vp, _u32, _u32, _u32, _vp, _vp, _vp],
    "metade_get_best": [_vp, _vp],
    "metade_get_state": [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)],
    "metade_set_state": [_vp, _vp, ctypes.c_size_t],
    "metade_kernel_timing": [_vp, ctypes.c_int],
    "metade_kernel_time": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)],
    "metade_get_counters": [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
    "metade_get_bound_check": [_vp] + [ctypes.POINTER(ctypes.c_uint64)] * 4
                              + [ctypes.POINTER(ctypes.c_double)],
    "metade_get_tuning": [_vp, ctypes.POINTER(MetadeTuning)],
    "metade_set_tuning": [_vp, ctypes.POINTER(MetadeTuning)],
    "metade_autotune": [_vp, _u32, ctypes.c_char_p, ctypes.POINTER(MetadeTuning),
                        ctypes.POINTER(ctypes.c_double)],
}
EXPORTED = tuple(_SIGS) + ("metade_last_error", "metade_destroy")


def lib():
    """Load libmetade.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MetadeError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2502_10470_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.metade_last_error.argtypes = [_vp]
        L.metade_last_error.restype = ctypes.c_char_p
        L.metade_destroy.argtypes = [_vp]
        L.metade_destroy.restype = None
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != OK:
        msg = lib().metade_last_error(ctx).decode()
        raise MetadeError(f"metade status {status}: {msg}")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ------------------------------------------------------------------ C entry points

def metade_query_sizes(cfg: MetadeConfig):
    out = [ctypes.c_size_t() for _ in range(5)]
    _check(lib().metade_query_sizes(ctypes.byref(cfg), *[ctypes.byref(o) for o in out]))
    return tuple(int(o.value) for o in out)


def metade_init(cfg: MetadeConfig) -> int:
    ctx = _vp()
    _check(lib().metade_init(ctypes.byref(cfg), ctypes.byref(ctx)))
    return ctx.value


def metade_reset(ctx):
    _check(lib().metade_reset(ctx), ctx)


def metade_set_theta(ctx, theta: np.ndarray):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    _check(lib().metade_set_theta(ctx, th.ctypes.data), ctx)


def metade_inner_step(ctx, n_generations: int):
    _check(lib().metade_inner_step(ctx, int(n_generations)), ctx)


def metade_inner_step_static(ctx, n_generations: int):
    _check(lib().metade_inner_step_static(ctx, n_generations), ctx)


def metade_trace_sizes(ctx):
    out = [ctypes.c_size_t() for _ in range(3)]
    _check(lib().metade_trace_sizes(ctx, *[ctypes.byref(o) for o in out]), ctx)
    return tuple(int(o.value) for o in out)


def metade_inner_step_trace(ctx, u, fu, desc):
    _check(lib().metade_inner_step_trace(ctx, _ptr(u), _ptr(fu), _ptr(desc)), ctx)


def metade_outer_reset(ctx):
    _check(lib().metade_outer_reset(ctx), ctx)


def metade_outer_step(ctx, G_inner: int, power_up: int = 1):
    _check(lib().metade_outer_step(ctx, int(G_inner), int(power_up)), ctx)


def metade_get_outer(ctx, n_runs: int):
    X = np.empty((n_runs, 6), np.float32)
    y = np.empty(n_runs, np.float64)
    U = np.empty((n_runs, 6), np.float32)
    yt = np.empty(n_runs, np.float64)
    _check(lib().metade_get_outer(ctx, X.ctypes.data, y.ctypes.data, U.ctypes.data,
                                  yt.ctypes.data), ctx)
    return X, y, U, yt


def metade_set_outer(ctx, X, y, gen: int):
    X = np.ascontiguousarray(X, np.float32)
    y = np.ascontiguousarray(y, np.float64)
    _check(lib().metade_set_outer(ctx, X.ctypes.data, y.ctypes.data, int(gen)), ctx)


def metade_run(ctx, outer_gens: int, G_inner: int, power_up: int, D_best: int):
    by = np.empty(1, np.float64)
    bt = np.empty(6, np.float32)
    bx = np.empty(D_best, np.float32)
    _check(lib().metade_run(ctx, int(outer_gens), int(G_inner), int(power_up), by.ctypes.data,
                            bt.ctypes.data, bx.ctypes.data), ctx)
    return float(by[0]), bt, bx


def metade_get_best(ctx, n_runs: int):
    y = np.empty(n_runs, np.float64)
    _check(lib().metade_get_best(ctx, y.ctypes.data), ctx)
    return y


def metade_get_state(ctx) -> bytes:
    n = ctypes.c_size_t()
    _check(lib().metade_get_state(ctx, None, ctypes.byref(n)), ctx)
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().metade_get_state(ctx, buf, ctypes.byref(n)), ctx)
    return buf.raw


def metade_set_state(ctx, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().metade_set_state(ctx, buf, len(blob)), ctx)


def metade_kernel_timing(ctx, enable: bool):
    _check(lib().metade_kernel_timing(ctx, 1 if enable else 0), ctx)


def metade_kernel_time(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check(lib().metade_kernel_time(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return float(ms.value), int(n.value)


def metade_get_counters(ctx):
    t = ctypes.c_uint64()
    r = ctypes.c_uint64()
    _check(lib().metade_get_counters(ctx, ctypes.byref(t), ctypes.byref(r)), ctx)
    return int(t.value), int(r.value)


def metade_get_bound_check(ctx):
    """(checked, outside, screened, screen_wrong, max_ratio) of traced bf16 generations."""
    v = [ctypes.c_uint64() for _ in range(4)]
    r = ctypes.c_double()
    _check(lib().metade_get_bound_check(ctx, *[ctypes.byref(x) for x in v], ctypes.byref(r)), ctx)
    return tuple(int(x.value) for x in v) + (float(r.value),)


def metade_get_tuning(ctx):
    t = MetadeTuning()
    _check(lib().metade_get_tuning(ctx, ctypes.byref(t)), ctx)
    return {"lane_parts": int(t.lane_parts), "mfma_rows": int(t.mfma_rows)}


def metade_set_tuning(ctx, lane_parts: int = 0, mfma_rows: int = 0):
    t = MetadeTuning(lane_parts, mfma_rows)
    _check(lib().metade_set_tuning(ctx, ctypes.byref(t)), ctx)


def metade_autotune(ctx, n_generations: int, cache_path: Optional[str] = None):
    """(chosen tuning as a dict, its milliseconds for n_generations)."""
    t = MetadeTuning()
    ms = ctypes.c_double()
    path = cache_path.encode() if cache_path else None
    _check(lib().metade_autotune(ctx, int(n_generations), path, ctypes.byref(t), ctypes.byref(ms)),
           ctx)
    return {"lane_parts": int(t.lane_parts), "mfma_rows": int(t.mfma_rows)}, float(ms.value)


def metade_last_error(ctx=None) -> str:
    return lib().metade_last_error(ctx).decode()


def metade_destroy(ctx):
    lib().metade_destroy(ctx)


# ------------------------------------------------------------------ convenience wrapper

class Batch:
    """A batch of executor runs on one GPU, built from a ``workloads.Workload``."""

    def __init__(self, wl, precision: int = FP32, device: str = "cuda:0", stream=None,
                 evolver: int = EVOLVER_DE, graph: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise MetadeError("no GPU visible: the MetaDE library runs on the GPU only")
        lib()
        self.torch = torch
        self.wl = wl
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = []
        dev = self.device

        def up(a, dtype):
            t = torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)
            self._keep.append(t)
            return t

        probs = (MetadeProblem * len(wl.problems))()
        for k, p in enumerate(wl.problems):
            q = probs[k]
            q.kind = FN[p.kind]
            q.D = p.D
            q.bias = float(p.bias)
            q.cond = float(p.cond)
            if p.o is not None:
                q.o = _ptr(up(p.o, torch.float32))
                q.R = _ptr(up(p.R, torch.float32))
            if p.perm is not None:
                q.perm = _ptr(up(p.perm.astype(np.int32), torch.int32))
                q.split[:] = list(p.split)
            if p.kind == "lqr_mlp":
                q.obs, q.act = p.A.shape[0], p.B.shape[1]
                q.hidden1, q.hidden2 = p.hidden
                q.steps = p.steps
                q.n_rollouts = p.x0.shape[0]
                q.ctrl_weight = p.ctrl_weight
                q.A = _ptr(up(p.A, torch.float32))
                q.B = _ptr(up(p.B, torch.float32))
                q.x0 = _ptr(up(p.x0, torch.float32))
        self._probs = probs
        self._N = np.ascontiguousarray(wl.N, np.uint32)
        self._P = np.ascontiguousarray(wl.problem, np.uint32)
        self._S = np.ascontiguousarray(wl.stream, np.uint32)
        cfg = MetadeConfig()
        cfg.n_runs = wl.n_runs
        cfg.N = self._N.ctypes.data
        cfg.problem = self._P.ctypes.data
        cfg.stream_id = self._S.ctypes.data
        cfg.n_problems = len(wl.problems)
        cfg.problems = ctypes.addressof(probs)
        cfg.seed = int(wl.seed)
        cfg.lb = float(wl.lb)
        cfg.ub = float(wl.ub)
        cfg.n_cs = int(wl.n_cs)
        cfg.precision = int(precision)
        cfg.evolver = int(evolver)
        cfg.graph = 1 if graph else 0
        cfg.stream = self.stream.cuda_stream
        pop_b, fit_b, by_b, bx_b, _ = metade_query_sizes(cfg)
        self.pop = torch.zeros(pop_b // 4, dtype=torch.float32, device=dev)
        self.fit = torch.zeros(fit_b // 4, dtype=torch.float32, device=dev)
        self.best_y = torch.zeros(by_b // 8, dtype=torch.float64, device=dev)
        self.best_x = torch.zeros(bx_b // 4, dtype=torch.float32, device=dev)
        cfg.pop = _ptr(self.pop)
        cfg.fit = _ptr(self.fit)
        cfg.best_y = _ptr(self.best_y)
        cfg.best_x = _ptr(self.best_x)
        self.cfg = cfg
        self.ctx = metade_init(cfg)
        Ds = np.array([wl.D_of(r) for r in range(wl.n_runs)], np.int64)
        Ns = self._N.astype(np.int64)
        self.D = Ds
        self.N = Ns
        self.pop_off = np.concatenate([[0], np.cumsum(Ns * Ds)])
        self.fit_off = np.concatenate([[0], np.cumsum(Ns)])
        self.bx_off = np.concatenate([[0], np.cumsum(Ds)])
        if wl.theta is not None:
            metade_set_theta(self.ctx, wl.theta)

    # -- thin forwards
    def reset(self):
        metade_reset(self.ctx)

    def set_theta(self, theta):
        metade_set_theta(self.ctx, theta)

    def inner_step(self, n):
        metade_inner_step(self.ctx, n)

    def inner_step_static(self, n):
        metade_inner_step_static(self.ctx, n)

    def trace_step(self):
        torch = self.torch
        ub, fb, db = metade_trace_sizes(self.ctx)
        u = torch.zeros(ub // 4, dtype=torch.float32, device=self.device)
        fu = torch.zeros(fb // 4, dtype=torch.float32, device=self.device)
        desc = torch.zeros(db // 4, dtype=torch.int32, device=self.device)
        metade_inner_step_trace(self.ctx, u, fu, desc)
        self.stream.synchronize()
        return u.cpu().numpy(), fu.cpu().numpy(), desc.cpu().numpy().reshape(-1, 16)

    def outer_reset(self):
        metade_outer_reset(self.ctx)

    def outer_step(self, G, power_up=1):
        metade_outer_step(self.ctx, G, power_up)

    def get_outer(self):
        return metade_get_outer(self.ctx, self.wl.n_runs)

    def set_outer(self, X, y, gen):
        metade_set_outer(self.ctx, X, y, gen)

    def run(self, outer_gens, G, power_up=5):
        return metade_run(self.ctx, outer_gens, G, power_up, int(self.D.max()))

    def get_best(self):
        return metade_get_best(self.ctx, self.wl.n_runs)

    def get_state(self):
        return metade_get_state(self.ctx)

    def set_state(self, blob):
        metade_set_state(self.ctx, blob)

    def kernel_timing(self, enable=True):
        metade_kernel_timing(self.ctx, enable)

    def kernel_time(self):
        return metade_kernel_time(self.ctx)

    def counters(self):
        return metade_get_counters(self.ctx)

    def bound_check(self):
        return metade_get_bound_check(self.ctx)

    def tuning(self):
        return metade_get_tuning(self.ctx)

    def set_tuning(self, lane_parts=0, mfma_rows=0):
        metade_set_tuning(self.ctx, lane_parts, mfma_rows)

    def autotune(self, n_generations, cache_path=None):
        return metade_autotune(self.ctx, n_generations, cache_path)

    # -- host views (synchronise)
    def host_state(self):
        self.stream.synchronize()
        pop = self.pop.cpu().numpy()
        fit = self.fit.cpu().numpy()
        return pop, fit

    def run_pop(self, pop, r):
        return pop[self.pop_off[r]:self.pop_off[r + 1]].reshape(int(self.N[r]), int(self.D[r]))

    def run_fit(self, fit, r):
        return fit[self.fit_off[r]:self.fit_off[r + 1]]

    def run_bx(self, bx, r):
        return bx[self.bx_off[r]:self.bx_off[r + 1]]

    def close(self):
        if getattr(self, "ctx", None):
            metade_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
