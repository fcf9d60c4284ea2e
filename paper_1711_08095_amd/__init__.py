"""Python binding of libsnect (the C ABI declared in include/snect.h).

Argument marshalling only: every step of the SGD runs in the HIP kernels of
libsnect.so.  PyTorch supplies device memory (the factor tensors) and the
stream.  Importing this package does not need a GPU, but every call that does
device work fails loudly if the library is missing or no GPU is visible.
"""
from __future__ import annotations

import ctypes
import os
import sys
import weakref

from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnect.so")

SNECT_OK = 0
ERRORS = {
    -1: "SNECT_E_ARG", -2: "SNECT_E_INDEX", -3: "SNECT_E_DUPLICATE", -4: "SNECT_E_RANK",
    -5: "SNECT_E_OOM", -6: "SNECT_E_HIP", -7: "SNECT_E_DIVERGED", -8: "SNECT_E_BUSY",
    -9: "SNECT_E_UNSUPPORTED",
}
PRECISION_FP32 = 0
PRECISION_BF16 = 1

# Every symbol include/snect.h declares.
EXPORTS = (
    "snect_create", "snect_destroy", "snect_last_error", "snect_problem_create",
    "snect_problem_destroy", "snect_problem_info", "snect_train", "snect_evaluate",
    "snect_decompose", "snect_plan_export", "snect_last_timing", "snect_set_exec",
    "snect_exec_path", "snect_orthonormalize", "snect_server_create", "snect_server_destroy",
    "snect_server_submit", "snect_server_poll", "snect_server_replay", "snect_sweep_train",
    "snect_autotune", "snect_sweep_autotune", "snect_plan_layout", "snect_orthonormalize_noalloc",
)
PATH_AUTO, PATH_PERSISTENT, PATH_MULTI = 0, 1, 2


class SnectError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Tensor(ctypes.Structure):
    _fields_ = [("I1", ctypes.c_int32), ("I2", ctypes.c_int32), ("I3", ctypes.c_int32),
                ("nnz", ctypes.c_int64),
                ("i", ctypes.c_void_p), ("j", ctypes.c_void_p), ("k", ctypes.c_void_p),
                ("x", ctypes.c_void_p)]


class Graph(ctypes.Structure):
    _fields_ = [("E", ctypes.c_int64), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("J1", ctypes.c_int32), ("J2", ctypes.c_int32), ("J3", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("lambda_g", ctypes.c_double), ("lr", ctypes.c_double),
                ("core_lr_scale", ctypes.c_double),
                ("strata_P", ctypes.c_int32), ("tile_T", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class Factors(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("G", ctypes.c_void_p)]


class Exec(ctypes.Structure):
    _fields_ = [("per_launch_timing", ctypes.c_int32), ("path", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("rec_cap", ctypes.c_int32), ("wait_limit", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("pool_bytes", ctypes.c_int64), ("pg_iters", ctypes.c_int32),
                ("topk", ctypes.c_int32), ("lambda_", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("ntiles", ctypes.c_int64), ("edges_csr", ctypes.c_int64),
                ("P", ctypes.c_int32), ("T", ctypes.c_int32), ("rows1_max", ctypes.c_int32),
                ("rows2_max", ctypes.c_int32), ("bits_i", ctypes.c_int32), ("bits_j", ctypes.c_int32),
                ("n_sub", ctypes.c_int32), ("d_max", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("plan_seconds", ctypes.c_double),
                ("upload_seconds", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libsnect.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1711_08095_amd.build`")
    # torch brings the HIP runtime the library must share (device memory and
    # streams come from torch), so it is loaded first
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "snect_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp]),
        "snect_destroy": (ctypes.c_int, [vp]),
        "snect_last_error": (ctypes.c_char_p, [vp]),
        "snect_problem_create": (ctypes.c_int, [vp, ctypes.POINTER(Tensor), ctypes.POINTER(Graph),
                                                ctypes.POINTER(Params), ctypes.POINTER(vp)]),
        "snect_problem_destroy": (ctypes.c_int, [vp]),
        "snect_problem_info": (ctypes.c_int, [vp, ctypes.POINTER(Info)]),
        "snect_train": (ctypes.c_int, [vp, ctypes.POINTER(Factors), i32, i32, vp, vp]),
        "snect_evaluate": (ctypes.c_int, [vp, ctypes.POINTER(Factors), vp, vp]),
        "snect_decompose": (ctypes.c_int, [vp, ctypes.POINTER(Tensor), ctypes.POINTER(Graph),
                                           ctypes.POINTER(Params), ctypes.POINTER(Factors),
                                           ctypes.POINTER(Factors), i32, i32, vp, vp]),
        "snect_plan_export": (ctypes.c_int, [vp, i32, vp, vp, vp]),
        "snect_plan_layout": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "snect_last_timing": (ctypes.c_int, [vp, vp]),
        "snect_set_exec": (ctypes.c_int, [vp, ctypes.POINTER(Exec)]),
        "snect_exec_path": (ctypes.c_int, [vp]),
        "snect_orthonormalize": (ctypes.c_int, [vp, i32, i32, i32, i32, i32, i32, ctypes.POINTER(Factors)]),
        "snect_orthonormalize_noalloc": (ctypes.c_int, [vp, i32, i32, i32, i32, i32, i32,
                                                        ctypes.POINTER(Factors)]),
        "snect_server_create": (ctypes.c_int, [vp, i32, i32, i32, i32, i32, i32, ctypes.POINTER(Factors),
                                               ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
        "snect_server_destroy": (ctypes.c_int, [vp]),
        "snect_server_submit": (ctypes.c_int, [vp, i64, vp, vp, vp, ctypes.POINTER(i64)]),
        "snect_server_poll": (ctypes.c_int, [vp, i64, vp, vp, vp]),
        "snect_server_replay": (ctypes.c_int, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "snect_sweep_train": (ctypes.c_int, [vp, i32, vp, vp, i32, i32, vp, vp]),
        "snect_autotune": (ctypes.c_int, [vp, ctypes.POINTER(Factors), i32, ctypes.POINTER(Exec), vp]),
        "snect_sweep_autotune": (ctypes.c_int, [vp, i32, vp, vp, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _ = (i64, dbl)
    _lib = lib
    return lib


def _check(rc: int, ctx=None):
    if rc != SNECT_OK:
        msg = ""
        if ctx is not None:
            m = load().snect_last_error(ctx)
            msg = m.decode() if m else ""
        raise SnectError(rc, msg)


def _dev_ptr(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


@dataclass
class Hyper:
    ranks: tuple
    lam: float = 0.01
    lam_g: float = 0.1
    lr: float = 1e-3
    core_lr_scale: float = 1.0
    P: int = 8
    T: int = 64
    precision: int = PRECISION_FP32
    seed: int = 0

    def c(self) -> Params:
        p = Params()
        p.J1, p.J2, p.J3 = (int(r) for r in self.ranks)
        p.lambda_, p.lambda_g, p.lr = float(self.lam), float(self.lam_g), float(self.lr)
        p.core_lr_scale = float(self.core_lr_scale)
        p.strata_P, p.tile_T, p.precision = int(self.P), int(self.T), int(self.precision)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        return p


class Context:
    """snect_create / snect_destroy on a device and a stream (default: the
    current torch stream of that device)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        lib = load()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(lib.snect_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream)))
        self.h = h
        self.device = device
        self._problems = weakref.WeakSet()

    def close(self):
        """Destroy the context and every problem still open on it."""
        if self.h:
            for p in list(self._problems):
                p.close()
            _check(load().snect_destroy(self.h), self.h)
            self.h = None

    def __del__(self, _fin=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone (and
        # module globals already cleared, hence the bound default); the
        # process exit releases the memory
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass


def orthonormalize(ctx: "Context", A, B, C, G):
    """snect_orthonormalize on torch device tensors (in place)."""
    I1, J1 = A.shape
    I2, J2 = B.shape
    I3, J3 = C.shape
    f = Factors()
    f.A = _dev_ptr(A, (I1, J1), "A")
    f.B = _dev_ptr(B, (I2, J2), "B")
    f.C = _dev_ptr(C, (I3, J3), "C")
    f.G = _dev_ptr(G, (J1, J2, J3), "G")
    _check(load().snect_orthonormalize(ctx.h, I1, I2, I3, J1, J2, J3, ctypes.byref(f)), ctx.h)


def decompose(ctx: "Context", dims, i, j, k, x, eu, ev, ew, hyper: "Hyper", out, init=None, epochs: int = 1,
              start_epoch: int = 0):
    """snect_decompose: plan, train `epochs` epochs and release the plan in
    one call.  out = (A, B, C, G) torch device tensors receive the result;
    init = (A, B, C, G) device tensors, or None for the library's seeded
    N(0, sigma^2) start.  Returns (loss, rmse)."""
    lib = load()
    I1, I2, I3 = (int(d) for d in dims)
    J1, J2, J3 = (int(r) for r in hyper.ranks)
    shapes = ((I1, J1), (I2, J2), (I3, J3), (J1, J2, J3))

    def fac(ts, what):
        f = Factors()
        f.A, f.B, f.C, f.G = (_dev_ptr(t, sh, f"{what}.{n}") for t, sh, n in zip(ts, shapes, "ABCG"))
        return f

    keep = [np.ascontiguousarray(a, dtype=np.int32) for a in (i, j, k)]
    keep.append(np.ascontiguousarray(x, dtype=np.float32))
    t = Tensor()
    t.I1, t.I2, t.I3 = I1, I2, I3
    t.nnz = int(keep[0].shape[0])
    t.i, t.j, t.k, t.x = (a.ctypes.data for a in keep)
    eu = np.ascontiguousarray(np.zeros(0) if eu is None else eu, dtype=np.int32)
    ev = np.ascontiguousarray(np.zeros(0) if ev is None else ev, dtype=np.int32)
    ewa = None if ew is None else np.ascontiguousarray(ew, dtype=np.float32)
    g = Graph()
    g.E = int(eu.shape[0])
    g.u, g.v = eu.ctypes.data, ev.ctypes.data
    g.w = None if ewa is None else ewa.ctypes.data
    p = hyper.c()
    fo = fac(out, "out")
    fi = None if init is None else fac(init, "init")
    loss = np.zeros(max(epochs, 1))
    rmse = np.zeros(max(epochs, 1))
    _check(lib.snect_decompose(ctx.h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(p),
                               None if fi is None else ctypes.byref(fi), ctypes.byref(fo), int(start_epoch),
                               int(epochs), loss.ctypes.data, rmse.ctypes.data), ctx.h)
    return loss[:epochs], rmse[:epochs]


def orthonormalize_noalloc(ctx: "Context", A, B, C, G):
    """snect_orthonormalize_noalloc: the same, on the library's fixed
    per-device scratch (no allocation; overlapping calls on one device race)."""
    I1, J1 = A.shape
    I2, J2 = B.shape
    I3, J3 = C.shape
    f = Factors()
    f.A = _dev_ptr(A, (I1, J1), "A")
    f.B = _dev_ptr(B, (I2, J2), "B")
    f.C = _dev_ptr(C, (I3, J3), "C")
    f.G = _dev_ptr(G, (J1, J2, J3), "G")
    _check(load().snect_orthonormalize_noalloc(ctx.h, I1, I2, I3, J1, J2, J3, ctypes.byref(f)), ctx.h)


def _sweep_args(problems, factors):
    n = len(problems)
    if n == 0 or len(factors) != n:
        raise ValueError("one factor set per problem")
    hs = (ctypes.c_void_p * n)(*[p.h.value for p in problems])
    fs = (Factors * n)(*[p._factors(*f) for p, f in zip(problems, factors)])
    return n, hs, fs


def sweep_train(ctx: "Context", problems, factors, epochs: int, start_epoch: int = 0):
    """snect_sweep_train: the problems trained together (bit-identical to
    training each alone); factors[i] = (A, B, C, G) torch tensors of
    problem i (updated in place).  Returns (loss, rmse), arrays of shape
    (n, epochs)."""
    n, hs, fs = _sweep_args(problems, factors)
    loss = np.zeros((n, max(epochs, 1)))
    rmse = np.zeros((n, max(epochs, 1)))
    _check(load().snect_sweep_train(ctx.h, n, ctypes.cast(hs, ctypes.c_void_p), ctypes.cast(fs, ctypes.c_void_p),
                                    int(start_epoch), int(epochs), loss.ctypes.data, rmse.ctypes.data), ctx.h)
    return loss[:, :epochs], rmse[:, :epochs]


def sweep_autotune(ctx: "Context", problems, factors, trials: int = 1) -> float:
    """snect_sweep_autotune; returns the best sweep epoch time in ms."""
    n, hs, fs = _sweep_args(problems, factors)
    ms = ctypes.c_double()
    _check(load().snect_sweep_autotune(ctx.h, n, ctypes.cast(hs, ctypes.c_void_p), ctypes.cast(fs, ctypes.c_void_p),
                                       int(trials), ctypes.addressof(ms)), ctx.h)
    return ms.value


class Server:
    """snect_server_*: fold-in and top-k search for new patients against
    fixed device factors, with continuous batching.  The server derives what
    it needs from the factors before the constructor returns and does not
    read them afterwards."""

    def __init__(self, ctx: "Context", A, B, C, G, max_slots: int = 16, pool_bytes: int = 256 << 20,
                 pg_iters: int = 20, topk: int = 10, lam: float = 0.01):
        I1, J1 = A.shape
        I2, J2 = B.shape
        I3, J3 = C.shape
        self.ctx = ctx
        self.J1, self.topk = int(J1), int(topk)
        f = Factors()
        f.A = _dev_ptr(A, (I1, J1), "A")
        f.B = _dev_ptr(B, (I2, J2), "B")
        f.C = _dev_ptr(C, (I3, J3), "C")
        f.G = _dev_ptr(G, (J1, J2, J3), "G")
        cfg = ServerConfig()
        cfg.max_slots, cfg.pool_bytes, cfg.pg_iters = int(max_slots), int(pool_bytes), int(pg_iters)
        cfg.topk, cfg.lambda_ = int(topk), float(lam)
        h = ctypes.c_void_p()
        _check(load().snect_server_create(ctx.h, I1, I2, I3, J1, J2, J3, ctypes.byref(f), ctypes.byref(cfg),
                                          ctypes.byref(h)), ctx.h)
        self.h = h
        ctx._problems.add(self)

    def submit(self, j, k, x) -> int:
        """Returns a ticket; raises SnectError (code -8 when busy)."""
        j = np.ascontiguousarray(j, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = ctypes.c_int64()
        _check(load().snect_server_submit(self.h, int(j.shape[0]), j.ctypes.data, k.ctypes.data, x.ctypes.data,
                                          ctypes.byref(t)), self.ctx.h)
        return t.value

    def poll(self, ticket: int):
        """None while running, else (u, idx, score)."""
        u = np.zeros(self.J1)
        idx = np.zeros(self.topk, np.int32)
        sc = np.zeros(self.topk)
        rc = load().snect_server_poll(self.h, int(ticket), u.ctypes.data, idx.ctypes.data, sc.ctypes.data)
        if rc == 0:
            return None
        if rc != 1:
            _check(rc, self.ctx.h)
        return u, idx, sc

    def replay(self, arrival_s, offsets, j, k, x, gpu_busy=False):
        """Native open-loop replay; returns latencies, results and status
        (and, with gpu_busy, the seconds during which request kernels ran)."""
        arrival_s = np.ascontiguousarray(arrival_s, dtype=np.float64)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        j = np.ascontiguousarray(j, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        x = np.ascontiguousarray(x, dtype=np.float32)
        n = int(arrival_s.shape[0])
        lat = np.zeros(n)
        u = np.zeros((n, self.J1))
        idx = np.zeros((n, self.topk), np.int32)
        sc = np.zeros((n, self.topk))
        st = np.zeros(n, np.int32)
        wall = ctypes.c_double()
        busy = ctypes.c_double(-1.0)
        _check(load().snect_server_replay(self.h, n, arrival_s.ctypes.data, offsets.ctypes.data, j.ctypes.data,
                                          k.ctypes.data, x.ctypes.data, lat.ctypes.data, u.ctypes.data,
                                          idx.ctypes.data, sc.ctypes.data, st.ctypes.data,
                                          ctypes.addressof(wall), ctypes.addressof(busy) if gpu_busy else None),
               self.ctx.h)
        out = dict(latency_s=lat, u=u, idx=idx, score=sc, status=st, wall_s=wall.value)
        if gpu_busy:
            out["gpu_busy_s"] = busy.value
        return out

    def close(self):
        if getattr(self, "h", None):
            load().snect_server_destroy(self.h)
            self.h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """snect_problem_create on host arrays; the plan lives on the device."""

    def __init__(self, ctx: Context, dims, i, j, k, x, eu=None, ev=None, ew=None, hyper: Hyper = None):
        lib = load()
        self.ctx = ctx
        self.dims = tuple(int(d) for d in dims)
        self.hyper = hyper
        self._keep = [np.ascontiguousarray(a, dtype=np.int32) for a in (i, j, k)]
        self._keep.append(np.ascontiguousarray(x, dtype=np.float32))
        t = Tensor()
        t.I1, t.I2, t.I3 = self.dims
        t.nnz = int(self._keep[0].shape[0])
        t.i, t.j, t.k, t.x = (a.ctypes.data for a in self._keep)
        g = Graph()
        eu = np.zeros(0, np.int32) if eu is None else np.ascontiguousarray(eu, dtype=np.int32)
        ev = np.zeros(0, np.int32) if ev is None else np.ascontiguousarray(ev, dtype=np.int32)
        g.E = int(eu.shape[0])
        g.u, g.v = eu.ctypes.data, ev.ctypes.data
        ewa = None if ew is None else np.ascontiguousarray(ew, dtype=np.float32)
        g.w = None if ewa is None else ewa.ctypes.data
        h = ctypes.c_void_p()
        p = hyper.c()
        _check(lib.snect_problem_create(ctx.h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(p),
                                        ctypes.byref(h)), ctx.h)
        self.h = h
        self._keep = None  # the library copied what it needs
        ctx._problems.add(self)

    def _factors(self, A, B, C, G) -> Factors:
        I1, I2, I3 = self.dims
        J1, J2, J3 = self.hyper.ranks
        f = Factors()
        f.A = _dev_ptr(A, (I1, J1), "A")
        f.B = _dev_ptr(B, (I2, J2), "B")
        f.C = _dev_ptr(C, (I3, J3), "C")
        f.G = _dev_ptr(G, (J1, J2, J3), "G")
        return f

    def train(self, A, B, C, G, epochs: int, start_epoch: int = 0):
        """snect_train: updates the torch tensors in place; returns (loss, rmse)."""
        f = self._factors(A, B, C, G)
        loss = np.zeros(max(epochs, 1))
        rmse = np.zeros(max(epochs, 1))
        rc = load().snect_train(self.h, ctypes.byref(f), int(start_epoch), int(epochs),
                                loss.ctypes.data, rmse.ctypes.data)
        if rc != SNECT_OK:
            err = SnectError(rc, load().snect_last_error(self.ctx.h).decode())
            err.loss, err.rmse = loss[:epochs], rmse[:epochs]
            raise err
        return loss[:epochs], rmse[:epochs]

    def evaluate(self, A, B, C, G):
        f = self._factors(A, B, C, G)
        loss = ctypes.c_double()
        rmse = ctypes.c_double()
        _check(load().snect_evaluate(self.h, ctypes.byref(f), ctypes.addressof(loss),
                                     ctypes.addressof(rmse)), self.ctx.h)
        return loss.value, rmse.value

    def info(self) -> dict:
        inf = Info()
        _check(load().snect_problem_info(self.h, ctypes.byref(inf)), self.ctx.h)
        return {n: getattr(inf, n) for n, _ in Info._fields_}

    def plan_export(self, epoch: int = 0):
        I1, I2, _ = self.dims
        P = self.hyper.P
        perm1 = np.zeros(I1, np.int32)
        perm2 = np.zeros(I2, np.int32)
        strata = np.zeros(P, np.int32)
        _check(load().snect_plan_export(self.h, int(epoch), perm1.ctypes.data, perm2.ctypes.data,
                                        strata.ctypes.data), self.ctx.h)
        return dict(perm1=perm1, perm2=perm2, strata=strata)

    def plan_layout(self):
        """snect_plan_layout: the packed records (word, x), tile offsets and
        platforms and block -> tile ranges exactly as they sit on the device,
        with the field widths bits_i, bits_j."""
        inf = self.info()
        nnz, nt, P = int(inf["nnz"]), int(inf["ntiles"]), int(inf["P"])
        word = np.zeros(max(nnz, 1), np.uint32)
        x = np.zeros(max(nnz, 1), np.float32)
        tile_off = np.zeros(nt + 1, np.int32)
        tile_k = np.zeros(max(nt, 1), np.int32)
        blk_tile = np.zeros(P * P + 1, np.int32)
        _check(load().snect_plan_layout(self.h, word.ctypes.data, x.ctypes.data, tile_off.ctypes.data,
                                        tile_k.ctypes.data, blk_tile.ctypes.data), self.ctx.h)
        return dict(word=word[:nnz], x=x[:nnz], tile_off=tile_off, tile_k=tile_k[:nt], blk_tile=blk_tile,
                    bits_i=int(inf["bits_i"]), bits_j=int(inf["bits_j"]))

    def set_exec(self, per_launch_timing: bool = False, path: int = PATH_AUTO, waves: int = 0,
                 rec_cap: int = 0, wait_limit: int = 0):
        """snect_set_exec: per-launch timing events, the stratum driver, the
        wavefronts per workgroup and the record chunk (results unchanged),
        and the persistent kernel's wait limit (0: the default)."""
        e = Exec()
        e.per_launch_timing = 1 if per_launch_timing else 0
        e.path = int(path)
        e.waves = int(waves)
        e.rec_cap = int(rec_cap)
        e.wait_limit = int(wait_limit)
        _check(load().snect_set_exec(self.h, ctypes.byref(e)), self.ctx.h)

    def autotune(self, A, B, C, G, trials: int = 1):
        """snect_autotune on copies of the given factors; returns the chosen
        execution choice (dict) and its epoch time in ms."""
        f = self._factors(A, B, C, G)
        e = Exec()
        ms = ctypes.c_double()
        _check(load().snect_autotune(self.h, ctypes.byref(f), int(trials), ctypes.byref(e), ctypes.addressof(ms)),
               self.ctx.h)
        return {n: getattr(e, n) for n, _ in Exec._fields_}, ms.value

    def exec_path(self) -> int:
        return int(load().snect_exec_path(self.h))

    def last_timing(self):
        ms = np.zeros(5)
        _check(load().snect_last_timing(self.h, ms.ctypes.data), self.ctx.h)
        return dict(graph_ms=ms[0], strata_ms=ms[1], loss_ms=ms[2], kernel_ms=ms[3],
                    kernel_launches=int(ms[4]))

    def close(self):
        if getattr(self, "h", None):
            load().snect_problem_destroy(self.h)
            self.h = None

    def __del__(self, _fin=sys.is_finalizing):
        if _fin():
            return
        try:
            self.close()
        except Exception:
            pass


__all__ = ["load", "Context", "Problem", "Hyper", "SnectError", "EXPORTS", "ERRORS",
           "PRECISION_FP32", "PRECISION_BF16", "LIB_PATH", "PATH_AUTO", "PATH_PERSISTENT",
           "PATH_MULTI", "orthonormalize", "orthonormalize_noalloc", "Server", "sweep_train", "sweep_autotune", "decompose"]
