"""FP64 oracle for SNeCT (arXiv:1711.08095) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it, and it shares no
code with the HIP path.

Two layers:
  * ``snect_oracle.c`` (built into ``liboracle.so`` by :func:`build`): the
    plan, the stratified SGD iteration and the objective, in FP64 C with
    OpenMP over the independent blocks of a stratum;
  * Algorithm 1 read literally on one core (``run_literal``), the
    comparison run for the stratified schedule;
  * plain numpy definitions in this module: the dense Tucker model (Eq. 2 via
    the mode-n products of Eq. 1), the objective f_opt (Eq. 3 + lambda_g
    Eq. 4), its per-nonzero split (Section 2.3.2) and finite-difference
    gradients, the fold-in least squares of Eq. (6), cosine top-k and the QR
    post-step of Algorithm 1.

Pins for every function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snect_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    lib.oracle_splitmix64_at.restype = ctypes.c_uint64
    lib.oracle_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_stream_state.restype = ctypes.c_uint64
    lib.oracle_stream_state.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_shuffle.restype = None
    lib.oracle_shuffle.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.oracle_run_literal.restype = ctypes.c_int
    lib.oracle_run_literal.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int32, ctypes.c_int32,
                                                               ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_loss.restype = ctypes.c_double
    lib.oracle_loss.argtypes = [ctypes.c_void_p] * 7
    lib.oracle_model_values.restype = None
    lib.oracle_model_values.argtypes = [ctypes.c_void_p] * 6
    lib.oracle_plan_export.restype = ctypes.c_int
    lib.oracle_plan_export.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 7
    lib.oracle_random_start.restype = None
    lib.oracle_random_start.argtypes = [ctypes.c_void_p] * 5
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    _lib = lib
    return lib


class _Prob(ctypes.Structure):
    _fields_ = [
        ("I1", ctypes.c_int32), ("I2", ctypes.c_int32), ("I3", ctypes.c_int32),
        ("J1", ctypes.c_int32), ("J2", ctypes.c_int32), ("J3", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("i", ctypes.c_void_p), ("j", ctypes.c_void_p), ("k", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("E", ctypes.c_int64),
        ("eu", ctypes.c_void_p), ("ev", ctypes.c_void_p), ("ew", ctypes.c_void_p),
        ("lam", ctypes.c_double), ("lam_g", ctypes.c_double), ("lr", ctypes.c_double),
        ("core_lr_scale", ctypes.c_double),
        ("P", ctypes.c_int32), ("T", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


ERRORS = {-1: "E_ARG", -2: "E_INDEX", -3: "E_DUPLICATE", -5: "E_OOM"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')})")
        self.code = code


class Problem:
    """Holds contiguous copies of a problem's arrays for the C oracle."""

    def __init__(self, dims, ranks, i, j, k, x, eu=None, ev=None, ew=None, lam=0.0,
                 lam_g=0.0, lr=1e-3, core_lr_scale=1.0, P=1, T=1, seed=0):
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.i = np.ascontiguousarray(i, dtype=np.int32)
        self.j = np.ascontiguousarray(j, dtype=np.int32)
        self.k = np.ascontiguousarray(k, dtype=np.int32)
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.eu = np.ascontiguousarray(eu if eu is not None else np.zeros(0), dtype=np.int32)
        self.ev = np.ascontiguousarray(ev if ev is not None else np.zeros(0), dtype=np.int32)
        self.ew = None if ew is None else np.ascontiguousarray(ew, dtype=np.float64)
        self.lam, self.lam_g, self.lr = float(lam), float(lam_g), float(lr)
        self.core_lr_scale = float(core_lr_scale)
        self.P, self.T, self.seed = int(P), int(T), int(seed)

    @property
    def nnz(self):
        return int(self.i.shape[0])

    def _c(self):
        def ptr(a):
            return None if a is None else a.ctypes.data
        s = _Prob()
        s.I1, s.I2, s.I3 = self.dims
        s.J1, s.J2, s.J3 = self.ranks
        s.nnz = self.nnz
        s.i, s.j, s.k, s.x = ptr(self.i), ptr(self.j), ptr(self.k), ptr(self.x)
        s.E = int(self.eu.shape[0])
        s.eu, s.ev, s.ew = ptr(self.eu), ptr(self.ev), ptr(self.ew)
        s.lam, s.lam_g, s.lr, s.core_lr_scale = self.lam, self.lam_g, self.lr, self.core_lr_scale
        s.P, s.T, s.seed = self.P, self.T, self.seed & 0xFFFFFFFFFFFFFFFF
        return s


def _f64(a, shape):
    out = np.array(a, dtype=np.float64, copy=True, order="C")
    if out.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {out.shape}")
    return out


def run(prob: Problem, A, B, C, G, epochs: int, start_epoch: int = 0, threads: int = 0):
    """Run the stratified SGD iteration; returns (A, B, C, G, loss[], rmse[])."""
    lib = _load()
    I1, I2, I3 = prob.dims
    J1, J2, J3 = prob.ranks
    A = _f64(A, (I1, J1)); B = _f64(B, (I2, J2)); C = _f64(C, (I3, J3)); G = _f64(G, (J1, J2, J3))
    loss = np.zeros(max(epochs, 1)); rmse = np.zeros(max(epochs, 1))
    s = prob._c()
    rc = lib.oracle_run(ctypes.byref(s), A.ctypes.data, B.ctypes.data, C.ctypes.data, G.ctypes.data,
                        int(start_epoch), int(epochs), loss.ctypes.data, rmse.ctypes.data, int(threads))
    if rc != 0:
        raise OracleError(rc)
    return A, B, C, G, loss[:epochs], rmse[:epochs]


def run_literal(prob: Problem, A, B, C, G, epochs: int, start_epoch: int = 0):
    """Algorithm 1 read literally on one core (per-nonzero C and G steps,
    nonzeros and edges interleaved in a seeded random order); the comparison
    run for the stratified schedule.  Returns (A, B, C, G, loss[], rmse[])."""
    lib = _load()
    I1, I2, I3 = prob.dims
    J1, J2, J3 = prob.ranks
    A = _f64(A, (I1, J1)); B = _f64(B, (I2, J2)); C = _f64(C, (I3, J3)); G = _f64(G, (J1, J2, J3))
    loss = np.zeros(max(epochs, 1)); rmse = np.zeros(max(epochs, 1))
    s = prob._c()
    rc = lib.oracle_run_literal(ctypes.byref(s), A.ctypes.data, B.ctypes.data, C.ctypes.data, G.ctypes.data,
                                int(start_epoch), int(epochs), loss.ctypes.data, rmse.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return A, B, C, G, loss[:epochs], rmse[:epochs]


LITERAL_STREAM = 1 << 32  # stream offset of the literal run's visiting order


def loss(prob: Problem, A, B, C, G):
    """(f_opt, rmse, parts) at the given factors, from the C definition."""
    lib = _load()
    I1, I2, I3 = prob.dims
    J1, J2, J3 = prob.ranks
    A = _f64(A, (I1, J1)); B = _f64(B, (I2, J2)); C = _f64(C, (I3, J3)); G = _f64(G, (J1, J2, J3))
    r = ctypes.c_double(0.0)
    parts = np.zeros(3)
    s = prob._c()
    f = lib.oracle_loss(ctypes.byref(s), A.ctypes.data, B.ctypes.data, C.ctypes.data, G.ctypes.data,
                        ctypes.addressof(r), parts.ctypes.data)
    return float(f), float(r.value), parts


def model_values(prob: Problem, A, B, C, G):
    lib = _load()
    I1, I2, I3 = prob.dims
    J1, J2, J3 = prob.ranks
    A = _f64(A, (I1, J1)); B = _f64(B, (I2, J2)); C = _f64(C, (I3, J3)); G = _f64(G, (J1, J2, J3))
    out = np.zeros(prob.nnz)
    s = prob._c()
    lib.oracle_model_values(ctypes.byref(s), A.ctypes.data, B.ctypes.data, C.ctypes.data,
                            G.ctypes.data, out.ctypes.data)
    return out


def plan_export(prob: Problem, epoch: int = 0):
    """The oracle's plan: dict of perm1, perm2, order, tile_start, block_tile, strata."""
    lib = _load()
    I1, I2, _ = prob.dims
    P = prob.P
    perm1 = np.zeros(I1, np.int32); perm2 = np.zeros(I2, np.int32)
    order = np.zeros(max(prob.nnz, 1), np.int64)
    tile_start = np.zeros(prob.nnz + 1, np.int64)
    block_tile = np.zeros(P * P + 1, np.int64)
    strata = np.zeros(P, np.int32)
    nt = ctypes.c_int64(0)
    s = prob._c()
    rc = lib.oracle_plan_export(ctypes.byref(s), int(epoch), perm1.ctypes.data, perm2.ctypes.data,
                                order.ctypes.data, tile_start.ctypes.data, block_tile.ctypes.data,
                                strata.ctypes.data, ctypes.addressof(nt))
    if rc != 0:
        raise OracleError(rc)
    n = nt.value
    return dict(perm1=perm1, perm2=perm2, order=order[:prob.nnz], tile_start=tile_start[: n + 1],
                block_tile=block_tile, strata=strata)


def random_start(prob: Problem):
    """Algorithm 1's random start as read here: A, B, C, G i.i.d.
    N(0, sigma^2), sigma = (mean x^2 / (J1 J2 J3))^(1/8), Box-Muller normals
    from stream 2^40 of the plan seed (see oracle_random_start)."""
    lib = _load()
    I1, I2, I3 = prob.dims
    J1, J2, J3 = prob.ranks
    A = np.zeros((I1, J1)); B = np.zeros((I2, J2)); C = np.zeros((I3, J3)); G = np.zeros((J1, J2, J3))
    s = prob._c()
    lib.oracle_random_start(ctypes.byref(s), A.ctypes.data, B.ctypes.data, C.ctypes.data, G.ctypes.data)
    return A, B, C, G


def splitmix64_at(seed: int, n: int) -> int:
    return int(_load().oracle_splitmix64_at(seed & 0xFFFFFFFFFFFFFFFF, n))


def shuffle(n: int, seed: int, stream: int) -> np.ndarray:
    a = np.arange(n, dtype=np.int32)
    _load().oracle_shuffle(a.ctypes.data, n, seed & 0xFFFFFFFFFFFFFFFF, stream)
    return a


def num_threads() -> int:
    return int(_load().oracle_num_threads())


# ---------------------------------------------------------------------------
# Plain numpy definitions (tiny inputs)
# ---------------------------------------------------------------------------
def mode_product(X: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """Eq. (1): (X x_n M)[..., j, ...] = sum_{i_n} X[..., i_n, ...] M[j, i_n]."""
    Y = np.tensordot(X, M, axes=([n], [1]))   # contracted axis moves to the end
    return np.moveaxis(Y, -1, n)


def dense_model(G, A, B, C) -> np.ndarray:
    """Eq. (2): G x1 A x2 B x3 C as a dense I1 x I2 x I3 array."""
    return mode_product(mode_product(mode_product(np.asarray(G, np.float64), A, 0), B, 1), C, 2)


def f_opt_dense(prob: Problem, A, B, C, G) -> float:
    """Eq. (3) + lambda_g Eq. (4) from the dense model; R sums |G|^2 and the
    rows that carry at least one observed cell."""
    X = dense_model(G, A, B, C)
    e = prob.x - X[prob.i, prob.j, prob.k]
    reg = float(np.sum(np.asarray(G) ** 2))
    reg += float(np.sum(np.asarray(A)[np.unique(prob.i)] ** 2))
    reg += float(np.sum(np.asarray(B)[np.unique(prob.j)] ** 2))
    reg += float(np.sum(np.asarray(C)[np.unique(prob.k)] ** 2))
    w = np.ones(prob.eu.shape[0]) if prob.ew is None else prob.ew
    d = np.asarray(B)[prob.eu] - np.asarray(B)[prob.ev]
    net = float(np.sum(w * np.sum(d * d, axis=1)))
    return 0.5 * float(e @ e) + 0.5 * prob.lam * reg + 0.5 * prob.lam_g * net


def f_split(prob: Problem, A, B, C, G, subset=None) -> float:
    """The per-nonzero (SGD-amenable) split of f in Section 2.3.2, summed over
    `subset` (indices into the nonzeros; all by default):
      1/2 sum_t [ e_t^2 + lambda/|Omega| |G|^2 + lambda sum_n |u_n|^2 / n_n ]
    with the slice counts n_n taken over the whole tensor."""
    I1, I2, I3 = prob.dims
    n1 = np.bincount(prob.i, minlength=I1)
    n2 = np.bincount(prob.j, minlength=I2)
    n3 = np.bincount(prob.k, minlength=I3)
    idx = np.arange(prob.nnz) if subset is None else np.asarray(subset)
    X = dense_model(G, A, B, C)
    ii, jj, kk = prob.i[idx], prob.j[idx], prob.k[idx]
    e = prob.x[idx] - X[ii, jj, kk]
    A = np.asarray(A); B = np.asarray(B); C = np.asarray(C)
    per = (e * e + prob.lam / prob.nnz * float(np.sum(np.asarray(G) ** 2))
           + prob.lam * (np.sum(A[ii] ** 2, 1) / n1[ii] + np.sum(B[jj] ** 2, 1) / n2[jj]
                         + np.sum(C[kk] ** 2, 1) / n3[kk]))
    return 0.5 * float(np.sum(per))


def fd_grad(fun, X: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of a scalar function of the array X."""
    X = np.array(X, dtype=np.float64, copy=True)
    g = np.zeros_like(X)
    flat = X.reshape(-1)
    gf = g.reshape(-1)
    for q in range(flat.shape[0]):
        old = flat[q]
        flat[q] = old + h
        fp = fun(X)
        flat[q] = old - h
        fm = fun(X)
        flat[q] = old
        gf[q] = (fp - fm) / (2 * h)
    return g


def laplacian_dense(I2: int, eu, ev, ew=None) -> np.ndarray:
    """L = D - W of the undirected gene graph (repeated pairs add up)."""
    W = np.zeros((I2, I2))
    w = np.ones(len(eu)) if ew is None else np.asarray(ew, np.float64)
    np.add.at(W, (np.asarray(eu), np.asarray(ev)), w)
    np.add.at(W, (np.asarray(ev), np.asarray(eu)), w)
    return np.diag(W.sum(1)) - W


# ---------------------------------------------------------------------------
# Fold-in of a new patient (Eq. 6) and top-k search (Section 3.2.1)
# ---------------------------------------------------------------------------
def fold_in(B, C, G, j, k, x, lam: float = 0.0) -> np.ndarray:
    """u = argmin_u 1/2 |x - W u|^2 + lam/2 |u|^2 with row (j,k) of W equal to
    G x2 b_j x3 c_k (Eq. 6 with the fixed B, C, G), solved as an augmented
    ordinary least-squares problem with numpy.linalg.lstsq."""
    G = np.asarray(G, np.float64)
    J1 = G.shape[0]
    Bj = np.asarray(B, np.float64)[np.asarray(j)]
    Ck = np.asarray(C, np.float64)[np.asarray(k)]
    W = np.einsum("abc,nb,nc->na", G, Bj, Ck)
    Wa = np.vstack([W, np.sqrt(lam) * np.eye(J1)])
    xa = np.concatenate([np.asarray(x, np.float64), np.zeros(J1)])
    u, *_ = np.linalg.lstsq(Wa, xa, rcond=None)
    return u


def topk_cosine(A, u, k: int = 10):
    """Indices of the k rows of A with the largest cosine similarity to u;
    zero-norm rows are skipped and ties go to the lower index."""
    A = np.asarray(A, np.float64)
    u = np.asarray(u, np.float64)
    na = np.linalg.norm(A, axis=1)
    nu = np.linalg.norm(u)
    valid = na > 0
    score = np.full(A.shape[0], -np.inf)
    if nu > 0:
        score[valid] = (A[valid] @ u) / (na[valid] * nu)
    order = np.lexsort((np.arange(A.shape[0]), -score))
    order = [int(t) for t in order if valid[t]][:k]
    return np.array(order, dtype=np.int64), score[order]


def qr_post(A, B, C, G):
    """Algorithm 1's last step: U = Q R per mode with a non-negative R
    diagonal, U <- Q, G <- G x_n R."""
    outs = []
    G = np.asarray(G, np.float64)
    for n, U in enumerate((A, B, C)):
        Q, R = np.linalg.qr(np.asarray(U, np.float64))
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        Q = Q * s
        R = R * s[:, None]
        outs.append(Q)
        G = mode_product(G, R, n)
    return outs[0], outs[1], outs[2], G
