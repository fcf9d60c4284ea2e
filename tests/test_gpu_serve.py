"""Fold-in / top-k server on the GPU against the oracle, alone vs. in the mix,
admission and error handling."""
import numpy as np
import pytest

import oracle
import snect_synth as synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_1711_08095_amd as sn
    ctx = sn.Context(0)
    rng = np.random.default_rng(5)
    I1, I2, I3, J = 700, 900, 5, (10, 10, 5)
    f = [rng.standard_normal((I1, J[0])) * 0.5, rng.standard_normal((I2, J[1])) * 0.5,
         rng.standard_normal((I3, J[2])) * 0.5, rng.standard_normal(J) * 0.5]
    f[0][13] = 0.0  # a zero-norm patient row is never returned
    f = [a.astype(np.float32) for a in f]
    t = [torch.tensor(a, device="cuda") for a in f]
    reqs = synth.fold_in_requests(seed=77, count=24, I2=I2, I3=I3, nnz_lo=1, nnz_hi=3000)
    yield ctx, f, t, reqs
    ctx.close()


def _oracle(f, r, lam, k=10):
    A, B, C, G = (np.asarray(a, np.float64) for a in f)
    u = oracle.fold_in(B, C, G, r["j"], r["k"], r["x"].astype(np.float64), lam=lam)
    idx, sc = oracle.topk_cosine(A, u, k)
    return u, idx, sc


U32 = 2.0 ** -24


def _tolerance(f, r, lam, uo):
    """Bounds on the server's errors, from its arithmetic.  The rows w of W
    are FP32 dot products of lengths J2 and J3, and Q = W^T W + lam I and
    r = W^T x are FP32 sums in fixed trees whose sequential chains are at
    most 256 terms inside a workgroup, the slices of a workgroup and 256
    partials: every entry of Q and r is off by at most
    gamma = (520 + 2 (J2 + J3 + 1)) u times the same sum of absolute values
    (u = 2^-24, first order).  The FP64 refinement then solves the formed
    system exactly, so |u - u_oracle| <= |Q^-1| (|dr| + |dQ| |u|).  The
    cosine scores use u rounded to FP32 and FP32 dot products of J1 terms:
    |d cos| <= 2 |du| / |u| + (J1 + 4) u.  A factor 2 covers the second-order
    terms."""
    B, C, G = (np.asarray(a, np.float64) for a in f[1:])
    J1, J2, J3 = G.shape
    j, k, x = np.asarray(r["j"]), np.asarray(r["k"]), np.asarray(r["x"], np.float64)
    W = np.einsum("abc,nb,nc->na", G, B[j], C[k])
    Wabs = np.einsum("abc,nb,nc->na", np.abs(G), np.abs(B[j]), np.abs(C[k]))
    gamma = (520 + 2 * (J2 + J3 + 1)) * U32
    Q = W.T @ W + lam * np.eye(J1)
    dQ = gamma * (Wabs.T @ Wabs)
    dr = gamma * (Wabs.T @ np.abs(x))
    qinv = np.linalg.norm(np.linalg.inv(Q), 2)
    tol_u = 2.0 * qinv * (np.linalg.norm(dr) + np.linalg.norm(dQ, 2) * np.linalg.norm(uo))
    tol_s = 2.0 * (2.0 * tol_u / max(np.linalg.norm(uo), 1e-300) + (J1 + 4) * U32)
    return tol_u, tol_s


def _check(f, r, got, lam):
    u, idx, sc = got
    uo, io, so = _oracle(f, r, lam)
    tol_u, tol_s = _tolerance(f, r, lam, uo)
    assert np.linalg.norm(u - uo) <= tol_u, (np.linalg.norm(u - uo), tol_u)
    np.testing.assert_allclose(sc, so, rtol=0, atol=tol_s)
    # the returned rows are a top set of the oracle's scores (rows whose
    # scores lie within the tolerance of each other may change places)
    A = np.asarray(f[0], np.float64)
    cos = (A @ uo) / (np.linalg.norm(A, axis=1) * np.linalg.norm(uo) + 1e-300)
    assert np.all(np.abs(cos[idx] - so) <= 2 * tol_s)


def test_fold_in_and_topk_match_oracle(setup):
    import paper_1711_08095_amd as sn
    ctx, f, t, reqs = setup
    srv = sn.Server(ctx, *t, max_slots=4, pg_iters=20, topk=10, lam=0.01)
    for r in reqs[:8]:
        tk = srv.submit(r["j"], r["k"], r["x"])
        got = None
        while got is None:
            got = srv.poll(tk)
        _check(f, r, got, 0.01)
    srv.close()


@pytest.mark.parametrize("I1,J", [(7000, (20, 8, 3)), (300, (32, 6, 2))])
def test_many_patients_and_full_rank(I1, J):
    """More patients than the scores kept in registers (global scores path),
    and the largest supported patient rank."""
    import torch
    import paper_1711_08095_amd as sn
    rng = np.random.default_rng(11)
    I2, I3 = 400, 3
    f = [rng.standard_normal((I1, J[0])) * 0.5, rng.standard_normal((I2, J[1])) * 0.5,
         rng.standard_normal((I3, J[2])) * 0.5, rng.standard_normal(J) * 0.5]
    f[0][I1 - 2] = 0.0
    f = [a.astype(np.float32) for a in f]
    ctx = sn.Context(0)
    t = [torch.tensor(a, device="cuda") for a in f]
    srv = sn.Server(ctx, *t, max_slots=2, pg_iters=20, topk=10, lam=0.01)
    for r in synth.fold_in_requests(seed=78, count=4, I2=I2, I3=I3, nnz_lo=200, nnz_hi=1200):
        tk = srv.submit(r["j"], r["k"], r["x"])
        got = None
        while got is None:
            got = srv.poll(tk)
        _check(f, r, got, 0.01)
    srv.close()
    ctx.close()


@pytest.mark.parametrize("J", [(10, 10, 5), (20, 20, 5)])
def test_large_requests_alone_and_in_the_mix(J):
    """Requests of 30,000-60,000 cells (the serving workload's upper range,
    up to 256 partial sums per request) against the oracle, alone and
    overlapping, with bit-identical results both ways."""
    import torch
    import paper_1711_08095_amd as sn
    rng = np.random.default_rng(21)
    I1, I2, I3 = 900, 14000, 5
    f = [rng.standard_normal((I1, J[0])) * 0.5, rng.standard_normal((I2, J[1])) * 0.5,
         rng.standard_normal((I3, J[2])) * 0.5, rng.standard_normal(J) * 0.5]
    f = [a.astype(np.float32) for a in f]
    ctx = sn.Context(0)
    t = [torch.tensor(a, device="cuda") for a in f]
    reqs = synth.fold_in_requests(seed=79, count=4, I2=I2, I3=I3, nnz_lo=30000, nnz_hi=60000)
    print(f"large requests J={J}: nnz {[len(r['j']) for r in reqs]}", flush=True)
    srv = sn.Server(ctx, *t, max_slots=4, pg_iters=20, topk=10, lam=0.01)
    alone = []
    for r in reqs:
        tk = srv.submit(r["j"], r["k"], r["x"])
        got = None
        while got is None:
            got = srv.poll(tk)
        _check(f, r, got, 0.01)
        alone.append(got)
    tks = [srv.submit(r["j"], r["k"], r["x"]) for r in reqs]
    for a, tk in zip(alone, tks):
        got = None
        while got is None:
            got = srv.poll(tk)
        for x, y in zip(a, got):
            np.testing.assert_array_equal(x, y)
    srv.close()
    ctx.close()


def test_alone_equals_in_the_mix(setup):
    import paper_1711_08095_amd as sn
    ctx, f, t, reqs = setup
    srv = sn.Server(ctx, *t, max_slots=8, pg_iters=20, topk=10, lam=0.01)
    alone = []
    for r in reqs:
        tk = srv.submit(r["j"], r["k"], r["x"])
        got = None
        while got is None:
            got = srv.poll(tk)
        alone.append(got)
    # the same requests submitted as fast as slots allow, overlapping
    pending, mixed, nxt = {}, {}, 0
    while len(mixed) < len(reqs):
        while nxt < len(reqs):
            try:
                pending[srv.submit(reqs[nxt]["j"], reqs[nxt]["k"], reqs[nxt]["x"])] = nxt
                nxt += 1
            except sn.SnectError as e:
                assert e.code == -8
                break
        for tk in list(pending):
            got = srv.poll(tk)
            if got is not None:
                mixed[pending.pop(tk)] = got
    for a, (i, b) in zip(alone, sorted(mixed.items())):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    srv.close()


def test_replay_trace(setup):
    import paper_1711_08095_amd as sn
    ctx, f, t, reqs = setup
    srv = sn.Server(ctx, *t, max_slots=4, pg_iters=20, topk=10, lam=0.01)
    arr = np.array([r["arrival"] for r in reqs]) * 0.0  # all at once
    offs = np.concatenate([[0], np.cumsum([len(r["j"]) for r in reqs])])
    j = np.concatenate([r["j"] for r in reqs])
    k = np.concatenate([r["k"] for r in reqs])
    x = np.concatenate([r["x"] for r in reqs])
    out = srv.replay(arr, offs, j, k, x, gpu_busy=True)
    assert np.all(out["status"] == 0)
    assert np.all(out["latency_s"] >= 0)
    assert 0.0 < out["gpu_busy_s"] <= out["wall_s"]
    # the timed replay computes the same results as an untimed one
    out2 = srv.replay(arr, offs, j, k, x)
    np.testing.assert_array_equal(out["u"], out2["u"])
    np.testing.assert_array_equal(out["idx"], out2["idx"])
    for n in (0, 5, 23):
        _check(f, reqs[n], (out["u"][n], out["idx"][n], out["score"][n]), 0.01)
    srv.close()


def test_admission_and_errors(setup):
    import paper_1711_08095_amd as sn
    ctx, f, t, reqs = setup
    srv = sn.Server(ctx, *t, max_slots=2, pool_bytes=8192, pg_iters=5, topk=3, lam=0.0)
    with pytest.raises(sn.SnectError) as e:
        srv.submit(np.zeros(1000, np.int32), np.zeros(1000, np.int32), np.ones(1000, np.float32))
    assert e.value.code == -9  # larger than the whole pool
    with pytest.raises(sn.SnectError) as e:
        srv.submit(np.array([900], np.int32), np.array([0], np.int32), np.ones(1, np.float32))
    assert e.value.code == -2
    with pytest.raises(sn.SnectError) as e:
        srv.submit(np.array([3, 4], np.int32), np.array([0, 1], np.int32), np.array([1.0, np.nan], np.float32))
    assert e.value.code == -1  # non-finite value
    with pytest.raises(sn.SnectError) as e:
        srv.submit(np.array([3, 4], np.int32), np.array([0, -1], np.int32), np.ones(2, np.float32))
    assert e.value.code == -2  # negative platform
    # the same checks on cells inside the four-wide part of the pass and in its tail
    for pos in (0, 3, 6, 9):
        for field, bad, code in (("j", 900, -2), ("j", -5, -2), ("k", 5, -2), ("k", -1, -2), ("x", np.inf, -1),
                                 ("x", np.nan, -1)):
            cells = {"j": np.arange(11, dtype=np.int32) * 80, "k": np.arange(11, dtype=np.int32) % 5,
                     "x": np.ones(11, np.float32)}
            cells[field][pos] = bad
            with pytest.raises(sn.SnectError) as e:
                srv.submit(cells["j"], cells["k"], cells["x"])
            assert e.value.code == code, (pos, field, bad)
    # cells at the upper limits are admitted (with lam = 0 and five distinct
    # cells the system is singular, which the poll reports)
    tk = srv.submit(np.full(11, 899, np.int32), np.arange(11, dtype=np.int32) % 5, np.ones(11, np.float32))
    with pytest.raises(sn.SnectError) as e:
        while srv.poll(tk) is None:
            pass
    assert e.value.code == -1
    # lambda = 0 and a single cell: the system is singular, that request fails alone
    tk_bad = srv.submit(np.array([3], np.int32), np.array([1], np.int32), np.ones(1, np.float32))
    r = reqs[1]
    n = min(len(r["j"]), 200)
    tk_ok = srv.submit(r["j"][:n], r["k"][:n], r["x"][:n])
    with pytest.raises(sn.SnectError) as e:
        while srv.poll(tk_bad) is None:
            pass
    assert e.value.code == -1
    got = None
    while got is None:
        got = srv.poll(tk_ok)
    sub = dict(j=r["j"][:n], k=r["k"][:n], x=r["x"][:n])
    uo = oracle.fold_in(*(np.asarray(a, np.float64) for a in f[1:]), sub["j"], sub["k"],
                        sub["x"].astype(np.float64), lam=0.0)
    assert np.linalg.norm(got[0] - uo) <= _tolerance(f, sub, 0.0, uo)[0]
    srv.close()
