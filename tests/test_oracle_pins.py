"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
generator outputs, a hand-worked example, closed forms (identity factors,
rank-one cores, a matrix power of the graph Laplacian), library routines
(numpy.linalg, scipy's graph Laplacian), finite-difference gradients of the
objective, and textbook SGD written out separately.
"""
import json
import os

import numpy as np
import pytest

import oracle
import snect_synth as synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed=0, dims=(6, 7, 1), ranks=(2, 3, 2), nnz=20, lam=0.3, lam_g=0.0, lr=0.05,
          cls=1.0, P=1, T=1000, edges=0, scale=0.5):
    rng = np.random.default_rng(seed)
    I1, I2, I3 = dims
    cells = synth.sample_cells(rng, I1 * I2 * I3, nnz)
    i = (cells // (I2 * I3)).astype(np.int32)
    j = ((cells // I3) % I2).astype(np.int32)
    k = (cells % I3).astype(np.int32)
    x = rng.standard_normal(nnz)
    if edges:
        eu, ev = synth.erdos_renyi_edges(rng, I2, edges)
        ew = rng.uniform(0.5, 2.0, size=edges)
    else:
        eu = ev = np.zeros(0, np.int32)
        ew = None
    A, B, C, G = synth.normal_init(seed + 1, dims, ranks, scale)
    prob = oracle.Problem(dims, ranks, i, j, k, x, eu, ev, ew, lam=lam, lam_g=lam_g, lr=lr,
                          core_lr_scale=cls, P=P, T=T, seed=seed + 7)
    return prob, (A, B, C, G)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


# --------------------------------------------------------------------------
# Random streams
# --------------------------------------------------------------------------
def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [oracle.splitmix64_at(0, n) for n in range(3)] == vals


def test_splitmix64_state_advances_by_the_increment():
    # output n from the closed form equals n + 1 steps of the recurrence,
    # stepped here in plain Python integers
    mask = (1 << 64) - 1

    def steps(seed, n):
        s, z = seed, 0
        for _ in range(n + 1):
            s = (s + 0x9E3779B97F4A7C15) & mask
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
            z ^= z >> 31
        return z

    for seed in (0, 1, 3003, (1 << 64) - 5):
        for n in (0, 1, 2, 17, 200):
            assert oracle.splitmix64_at(seed, n) == steps(seed, n)


def _start_problem(x_scale=1.0, ranks=(3, 4, 2), seed=11, dims=(300, 400, 5), nnz=3000):
    rng = np.random.default_rng(seed)
    I1, I2, I3 = dims
    cells = synth.sample_cells(rng, I1 * I2 * I3, nnz)
    x = x_scale * rng.standard_normal(nnz)
    return oracle.Problem(dims, ranks, cells // (I2 * I3), (cells // I3) % I2, cells % I3, x, seed=seed)


def test_random_start_is_normal_with_the_stated_sigma():
    from scipy import stats
    prob = _start_problem()
    A, B, C, G = oracle.random_start(prob)
    z = np.concatenate([a.ravel() for a in (A, B, C, G)])
    J = np.prod(prob.ranks)
    sigma = (np.mean(prob.x ** 2) / J) ** 0.125
    # Kolmogorov-Smirnov against N(0, sigma^2) on 2,530 draws
    assert stats.kstest(z, "norm", args=(0.0, sigma)).pvalue > 1e-3
    assert abs(z.std() / sigma - 1.0) < 0.06
    assert abs(z.mean()) < 4 * sigma / np.sqrt(z.size)
    # cos and sin halves of a pair are uncorrelated
    n2 = z.size // 2 * 2
    assert abs(np.corrcoef(z[0:n2:2], z[1:n2:2])[0, 1]) < 0.1
    # same seed, same draw; another seed, another draw
    again = oracle.random_start(prob)
    for u, v in zip((A, B, C, G), again):
        np.testing.assert_array_equal(u, v)
    other = _start_problem(seed=12)
    assert not np.allclose(oracle.random_start(other)[0][:5], A[:5])


def test_random_start_sigma_scales_with_the_data_and_the_core():
    # the standard normals do not depend on the data: scaling x by s scales
    # sigma, and so every entry, by s^(1/4); a core with 16 times as many
    # entries divides sigma by 16^(1/8)
    base = oracle.random_start(_start_problem())
    scaled = oracle.random_start(_start_problem(x_scale=16.0))
    for u, v in zip(base, scaled):
        np.testing.assert_allclose(v, 2.0 * u, rtol=1e-13)
    big = _start_problem(ranks=(12, 8, 4))
    small = _start_problem(ranks=(3, 4, 2))
    a_big = oracle.random_start(big)[0]
    a_small = oracle.random_start(small)[0]
    # A is drawn first, so its first 3 columns' worth of draws coincide
    np.testing.assert_allclose(a_big.ravel()[:12] * 16.0 ** 0.125, a_small.ravel()[:12], rtol=1e-13)
    # no data: sigma = 1
    empty = oracle.Problem((4, 5, 2), (2, 2, 2), np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), seed=11)
    e = oracle.random_start(empty)
    assert 0.3 < np.concatenate([a.ravel() for a in e]).std() < 2.0


def test_shuffle_is_a_uniform_permutation():
    for n in (1, 2, 5, 97):
        s = oracle.shuffle(n, 123, 4)
        assert sorted(s.tolist()) == list(range(n))
    # all 6 orders of 3 items, 6000 independent streams: chi-square, 5 dof
    counts = {}
    for t in range(6000):
        key = tuple(oracle.shuffle(3, 99, t).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    chi2 = sum((c - 1000.0) ** 2 / 1000.0 for c in counts.values())
    assert chi2 < 20.5  # p ~ 0.001


# --------------------------------------------------------------------------
# Model value (Eq. 2) and objective (Eq. 3, 4)
# --------------------------------------------------------------------------
def test_model_identity_factors_give_core():
    J = (3, 4, 2)
    G = np.random.default_rng(1).standard_normal(J)
    A, B, C = np.eye(3), np.eye(4), np.eye(2)
    X = oracle.dense_model(G, A, B, C)
    np.testing.assert_array_equal(X, G)
    ii, jj, kk = np.meshgrid(range(3), range(4), range(2), indexing="ij")
    prob = oracle.Problem(J, J, ii.ravel(), jj.ravel(), kk.ravel(), np.zeros(24))
    np.testing.assert_allclose(oracle.model_values(prob, A, B, C, G), G.ravel(), atol=1e-15)


def test_model_rank_one_core():
    rng = np.random.default_rng(2)
    dims, J = (5, 6, 3), (3, 4, 2)
    A, B, C = (rng.standard_normal((d, r)) for d, r in zip(dims, J))
    G = np.zeros(J)
    G[2, 1, 0] = 1.7
    X = oracle.dense_model(G, A, B, C)
    ref = 1.7 * np.einsum("i,j,k->ijk", A[:, 2], B[:, 1], C[:, 0])
    np.testing.assert_allclose(X, ref, rtol=1e-14, atol=1e-14)
    ii, jj, kk = np.meshgrid(range(5), range(6), range(3), indexing="ij")
    prob = oracle.Problem(dims, J, ii.ravel(), jj.ravel(), kk.ravel(), np.zeros(90))
    np.testing.assert_allclose(oracle.model_values(prob, A, B, C, G), ref.ravel(), rtol=1e-13,
                               atol=1e-14)


def test_model_c_matches_dense_definition():
    prob, (A, B, C, G) = _tiny(dims=(9, 8, 4), ranks=(3, 2, 3), nnz=120)
    X = oracle.dense_model(G, A, B, C)
    np.testing.assert_allclose(oracle.model_values(prob, A, B, C, G), X[prob.i, prob.j, prob.k],
                               rtol=1e-12, atol=1e-14)


def test_loss_hand_worked_example():
    g = json.load(open(os.path.join(GOLD, "loss_hand.json")))
    prob = oracle.Problem(g["dims"], g["ranks"], g["i"], g["j"], g["k"], g["x"], g["eu"], g["ev"],
                          g["ew"], lam=g["lam"], lam_g=g["lam_g"])
    f, r, _ = oracle.loss(prob, g["A"], g["B"], g["C"], g["G"])
    assert f == pytest.approx(g["f"], rel=1e-14)
    assert r == pytest.approx(g["rmse"], rel=1e-14)
    assert oracle.f_opt_dense(prob, np.array(g["A"]), np.array(g["B"]), np.array(g["C"]),
                              np.array(g["G"])) == pytest.approx(g["f"], rel=1e-14)


def test_network_term_is_laplacian_quadratic_form():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import laplacian
    prob, (A, B, C, G) = _tiny(dims=(5, 30, 2), ranks=(2, 3, 2), nnz=0, lam=0.0, lam_g=0.7,
                               edges=60)
    # repeat three pairs, one of them reversed: their weights must add up
    prob.eu = np.concatenate([prob.eu, prob.eu[:2], prob.ev[2:3]]).astype(np.int32)
    prob.ev = np.concatenate([prob.ev, prob.ev[:2], prob.eu[2:3]]).astype(np.int32)
    prob.ew = np.concatenate([prob.ew, [0.25, 0.5, 1.0]])
    W = coo_matrix((np.concatenate([prob.ew, prob.ew]),
                    (np.concatenate([prob.eu, prob.ev]), np.concatenate([prob.ev, prob.eu]))),
                   shape=(30, 30)).toarray()
    L = laplacian(W)
    f, _, parts = oracle.loss(prob, A, B, C, G)
    assert parts[2] == pytest.approx(0.5 * 0.7 * np.trace(B.T @ L @ B), rel=1e-12)
    assert parts[0] == 0.0 and parts[1] == 0.0


def test_split_objective_sums_to_f():
    prob, (A, B, C, G) = _tiny(dims=(7, 9, 3), ranks=(2, 3, 2), nnz=70, lam=0.4)
    f_c, _, _ = oracle.loss(prob, A, B, C, G)
    assert oracle.f_split(prob, A, B, C, G) == pytest.approx(f_c, rel=1e-12)
    assert oracle.f_opt_dense(prob, A, B, C, G) == pytest.approx(f_c, rel=1e-12)


def test_fd_gradient_of_a_quadratic():
    M = np.array([[2.0, 1.0], [1.0, 3.0]])
    x0 = np.array([0.3, -0.7])
    g = oracle.fd_grad(lambda v: 0.5 * v @ M @ v, x0)
    np.testing.assert_allclose(g, M @ x0, rtol=1e-8)


# --------------------------------------------------------------------------
# The iteration, pinned by finite-difference gradients of the objective
# --------------------------------------------------------------------------
def _grads(fun, A, B, C, G):
    gA = oracle.fd_grad(lambda X: fun(X, B, C, G), A)
    gB = oracle.fd_grad(lambda X: fun(A, X, C, G), B)
    gC = oracle.fd_grad(lambda X: fun(A, B, X, G), C)
    gG = oracle.fd_grad(lambda X: fun(A, B, C, X), G)
    return gA, gB, gC, gG


def test_single_tile_epoch_is_a_full_gradient_step():
    # one platform, one block, a tile holding every nonzero: one epoch is one
    # gradient step on f (factor rows, step eta) and one mean-gradient step on
    # C and G (step eta * core_lr_scale / nnz)
    prob, (A, B, C, G) = _tiny(dims=(6, 7, 1), ranks=(2, 3, 2), nnz=25, lam=0.3, lr=0.05, cls=3.0)
    A1, B1, C1, G1, _, _ = oracle.run(prob, A, B, C, G, 1)
    f = lambda a, b, c, g: oracle.f_opt_dense(prob, a, b, c, g)
    gA, gB, gC, gG = _grads(f, A, B, C, G)
    eta, etac = prob.lr, prob.lr * prob.core_lr_scale / prob.nnz
    assert _rel(A1, A - eta * gA) < 1e-7
    assert _rel(B1, B - eta * gB) < 1e-7
    assert _rel(C1, C - etac * gC) < 1e-7
    assert _rel(G1, G - etac * gG) < 1e-7


def test_platform_slices_run_in_order():
    # one block, three platforms: one tile per platform in ascending k, each a
    # gradient step on the split objective restricted to that slice, with the
    # core step taking the mean of the slice gradients at the rows each saw
    prob, (A, B, C, G) = _tiny(dims=(6, 7, 3), ranks=(2, 3, 2), nnz=40, lam=0.2, lr=0.04, cls=2.0)
    A1, B1, C1, G1, _, _ = oracle.run(prob, A, B, C, G, 1)
    a, b = A.copy(), B.copy()
    sC = np.zeros_like(C)
    sG = np.zeros_like(G)
    for kk in range(3):
        sub = np.nonzero(prob.k == kk)[0]
        f = lambda a_, b_, c_, g_: oracle.f_split(prob, a_, b_, c_, g_, sub)
        gA, gB, gC, gG = _grads(f, a, b, C, G)
        sC += gC
        sG += gG
        a, b = a - prob.lr * gA, b - prob.lr * gB
    etac = prob.lr * prob.core_lr_scale / prob.nnz
    assert _rel(A1, a) < 1e-7 and _rel(B1, b) < 1e-7
    assert _rel(C1, C - etac * sC) < 1e-7
    assert _rel(G1, G - etac * sG) < 1e-7


def test_strata_with_network_step():
    # P = 3 row/column blocks, one platform, one tile per block: the epoch is a
    # network Jacobi step on B, then one gradient step per stratum (in the
    # plan's stratum order) on the nonzeros of that stratum, each followed by
    # the mean-gradient core step
    prob, (A, B, C, G) = _tiny(dims=(9, 12, 1), ranks=(2, 2, 2), nnz=60, lam=0.2, lam_g=0.3,
                               lr=0.03, cls=2.0, P=3, edges=20)
    A1, B1, C1, G1, _, _ = oracle.run(prob, A, B, C, G, 1)
    plan = oracle.plan_export(prob, epoch=0)
    I1, I2, _ = prob.dims
    pos1 = np.argsort(plan["perm1"])
    pos2 = np.argsort(plan["perm2"])
    blk1 = pos1 * prob.P // I1
    blk2 = pos2 * prob.P // I2
    stratum = (blk2[prob.j] - blk1[prob.i]) % prob.P
    L = oracle.laplacian_dense(I2, prob.eu, prob.ev, prob.ew)
    assert 2 * prob.lr * prob.lam_g * np.max(np.diag(L)) <= 1.0  # a single sub-step
    a, b, c, g = A.copy(), B - prob.lr * prob.lam_g * (L @ B), C.copy(), G.copy()
    for s in plan["strata"]:
        sub = np.nonzero(stratum == s)[0]
        if sub.size == 0:
            continue
        f = lambda a_, b_, c_, g_: oracle.f_split(prob, a_, b_, c_, g_, sub)
        gA, gB, gC, gG = _grads(f, a, b, c, g)
        etac = prob.lr * prob.core_lr_scale / sub.size
        a, b, c, g = a - prob.lr * gA, b - prob.lr * gB, c - etac * gC, g - etac * gG
    assert _rel(A1, a) < 1e-7 and _rel(B1, b) < 1e-7
    assert _rel(C1, c) < 1e-7 and _rel(G1, g) < 1e-7


def test_graph_only_is_a_laplacian_matrix_power():
    for lr, lam_g, epochs in ((0.05, 0.4, 3), (0.3, 1.0, 2)):
        prob, (A, B, C, G) = _tiny(dims=(4, 25, 2), ranks=(2, 3, 2), nnz=0, lam=0.0, lam_g=lam_g,
                                   lr=lr, edges=50, P=2)
        L = oracle.laplacian_dense(25, prob.eu, prob.ev, prob.ew)
        nsub = max(1, int(np.ceil(2 * lr * lam_g * np.max(np.diag(L)))))
        M = np.eye(25) - (lr * lam_g / nsub) * L
        _, B1, C1, G1, _, _ = oracle.run(prob, A, B, C, G, epochs)
        np.testing.assert_allclose(B1, np.linalg.matrix_power(M, nsub * epochs) @ B, rtol=1e-12,
                                   atol=1e-13)
        np.testing.assert_allclose(B1.sum(0), B.sum(0), rtol=1e-12, atol=1e-12)
        np.testing.assert_array_equal(C1, C)
        np.testing.assert_array_equal(G1, G)
    assert nsub > 1  # the second case exercises sub-stepping


def test_matrix_factorisation_special_case_is_textbook_sgd():
    # I3 = J3 = 1, C = [1], G = identity and a frozen core: the model is
    # x_ij ~ a_i . b_j and the iteration with T = 1, P = 1 is plain
    # matrix-factorisation SGD over the nonzeros sorted by (i, j)
    rng = np.random.default_rng(5)
    I1, I2, J = 8, 9, 3
    cells = synth.sample_cells(rng, I1 * I2, 40)
    i, j = (cells // I2).astype(np.int32), (cells % I2).astype(np.int32)
    x = rng.standard_normal(40)
    A = rng.standard_normal((I1, J)) * 0.5
    B = rng.standard_normal((I2, J)) * 0.5
    C = np.ones((1, 1))
    G = np.eye(J).reshape(J, J, 1)
    lam, lr = 0.3, 0.07
    prob = oracle.Problem((I1, I2, 1), (J, J, 1), i, j, np.zeros(40, np.int32), x, lam=lam,
                          lr=lr, core_lr_scale=0.0, P=1, T=1)
    A1, B1, C1, G1, _, _ = oracle.run(prob, A, B, C, G, 2)
    n1 = np.bincount(i, minlength=I1)
    n2 = np.bincount(j, minlength=I2)
    a, b = A.copy(), B.copy()
    order = np.lexsort((j, i))
    for _ in range(2):
        for t in order:
            u, v = i[t], j[t]
            err = x[t] - a[u] @ b[v]
            au, bv = a[u].copy(), b[v].copy()
            a[u] = au + lr * (err * bv - lam / n1[u] * au)
            b[v] = bv + lr * (err * au - lam / n2[v] * bv)
    np.testing.assert_allclose(A1, a, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(B1, b, rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(C1, C)
    np.testing.assert_array_equal(G1, G)


def test_tucker_sequential_sgd_with_intermediate_tensor():
    # T = 1, P = 1, frozen core: Algorithm 1's per-nonzero factor updates with
    # the cached tensor D = G * (a o b o c); the gradient for mode n is the
    # sum of D over the other modes divided by u_n (written here without the
    # division, as G contracted with the other two rows)
    prob, (A, B, C, G) = _tiny(dims=(5, 6, 3), ranks=(2, 3, 2), nnz=30, lam=0.2, lr=0.05, cls=0.0,
                               P=1, T=1)
    A1, B1, C1, G1, _, _ = oracle.run(prob, A, B, C, G, 1)
    n1 = np.bincount(prob.i, minlength=5)
    n2 = np.bincount(prob.j, minlength=6)
    a, b = A.copy(), B.copy()
    for t in np.lexsort((prob.j, prob.i, prob.k)):
        u, v, w = prob.i[t], prob.j[t], prob.k[t]
        D = G * np.einsum("p,q,r->pqr", a[u], b[v], C[w])
        err = prob.x[t] - D.sum()
        ga = np.einsum("pqr,q,r->p", G, b[v], C[w])
        gb = np.einsum("pqr,p,r->q", G, a[u], C[w])
        au, bv = a[u].copy(), b[v].copy()
        a[u] = au + prob.lr * (err * ga - prob.lam / n1[u] * au)
        b[v] = bv + prob.lr * (err * gb - prob.lam / n2[v] * bv)
    np.testing.assert_allclose(A1, a, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(B1, b, rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(C1, C)
    np.testing.assert_array_equal(G1, G)


def test_planted_truth_is_a_fixed_point():
    p = synth.planted(seed=11, dims=(30, 40, 3), ranks=(3, 3, 2), nnz=800, edges=0)
    pr0 = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, np.zeros(800))
    x = oracle.model_values(pr0, p.A, p.B, p.C, p.G)
    prob = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, x, lam=0.0, lam_g=0.0, lr=1e-3, P=4,
                          T=16, seed=5)
    A1, B1, C1, G1, loss, rmse = oracle.run(prob, p.A, p.B, p.C, p.G, 2)
    for u, v in ((A1, p.A), (B1, p.B), (C1, p.C), (G1, p.G)):
        np.testing.assert_allclose(u, v, rtol=0, atol=1e-11)
    assert rmse[-1] < 1e-12


def test_loss_decreases_on_planted_tensor():
    p = synth.planted()
    pr0 = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, np.zeros(len(p.i)))
    x = oracle.model_values(pr0, p.A, p.B, p.C, p.G) + p.noise
    prob = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, x, p.eu, p.ev, lam=0.01, lam_g=0.1,
                          lr=1e-3, P=8, T=64, seed=synth.PLAN_SEED)
    A, B, C, G = synth.normal_init(synth.INIT_SEED, p.dims, p.ranks, 1.0)
    f0, _, _ = oracle.loss(prob, A, B, C, G)
    *_, loss, rmse = oracle.run(prob, A, B, C, G, 10)
    seq = np.concatenate([[f0], loss])
    assert np.all(np.diff(seq) < 0)


def test_thread_count_does_not_change_bits():
    prob, (A, B, C, G) = _tiny(dims=(40, 50, 4), ranks=(3, 4, 2), nnz=900, lam=0.05, lam_g=0.1,
                               lr=0.01, P=5, T=8, edges=40)
    r1 = oracle.run(prob, A, B, C, G, 2, threads=1)
    r8 = oracle.run(prob, A, B, C, G, 2, threads=8)
    for u, v in zip(r1, r8):
        np.testing.assert_array_equal(u, v)


def test_resume_matches_uninterrupted_run():
    prob, (A, B, C, G) = _tiny(dims=(40, 50, 4), ranks=(3, 4, 2), nnz=900, lam=0.05, lam_g=0.1,
                               lr=0.01, P=5, T=8, edges=40)
    full = oracle.run(prob, A, B, C, G, 4)
    half = oracle.run(prob, A, B, C, G, 2)
    rest = oracle.run(prob, *half[:4], 2, start_epoch=2)
    for u, v in zip(full[:4], rest[:4]):
        np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(full[4], np.concatenate([half[4], rest[4]]))


# --------------------------------------------------------------------------
# Plan invariants and input validation
# --------------------------------------------------------------------------
def test_plan_invariants():
    prob, _ = _tiny(dims=(23, 31, 4), ranks=(2, 2, 2), nnz=500, P=4, T=7)
    plan = oracle.plan_export(prob, epoch=3)
    P, T = prob.P, prob.T
    assert sorted(plan["order"].tolist()) == list(range(prob.nnz))
    assert sorted(plan["strata"].tolist()) == list(range(P))
    I1, I2, _ = prob.dims
    blk1 = np.argsort(plan["perm1"]) * P // I1
    blk2 = np.argsort(plan["perm2"]) * P // I2
    # block sizes differ by at most one row
    assert np.ptp(np.bincount(blk1, minlength=P)) <= 1
    assert np.ptp(np.bincount(blk2, minlength=P)) <= 1
    ts, bt, order = plan["tile_start"], plan["block_tile"], plan["order"]
    for b in range(P * P):
        p, q = divmod(b, P)
        for tl in range(bt[b], bt[b + 1]):
            ids = order[ts[tl]:ts[tl + 1]]
            assert 1 <= ids.size <= T
            assert np.all(blk1[prob.i[ids]] == p) and np.all(blk2[prob.j[ids]] == q)
            assert np.unique(prob.k[ids]).size == 1
        ids = order[ts[bt[b]]:ts[bt[b + 1]]] if bt[b + 1] > bt[b] else order[:0]
        keys = list(zip(prob.k[ids], prob.i[ids], prob.j[ids]))
        assert keys == sorted(keys)
    # different epochs give different stratum orders (P = 4: 24 orders)
    orders = {tuple(oracle.plan_export(prob, epoch=e)["strata"]) for e in range(12)}
    assert len(orders) > 3


def test_validation_errors():
    prob, (A, B, C, G) = _tiny(dims=(6, 7, 2), nnz=10)
    dup = oracle.Problem(prob.dims, prob.ranks, np.r_[prob.i, prob.i[:1]],
                         np.r_[prob.j, prob.j[:1]], np.r_[prob.k, prob.k[:1]],
                         np.r_[prob.x, 1.0])
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(dup, A, B, C, G, 1)
    assert e.value.code == -3
    bad = oracle.Problem(prob.dims, prob.ranks, np.r_[prob.i, 6], np.r_[prob.j, 0],
                         np.r_[prob.k, 0], np.r_[prob.x, 1.0])
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(bad, A, B, C, G, 1)
    assert e.value.code == -2
    big_p = oracle.Problem(prob.dims, prob.ranks, prob.i, prob.j, prob.k, prob.x, P=7)
    with pytest.raises(oracle.OracleError):
        oracle.run(big_p, A, B, C, G, 1)


# --------------------------------------------------------------------------
# QR post-step (last step of Algorithm 1)
# --------------------------------------------------------------------------
def test_qr_post_keeps_the_model_and_orthonormalises():
    rng = np.random.default_rng(8)
    dims, J = (30, 40, 6), (4, 5, 3)
    A, B, C = (rng.standard_normal((d, r)) for d, r in zip(dims, J))
    G = rng.standard_normal(J)
    Q1, Q2, Q3, G2 = oracle.qr_post(A, B, C, G)
    np.testing.assert_allclose(oracle.dense_model(G2, Q1, Q2, Q3), oracle.dense_model(G, A, B, C),
                               rtol=1e-11, atol=1e-11)
    for Q, U in ((Q1, A), (Q2, B), (Q3, C)):
        np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)
        R = Q.T @ U
        np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-12)   # upper triangular
        assert np.all(np.diag(R) > 0)                                  # positive diagonal
        np.testing.assert_allclose(Q @ R, U, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# Fold-in (Eq. 6) and top-k search
# --------------------------------------------------------------------------
def test_fold_in_recovers_an_exact_profile():
    rng = np.random.default_rng(12)
    I2, I3, J = 40, 3, (4, 5, 2)
    B, C = rng.standard_normal((I2, J[1])), rng.standard_normal((I3, J[2]))
    G = rng.standard_normal(J)
    cells = synth.sample_cells(rng, I2 * I3, 60)
    j, k = cells // I3, cells % I3
    u_true = rng.standard_normal(J[0])
    # x = G x1 u x2 b_j x3 c_k, written with the dense model of a one-row A
    x = oracle.dense_model(G, u_true[None, :], B, C)[0, j, k]
    np.testing.assert_allclose(oracle.fold_in(B, C, G, j, k, x, lam=0.0), u_true, rtol=1e-10, atol=1e-12)


def test_fold_in_ridge_solves_the_normal_equations():
    rng = np.random.default_rng(13)
    I2, I3, J = 30, 4, (3, 4, 2)
    B, C = rng.standard_normal((I2, J[1])), rng.standard_normal((I3, J[2]))
    G = rng.standard_normal(J)
    cells = synth.sample_cells(rng, I2 * I3, 50)
    j, k = cells // I3, cells % I3
    x = rng.standard_normal(50)
    lam = 0.7
    W = np.stack([oracle.dense_model(G, np.eye(J[0]), B, C)[:, jj, kk] for jj, kk in zip(j, k)])
    u = oracle.fold_in(B, C, G, j, k, x, lam=lam)
    np.testing.assert_allclose((W.T @ W + lam * np.eye(J[0])) @ u, W.T @ x, rtol=1e-10, atol=1e-10)


def test_topk_cosine_brute_force_with_ties_and_zero_rows():
    A = np.array([[1.0, 0.0], [0.0, 0.0], [2.0, 0.0], [0.0, 1.0], [1.0, 1.0], [-1.0, 0.0]])
    idx, sc = oracle.topk_cosine(A, np.array([3.0, 0.0]), k=4)
    # rows 0 and 2 tie at cosine 1 (lower index first); row 1 has zero norm
    assert idx.tolist() == [0, 2, 4, 3]
    np.testing.assert_allclose(sc, [1.0, 1.0, np.sqrt(0.5), 0.0], atol=1e-15)


# --------------------------------------------------------------------------
# Algorithm 1 read literally (comparison run)
# --------------------------------------------------------------------------
def test_literal_epoch_is_sequential_per_item_gradient_steps():
    # one epoch visits nonzeros and edges in the seeded interleaving; each
    # nonzero is a gradient step on its own term of the split objective
    # (Section 2.3.2), each edge a step on its own network term (Eq. 4)
    prob, (A, B, C, G) = _tiny(seed=3, dims=(4, 5, 2), ranks=(2, 3, 2), nnz=9, lam=0.2, lam_g=0.7,
                               lr=0.05, edges=4)
    A1, B1, C1, G1, loss, rmse = oracle.run_literal(prob, A, B, C, G, 1)
    order = oracle.shuffle(prob.nnz + prob.eu.shape[0], prob.seed, oracle.LITERAL_STREAM)
    f = [np.array(a, np.float64) for a in (A, B, C, G)]
    for it in order:
        if it < prob.nnz:
            fun = lambda a, b, c, g: oracle.f_split(prob, a, b, c, g, subset=[it])
            g = _grads(fun, *f)
        else:
            e = it - prob.nnz
            u, v, w = prob.eu[e], prob.ev[e], prob.ew[e]
            fun = lambda b: 0.5 * prob.lam_g * w * float(np.sum((b[u] - b[v]) ** 2))
            g = [np.zeros_like(f[0]), oracle.fd_grad(fun, f[1]), np.zeros_like(f[2]), np.zeros_like(f[3])]
        f = [x - prob.lr * gx for x, gx in zip(f, g)]
    for got, ref in zip((A1, B1, C1, G1), f):
        assert _rel(got, ref) < 1e-7
    assert abs(loss[0] - oracle.f_opt_dense(prob, *f)) < 1e-8 * abs(loss[0])


def test_literal_first_epoch_descends_on_planted_tensor():
    p = synth.planted()
    pr0 = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, np.zeros(len(p.i)))
    x = oracle.model_values(pr0, p.A, p.B, p.C, p.G) + p.noise
    prob = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, x, p.eu, p.ev, lam=0.01, lam_g=0.1,
                          lr=1e-3, seed=synth.PLAN_SEED)
    A, B, C, G = synth.normal_init(synth.INIT_SEED, p.dims, p.ranks, 1.0)
    f0, _, _ = oracle.loss(prob, A, B, C, G)
    *_, loss, _ = oracle.run_literal(prob, A, B, C, G, 1)
    # plain SGD with a constant step only promises progress from far away
    assert loss[0] < 0.1 * f0
