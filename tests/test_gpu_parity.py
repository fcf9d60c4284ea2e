"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: factors within 1e-4 relative Frobenius error of the oracle after
one epoch, per-epoch loss within 1e-3 relative after ten epochs.  FP32 SGD
against FP64 accumulates rounding of order 1e-7 per update; the bounds leave
room for the amplification of that by the iteration.
"""
import numpy as np
import pytest

import oracle
import snect_synth as synth
from helpers import gpu_factors, gpu_problem, planted_case, rel_fro, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

FACTOR_TOL = 1e-4
LOSS_TOL = 1e-3


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1711_08095_amd as sn
    assert torch.cuda.is_available()
    c = sn.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _check_factors(gpu, orc, tol=FACTOR_TOL):
    for name, g, o in zip("ABCG", gpu, orc):
        r = rel_fro(g, o)
        assert r <= tol, f"{name}: relative Frobenius error {r:.3e} > {tol}"


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("P,T", [(8, 64), (1, 1), (4, 16), (3, 37)])
def test_planted_one_epoch_factors(ctx, P, T, path):
    case = planted_case(P=P, T=T)
    print(f"planted P={P} T={T} path={path}", flush=True)
    orc = run_oracle(case, 1)
    prob = gpu_problem(ctx, case)
    prob.set_exec(path=path)
    gpu, loss, rmse, _ = run_gpu(ctx, case, 1, prob=prob)
    _check_factors(gpu, orc[:4])
    assert abs(loss[0] - orc[4][0]) <= LOSS_TOL * abs(orc[4][0])


@pytest.mark.parametrize("P,T,ranks", [(8, 64, (5, 5, 2)), (5, 29, (20, 20, 5)), (3, 7, (16, 12, 3))])
def test_paths_are_bit_identical(ctx, P, T, ranks):
    import paper_1711_08095_amd as sn
    case = planted_case(seed=21, dims=(61, 83, 6), ranks=ranks, nnz=5000, edges=300, P=P, T=T, sigma=0.5,
                        lr=2e-4)
    prob = gpu_problem(ctx, case)
    assert prob.exec_path() == sn.PATH_PERSISTENT
    out = []
    for path in (sn.PATH_PERSISTENT, sn.PATH_MULTI):
        prob.set_exec(path=path)
        out.append(run_gpu(ctx, case, 3, prob=prob))
    for a, b in zip(out[0][0], out[1][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_planted_ten_epochs_loss(ctx):
    case = planted_case()
    orc = run_oracle(case, 10)
    gpu, loss, rmse, _ = run_gpu(ctx, case, 10)
    np.testing.assert_allclose(loss, orc[4], rtol=LOSS_TOL)
    np.testing.assert_allclose(rmse, orc[5], rtol=LOSS_TOL)
    assert np.all(np.diff(loss) < 0)


def test_plan_draws_match_oracle(ctx):
    case = planted_case(P=8, T=64)
    prob = gpu_problem(ctx, case)
    for ep in (0, 3):
        g = prob.plan_export(ep)
        o = oracle.plan_export(__import__("helpers").oracle_problem(case), epoch=ep)
        np.testing.assert_array_equal(g["perm1"], o["perm1"])
        np.testing.assert_array_equal(g["perm2"], o["perm2"])
        np.testing.assert_array_equal(g["strata"], o["strata"])
    info = prob.info()
    assert info["ntiles"] == len(o["tile_start"]) - 1


# every kernel instantiation (JP = the smallest of 2, 4, 5, 8, 10, 12, 16,
# 20, 24, 32 that holds max(J1, J2)), with J1 != J2 where it matters
CORE_SIZES = [(1, 1, 1), (4, 3, 2), (5, 4, 2), (3, 7, 2), (8, 7, 2), (10, 10, 5), (12, 11, 3), (12, 12, 3),
              (16, 12, 3), (20, 20, 5), (24, 21, 4), (24, 9, 3), (32, 17, 4)]


@pytest.mark.parametrize("ranks", CORE_SIZES)
def test_core_sizes(ctx, ranks):
    # ragged block and tile tails; the one-epoch factor bound and the loss
    # bound over two epochs
    case = planted_case(seed=77, dims=(61, 83, 6), ranks=ranks, nnz=5000, edges=300, P=5, T=29,
                        sigma=0.5, lr=2e-4)
    print(f"ranks {ranks}", flush=True)
    orc1 = run_oracle(case, 1)
    gpu, loss, _, prob = run_gpu(ctx, case, 1)
    _check_factors(gpu, orc1[:4])
    assert abs(loss[0] - orc1[4][0]) <= LOSS_TOL * abs(orc1[4][0])
    orc = run_oracle(case, 2)
    _, loss2, _, _ = run_gpu(ctx, case, 2, prob=prob)
    np.testing.assert_allclose(loss2, orc[4], rtol=LOSS_TOL)


def test_fewer_core_items_than_blocks(ctx):
    # core 1x1x1 over 3 platforms: 3 items of the stratum sums for 8 blocks,
    # so five of the workgroups reduce nothing and hand over only their rows
    import paper_1711_08095_amd as sn
    case = planted_case(seed=21, dims=(120, 160, 3), ranks=(1, 1, 1), nnz=6000, edges=400, P=8, T=64)
    prob = gpu_problem(ctx, case)
    assert prob.exec_path() == sn.PATH_PERSISTENT
    orc = run_oracle(case, 3)
    gpu, loss, _, _ = run_gpu(ctx, case, 3, prob=prob)
    _check_factors(gpu, orc[:4])
    np.testing.assert_allclose(loss, orc[4], rtol=LOSS_TOL)
    # and bit for bit the multi-launch driver's result
    prob.set_exec(path=sn.PATH_MULTI)
    gpu2, loss2, _, _ = run_gpu(ctx, case, 3, prob=prob)
    for a, b in zip(gpu, gpu2):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(loss, loss2)


def test_exchange_time_out_is_reported_and_leaves_no_trace(ctx):
    # a wait limit of one poll round forces the persistent kernel's time-out
    # path from the host: the waiting workgroups give up, the epoch fails
    # with the time-out error and every workgroup leaves the launch; the
    # exchange words that launch left behind carry tags no later launch uses,
    # so the next epochs are bit for bit those of a fresh problem
    import paper_1711_08095_amd as sn
    case = planted_case(P=8, T=64)
    ref, lref, _, _ = run_gpu(ctx, case, 2)
    prob = gpu_problem(ctx, case)
    assert prob.exec_path() == sn.PATH_PERSISTENT
    prob.set_exec(wait_limit=1)
    failed = 0
    for _ in range(3):
        try:
            run_gpu(ctx, case, 1, prob=prob)
        except sn.SnectError as e:
            assert "timed out" in str(e)
            failed += 1
    assert failed > 0
    with pytest.raises(sn.SnectError):
        prob.set_exec(wait_limit=-1)
    prob.set_exec()
    got, lgot, _, _ = run_gpu(ctx, case, 2, prob=prob)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(lref, lgot)


def test_empty_rows_and_platforms(ctx):
    # rows with no nonzeros stay put (except B through the graph), a platform
    # with no nonzeros keeps its C row
    case = planted_case(seed=5, dims=(50, 70, 4), ranks=(4, 4, 2), nnz=1500, edges=100, P=4, T=64)
    keep = (case["k"] != 2) & (case["i"] % 7 != 3) & (case["j"] % 5 != 1)
    for key in ("i", "j", "k", "x"):
        case[key] = case[key][keep]
    orc = run_oracle(case, 2)
    gpu, loss, _, _ = run_gpu(ctx, case, 2)
    _check_factors(gpu, orc[:4])
    np.testing.assert_array_equal(gpu[2][2], np.asarray(case["init"][2], np.float64)[2])
    np.testing.assert_array_equal(gpu[0][3], np.asarray(case["init"][0], np.float64)[3])


def test_graph_only(ctx):
    case = planted_case(seed=9, dims=(20, 300, 3), ranks=(3, 4, 2), nnz=1000, edges=900, P=2, T=8,
                        lam=0.0, lam_g=2.0, lr=0.05)
    for key in ("i", "j", "k", "x"):
        case[key] = case[key][:0]
    orc = run_oracle(case, 3)
    gpu, loss, rmse, prob = run_gpu(ctx, case, 3)
    assert prob.info()["n_sub"] > 1
    _check_factors(gpu, orc[:4], tol=1e-5)
    np.testing.assert_allclose(loss, orc[4], rtol=1e-5)
    assert np.all(rmse == 0)


def test_deterministic_and_resumable(ctx):
    case = planted_case(P=8, T=64)
    g1, l1, _, prob = run_gpu(ctx, case, 4)
    g2, l2, _, _ = run_gpu(ctx, case, 4, prob=prob)
    for a, b in zip(g1, g2):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(l1, l2)
    f = gpu_factors(case)
    la, _ = prob.train(*f, epochs=2, start_epoch=0)
    lb, _ = prob.train(*f, epochs=2, start_epoch=2)
    for a, b in zip(g1, [t.double().cpu().numpy() for t in f]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(l1, np.concatenate([la, lb]))


def test_evaluate_matches_oracle_loss(ctx):
    case = planted_case(seed=3, dims=(90, 110, 5), ranks=(6, 5, 3), nnz=4000, edges=250, P=6, T=32)
    prob = gpu_problem(ctx, case)
    f = gpu_factors(case)
    loss, rmse = prob.evaluate(*f)
    A, B, C, G = (np.asarray(a, np.float64) for a in case["init"])
    from helpers import oracle_problem
    fo, ro, _ = oracle.loss(oracle_problem(case), A, B, C, G)
    assert loss == pytest.approx(fo, rel=1e-5)
    assert rmse == pytest.approx(ro, rel=1e-5)


def test_evaluate_per_block_loss_kernel(ctx):
    """A gene block whose w1 table (600 rows x 24 platforms x 10 columns,
    576 KB) cannot sit in LDS: the loss pass falls back to the per-block
    kernel, which must agree with the oracle as the column-wise one does."""
    print("per-block loss kernel: (60, 1200, 24), ranks (10, 8, 3), P=2", flush=True)
    case = planted_case(seed=5, dims=(60, 1200, 24), ranks=(10, 8, 3), nnz=6000, edges=900, P=2, T=64)
    prob = gpu_problem(ctx, case)
    f = gpu_factors(case)
    loss, rmse = prob.evaluate(*f)
    A, B, C, G = (np.asarray(a, np.float64) for a in case["init"])
    from helpers import oracle_problem
    fo, ro, _ = oracle.loss(oracle_problem(case), A, B, C, G)
    assert loss == pytest.approx(fo, rel=1e-5)
    assert rmse == pytest.approx(ro, rel=1e-5)
    # and one training epoch through the same problem
    orc = run_oracle(case, 1)
    gpu, loss1, _, _ = run_gpu(ctx, case, 1)
    _check_factors(gpu, orc[:4])
    assert abs(loss1[0] - orc[4][0]) <= LOSS_TOL * abs(orc[4][0])


def test_divergence_returns_last_finite(ctx):
    import torch
    import paper_1711_08095_amd as sn
    case = planted_case(lr=5.0, P=4, T=16)
    prob = gpu_problem(ctx, case)
    f = gpu_factors(case)
    with pytest.raises(sn.SnectError) as e:
        prob.train(*f, epochs=6)
    assert e.value.code == -7
    for t in f:
        assert bool(t.isfinite().all())
    # the same factors as training one epoch per call up to the first
    # non-finite epoch (whose call rolls back to its own start); later epochs
    # may already have been queued when the divergence is seen
    g = gpu_factors(case)
    first_bad = None
    for ep in range(6):
        try:
            prob.train(*g, epochs=1, start_epoch=ep)
        except sn.SnectError as err:
            assert err.code == -7
            first_bad = ep
            break
    assert first_bad is not None
    print(f"first non-finite epoch {first_bad}", flush=True)
    for x, y in zip(f, g):
        assert torch.equal(x, y)


def test_validation_errors(ctx):
    import paper_1711_08095_amd as sn
    case = planted_case(nnz=500, edges=10)
    bad = dict(case)
    bad["i"] = np.r_[case["i"], case["i"][:1]]
    bad["j"] = np.r_[case["j"], case["j"][:1]]
    bad["k"] = np.r_[case["k"], case["k"][:1]]
    bad["x"] = np.r_[case["x"], np.float32(1.0)]
    with pytest.raises(sn.SnectError) as e:
        gpu_problem(ctx, bad)
    assert e.value.code == -3
    bad = dict(case)
    bad["i"] = case["i"].copy()
    bad["i"][7] = 200
    with pytest.raises(sn.SnectError) as e:
        gpu_problem(ctx, bad)
    assert e.value.code == -2
    for key, val, code in (("P", 0, -1), ("T", 65, -1), ("ranks", (33, 2, 2), -4)):
        bad = dict(case)
        bad[key] = val
        with pytest.raises(sn.SnectError) as e:
            gpu_problem(ctx, bad)
        assert e.value.code == code


@pytest.fixture(scope="module")
def pancan_data():
    import time
    t = time.time()
    data = synth.pancan_like()
    print(f"pancan inputs generated in {time.time() - t:.1f}s", flush=True)
    return data


def _pancan_case(data, ranks, init_offset):
    i, j, k, x, eu, ev = data
    sigma = synth.default_sigma(x, ranks)
    A, B, C, G = synth.normal_init(synth.INIT_SEED + init_offset, (4500, 14000, 5), ranks, sigma)
    return dict(dims=(4500, 14000, 5), ranks=ranks, i=i, j=j, k=k, x=x, eu=eu, ev=ev, ew=None,
                lam=0.01, lam_g=0.1, lr=1e-3, cls=1.0, P=128, T=64, seed=synth.PLAN_SEED + init_offset,
                init=tuple(a.astype(np.float32) for a in (A, B, C, G)))


def test_pancan_full_size_one_epoch(ctx, pancan_data):
    # the PanCan-shaped workload at full size (4,500 x 14,000 x 5, 25M
    # nonzeros, core 10x10x5, P = 128, T = 64), one epoch against the oracle
    import time
    t = time.time()
    case = _pancan_case(pancan_data, (10, 10, 5), 1)
    gpu, loss, rmse, prob = run_gpu(ctx, case, 1)
    print(f"gpu done {time.time() - t:.1f}s loss {loss}", flush=True)
    orc = run_oracle(case, 1)
    print(f"oracle done {time.time() - t:.1f}s loss {orc[4]}", flush=True)
    _check_factors(gpu, orc[:4])
    assert abs(loss[0] - orc[4][0]) <= LOSS_TOL * abs(orc[4][0])


def test_pancan_full_size_core20_fp32_and_bf16(ctx, pancan_data):
    # the same tensor with core 20x20x5 (the BF16 workload), one epoch: FP32
    # within the FP32 bound, BF16 within the rounding bound of the BF16
    # tests (8 u ||F_oracle - F_0|| + 1e-4 ||F_oracle||, u = 2^-8)
    import time
    t = time.time()
    case = _pancan_case(pancan_data, (20, 20, 5), 2)
    orc = run_oracle(case, 1)
    print(f"oracle core 20 done {time.time() - t:.1f}s loss {orc[4]}", flush=True)
    gpu, loss, _, _ = run_gpu(ctx, case, 1)
    print(f"fp32 core 20: loss {loss}", flush=True)
    _check_factors(gpu, orc[:4])
    assert abs(loss[0] - orc[4][0]) <= LOSS_TOL * abs(orc[4][0])
    gb, lb, _, _ = run_gpu(ctx, case, 1, precision=1)
    u = 2.0 ** -8
    for name, g, o, f0 in zip("ABCG", gb, orc[:4], case["init"]):
        d = np.linalg.norm(g - o)
        step = np.linalg.norm(o - np.asarray(f0, np.float64))
        bound = 8.0 * u * step + FACTOR_TOL * np.linalg.norm(o)
        print(f"  bf16 {name}: |F-F_orc|/|F_orc| {d / np.linalg.norm(o):.2e}  ratio to u|dF| "
              f"{d / max(u * step, 1e-300):.2f}", flush=True)
        assert d <= bound, name
    assert abs(lb[0] - orc[4][0]) <= 1e-2 * abs(orc[4][0])
