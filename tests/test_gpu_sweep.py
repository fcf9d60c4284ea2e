"""Execution choices (record chunk, driver), the autotuners and
the sweep: every one of them must leave the results bit-identical
to a plain snect_train of the same problem."""
import numpy as np
import pytest

from helpers import gpu_factors, gpu_problem, planted_case, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1711_08095_amd as sn
    assert torch.cuda.is_available()
    c = sn.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _same(a, b):
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("ranks,P,T", [((5, 5, 2), 8, 64), ((10, 10, 5), 5, 29), ((20, 20, 5), 4, 64)])
def test_execution_choices_are_bit_identical(ctx, precision, ranks, P, T):
    import paper_1711_08095_amd as sn
    case = planted_case(seed=31, dims=(90, 130, 5), ranks=ranks, nnz=7000, edges=400, P=P, T=T, sigma=0.5, lr=2e-4)
    print(f"exec choices ranks={ranks} P={P} T={T} precision={precision}", flush=True)
    prob = gpu_problem(ctx, case, precision=precision)
    ref = run_gpu(ctx, case, 2, prob=prob)
    for path, waves, rec_cap in [(sn.PATH_PERSISTENT, 8, 0), (sn.PATH_MULTI, 8, 64), (sn.PATH_PERSISTENT, 0, 128),
                                 (sn.PATH_MULTI, 0, 256)]:
        prob.set_exec(path=path, waves=waves, rec_cap=rec_cap)
        _same(ref, run_gpu(ctx, case, 2, prob=prob))


def test_exec_validation(ctx):
    import paper_1711_08095_amd as sn
    case = planted_case(seed=32, dims=(40, 60, 3), ranks=(4, 4, 2), nnz=1500, edges=50, P=4, T=16)
    prob = gpu_problem(ctx, case)
    for kw in (dict(waves=6), dict(waves=4), dict(rec_cap=100), dict(rec_cap=32), dict(rec_cap=1 << 20)):
        print("set_exec", kw, flush=True)
        with pytest.raises(sn.SnectError) as e:
            prob.set_exec(**kw)
        assert e.value.code == -1


def test_autotune_keeps_results_and_factors(ctx):
    case = planted_case(seed=33, ranks=(10, 10, 5), sigma=0.5, lr=2e-4)
    prob = gpu_problem(ctx, case)
    ref = run_gpu(ctx, case, 2, prob=prob)
    f = gpu_factors(case)
    before = [t.clone() for t in f]
    choice, ms = prob.autotune(*f, trials=1)
    print("autotune choice", choice, f"{ms:.3f} ms", flush=True)
    assert choice["waves"] == 8 and choice["rec_cap"] >= 64 and ms > 0
    for a, b in zip(f, before):
        assert bool((a == b).all())
    _same(ref, run_gpu(ctx, case, 2, prob=prob))


def _sweep_cases():
    specs = [((5, 5, 2), 8, 64, 200, 500, 20000), ((10, 10, 5), 6, 64, 300, 700, 30000),
             ((20, 20, 5), 5, 37, 150, 400, 15000), ((16, 12, 3), 7, 64, 250, 600, 25000),
             ((3, 7, 2), 3, 16, 60, 90, 2000)]
    out = []
    for n, (ranks, P, T, I1, I2, nnz) in enumerate(specs):
        out.append(planted_case(seed=40 + n, dims=(I1, I2, 5), ranks=ranks, nnz=nnz, edges=I2 * 2, P=P, T=T,
                                sigma=0.5, lr=2e-4, lam_g=[0.0, 0.01, 0.1, 1.0, 0.1][n], plan_seed=3100 + n))
    return out


@pytest.mark.skip(reason="the single batched sweep launch is switched off (the library's kSweepEnabled): its "
                         "first FP32 run after the LDS-layout change took a GPU memory-aperture fault with no "
                         "established cause; kept off the GPU")
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_launch_equals_individual_training(ctx, precision):
    import paper_1711_08095_amd as sn
    cases = _sweep_cases()
    probs = [gpu_problem(ctx, c, precision=precision) for c in cases]
    solo = [run_gpu(ctx, c, 3, prob=p) for c, p in zip(cases, probs)]
    fs = [gpu_factors(c) for c in cases]
    loss, rmse = sn.sweep_train(ctx, probs, fs, 3)
    for n, (c, s) in enumerate(zip(cases, solo)):
        got = [t.double().cpu().numpy() for t in fs[n]]
        print(f"sweep problem {n} ranks={c['ranks']}", flush=True)
        _same(s, (got, loss[n], rmse[n]))
    # the sweep autotuner changes execution only
    fs2 = [gpu_factors(c) for c in cases]
    ms = sn.sweep_autotune(ctx, probs, fs2, trials=1)
    assert ms > 0
    loss2, rmse2 = sn.sweep_train(ctx, probs, fs2, 3)
    np.testing.assert_array_equal(loss, loss2)
    for a, b in zip(fs, fs2):
        for x, y in zip(a, b):
            assert bool((x == y).all())


@pytest.mark.parametrize("precision", [0, 1])
def test_concurrent_sweep_equals_individual_training(ctx, precision):
    # with the batched launch switched off, the sweep runs every problem on
    # its own stream with the multi-launch driver, concurrently
    import paper_1711_08095_amd as sn
    cases = _sweep_cases()
    probs = [gpu_problem(ctx, c, precision=precision) for c in cases]
    solo = [run_gpu(ctx, c, 3, prob=p) for c, p in zip(cases, probs)]
    fs = [gpu_factors(c) for c in cases]
    print(f"concurrent sweep, precision {precision}", flush=True)
    loss, rmse = sn.sweep_train(ctx, probs, fs, 3)
    for n, (c, s) in enumerate(zip(cases, solo)):
        got = [t.double().cpu().numpy() for t in fs[n]]
        _same(s, (got, loss[n], rmse[n]))
    # resumed: 2 + 1 epochs equal 3
    fs2 = [gpu_factors(c) for c in cases]
    l1, _ = sn.sweep_train(ctx, probs, fs2, 2)
    l2, _ = sn.sweep_train(ctx, probs, fs2, 1, start_epoch=2)
    np.testing.assert_array_equal(np.concatenate([l1, l2], axis=1), loss)
    for a, b in zip(fs, fs2):
        for x, y in zip(a, b):
            assert bool((x == y).all())
    # the sweep autotuner changes execution only, and leaves the factors
    fs3 = [gpu_factors(c) for c in cases]
    before = [[t.clone() for t in f] for f in fs3]
    ms = sn.sweep_autotune(ctx, probs, fs3, trials=1)
    assert ms > 0
    for a, b in zip(fs3, before):
        for x, y in zip(a, b):
            assert bool((x == y).all())
    loss3, _ = sn.sweep_train(ctx, probs, fs3, 3)
    np.testing.assert_array_equal(loss, loss3)


def test_sweep_validation(ctx):
    import paper_1711_08095_amd as sn
    cases = _sweep_cases()[:2]
    p32 = gpu_problem(ctx, cases[0], precision=0)
    p16 = gpu_problem(ctx, cases[1], precision=1)
    with pytest.raises(sn.SnectError) as e:
        sn.sweep_train(ctx, [p32, p16], [gpu_factors(cases[0]), gpu_factors(cases[1])], 1)
    assert e.value.code == -1
    with pytest.raises(sn.SnectError) as e:
        sn.sweep_train(ctx, [p32, p32], [gpu_factors(cases[0]), gpu_factors(cases[0])], 1)
    assert e.value.code == -1
    with pytest.raises(sn.SnectError) as e:
        sn.sweep_train(ctx, [p32], [gpu_factors(cases[0])], -1)
    assert e.value.code == -1
