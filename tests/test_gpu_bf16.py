"""BF16 matrix-core contractions of the tile step (BF16 operands, FP32
accumulation, FP32 factor rows, residuals, updates and loss) against the
FP64 oracle.

Tolerance, from the arithmetic: every BF16 operand is the FP32 value rounded
once (unit roundoff u = 2^-8), so each contraction w1 = H_k b, w2 = H_k^T a,
x~ = a . w1 and each term of S = sum e a (x) b carries a relative error of a
few u, and so does every update built from them.  After one epoch a factor
F therefore differs from the oracle's by a few u times the change the epoch
made, ||F_bf16 - F_oracle|| <= KAPPA u ||F_oracle - F_0||, plus the FP32
tolerance of the FP32 path (KAPPA = 8 leaves room for the sums of a few
rounded terms and for the errors carried from tile to tile)."""
import numpy as np
import pytest

from helpers import planted_case, rel_fro, run_gpu, run_oracle, gpu_problem

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8
KAPPA = 8.0
FP32_TOL = 1e-4
BF16 = 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1711_08095_amd as sn
    assert torch.cuda.is_available()
    c = sn.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _check(gpu, orc, init):
    worst = 0.0
    for name, g, o, f0 in zip("ABCG", gpu, orc, init):
        o = np.asarray(o, np.float64)
        d = np.linalg.norm(np.asarray(g, np.float64) - o)
        step = np.linalg.norm(o - np.asarray(f0, np.float64))
        bound = KAPPA * U_BF16 * step + FP32_TOL * np.linalg.norm(o)
        print(f"  {name}: |F-F_orc| {d:.3e}  u|dF| {U_BF16 * step:.3e}  bound {bound:.3e}", flush=True)
        assert d <= bound, f"{name}: {d:.3e} > {bound:.3e}"
        worst = max(worst, d / max(U_BF16 * step, 1e-300))
    return worst


@pytest.mark.parametrize("ranks,P,T,lr", [((5, 5, 2), 8, 64, 1e-3), ((10, 10, 5), 8, 64, 1e-3),
                                          ((20, 20, 5), 8, 64, 2e-4), ((16, 12, 3), 3, 37, 2e-4),
                                          ((32, 17, 4), 8, 16, 2e-4), ((1, 1, 1), 2, 5, 1e-3),
                                          ((4, 3, 2), 8, 64, 1e-3), ((8, 7, 2), 5, 29, 1e-3),
                                          ((12, 11, 3), 8, 64, 5e-4), ((24, 21, 4), 4, 37, 2e-4),
                                          ((24, 9, 3), 3, 64, 2e-4)])
def test_bf16_one_epoch_within_rounding_bound(ctx, ranks, P, T, lr):
    case = planted_case(ranks=ranks, P=P, T=T, lr=lr, sigma=0.5)
    print(f"bf16 planted ranks={ranks} P={P} T={T}", flush=True)
    orc = run_oracle(case, 1)
    gpu, loss, rmse, _ = run_gpu(ctx, case, 1, precision=BF16)
    worst = _check(gpu, orc[:4], case["init"])
    print(f"  worst |F-F_orc| / (u |dF|) = {worst:.2f}", flush=True)
    # the loss is computed in FP32 from the end-of-epoch factors
    assert abs(loss[0] - orc[4][0]) <= 1e-2 * abs(orc[4][0])


@pytest.mark.parametrize("P,T,ranks", [(8, 64, (5, 5, 2)), (5, 29, (20, 20, 5))])
def test_bf16_paths_are_bit_identical(ctx, P, T, ranks):
    import paper_1711_08095_amd as sn
    case = planted_case(seed=21, dims=(61, 83, 6), ranks=ranks, nnz=5000, edges=300, P=P, T=T, sigma=0.5,
                        lr=2e-4)
    prob = gpu_problem(ctx, case, precision=BF16)
    out = []
    for path in (sn.PATH_PERSISTENT, sn.PATH_MULTI):
        prob.set_exec(path=path)
        out.append(run_gpu(ctx, case, 3, prob=prob))
    for a, b in zip(out[0][0], out[1][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_bf16_ten_epochs_track_the_oracle(ctx):
    case = planted_case()
    orc = run_oracle(case, 10)
    gpu, loss, rmse, _ = run_gpu(ctx, case, 10, precision=BF16)
    print("oracle loss", orc[4], "\nbf16 loss", loss, flush=True)
    np.testing.assert_allclose(loss, orc[4], rtol=1e-2)
    assert np.all(np.diff(loss) < 0)
