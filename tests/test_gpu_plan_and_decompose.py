"""The plan as the kernels read it, bit for bit against the oracle's plan,
and the one-shot snect_decompose (explicit and default random start)
against the oracle.

The plan is integer work: the packed records (patient and gene row inside
the block, the gene-slot rank inside the tile), the values, the tile cuts,
their platforms and the block -> tile ranges must equal what the oracle's
plan implies exactly.  The slot rank is a layout detail of the HIP path that
the oracle has no notion of; it is checked against its definition (the rank
of the record when its tile is stably ordered by gene row), computed here
from the oracle's order.
"""
import numpy as np
import pytest

import oracle
import snect_synth as synth
from helpers import gpu_factors, gpu_problem, oracle_problem, planted_case, rel_fro, run_oracle

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


def expected_layout(case):
    """Records, tiles and block ranges implied by the oracle's plan."""
    o = oracle.plan_export(oracle_problem(case))
    I1, I2, _ = case["dims"]
    P = case["P"]
    order, ts, bt = o["order"], o["tile_start"], o["block_tile"]
    nnz, nt = order.size, ts.size - 1
    pos1 = np.empty(I1, np.int64)
    pos1[o["perm1"]] = np.arange(I1)
    pos2 = np.empty(I2, np.int64)
    pos2[o["perm2"]] = np.arange(I2)
    # first position of block p: the smallest r with floor(r P / I) = p
    start1 = -((-np.arange(P + 1) * I1) // P)
    start2 = -((-np.arange(P + 1) * I2) // P)
    tile_of = np.repeat(np.arange(nt), np.diff(ts))
    blk_of_tile = np.repeat(np.arange(P * P), np.diff(bt))
    blk = blk_of_tile[tile_of]
    p, q = blk // P, blk % P
    gi, gj = case["i"][order], case["j"][order]
    il = pos1[gi] - start1[p]
    jl = pos2[gj] - start2[q]
    # slot: rank inside the tile under a stable order by gene row
    rank_order = np.lexsort((np.arange(nnz), jl, tile_of))
    slot = np.empty(nnz, np.int64)
    slot[rank_order] = np.arange(nnz) - ts[tile_of[rank_order]]
    tile_k = case["k"][order[ts[:-1]]] if nt > 0 else np.zeros(0, np.int64)
    return dict(il=il, jl=jl, slot=slot, x=np.asarray(case["x"], np.float32)[order],
                tile_off=ts, tile_k=tile_k, blk_tile=bt, order=order)


def check_layout(prob, case):
    g = prob.plan_layout()
    e = expected_layout(case)
    np.testing.assert_array_equal(g["tile_off"].astype(np.int64), e["tile_off"])
    np.testing.assert_array_equal(g["tile_k"].astype(np.int64), e["tile_k"])
    np.testing.assert_array_equal(g["blk_tile"].astype(np.int64), e["blk_tile"])
    w = g["word"].astype(np.int64)
    bi, bj = g["bits_i"], g["bits_j"]
    np.testing.assert_array_equal(w & ((1 << bi) - 1), e["il"])
    np.testing.assert_array_equal((w >> bi) & ((1 << bj) - 1), e["jl"])
    np.testing.assert_array_equal(w >> (bi + bj), e["slot"])
    np.testing.assert_array_equal(g["x"].view(np.uint32), e["x"].view(np.uint32))
    # the field widths are the smallest that hold a block's rows
    I1, I2, _ = case["dims"]
    P = case["P"]
    assert bi == max(1, int(np.ceil(np.log2(-(-I1 // P)))))
    assert bj == max(1, int(np.ceil(np.log2(-(-I2 // P)))))


@pytest.mark.parametrize("P,T", [(8, 64), (1, 1), (4, 16), (3, 37)])
def test_plan_layout_is_bit_exact(ctx, P, T):
    case = planted_case(P=P, T=T)
    print(f"plan layout planted P={P} T={T}", flush=True)
    check_layout(gpu_problem(ctx, case), case)


def test_plan_layout_ragged_and_empty_blocks(ctx):
    # few nonzeros: many blocks empty, blocks of one nonzero, uneven rows
    case = planted_case(seed=13, dims=(37, 53, 3), ranks=(3, 3, 2), nnz=150, edges=20, P=9, T=5)
    print("plan layout ragged P=9 T=5", flush=True)
    prob = gpu_problem(ctx, case)
    check_layout(prob, case)
    bt = prob.plan_layout()["blk_tile"]
    assert np.any(np.diff(bt) == 0)


def test_plan_layout_pancan_full_size(ctx):
    import time
    t = time.time()
    i, j, k, x, eu, ev = synth.pancan_like()
    case = dict(dims=(4500, 14000, 5), ranks=(10, 10, 5), i=i, j=j, k=k, x=x, eu=eu, ev=ev, ew=None,
                lam=0.01, lam_g=0.1, lr=1e-3, cls=1.0, P=128, T=64, seed=synth.PLAN_SEED + 1)
    print(f"plan layout pancan 25M generated in {time.time() - t:.1f}s", flush=True)
    prob = gpu_problem(ctx, case)
    check_layout(prob, case)
    print(f"plan layout pancan checked in {time.time() - t:.1f}s", flush=True)


def _decompose(ctx, case, epochs, init):
    import torch
    import paper_1711_08095_amd as sn
    I1, I2, I3 = case["dims"]
    J1, J2, J3 = case["ranks"]
    out = [torch.zeros(s, device="cuda") for s in ((I1, J1), (I2, J2), (I3, J3), (J1, J2, J3))]
    hyper = sn.Hyper(ranks=case["ranks"], lam=case["lam"], lam_g=case["lam_g"], lr=case["lr"],
                     core_lr_scale=case["cls"], P=case["P"], T=case["T"], seed=case["seed"])
    loss, rmse = sn.decompose(ctx, case["dims"], case["i"], case["j"], case["k"], case["x"], case["eu"],
                              case["ev"], case["ew"], hyper, out, init=init, epochs=epochs)
    return [t.double().cpu().numpy() for t in out], loss, rmse


def test_decompose_with_init_matches_the_oracle(ctx):
    case = planted_case(P=8, T=64)
    print("decompose explicit init, 1 epoch", flush=True)
    got, loss, _ = _decompose(ctx, case, 1, gpu_factors(case))
    orc = run_oracle(case, 1)
    for name, g, o in zip("ABCG", got, orc[:4]):
        assert rel_fro(g, o) <= 1e-4, name
    assert abs(loss[0] - orc[4][0]) <= 1e-3 * abs(orc[4][0])


def test_decompose_random_start_matches_the_oracle(ctx):
    case = planted_case(P=4, T=16)
    print("decompose random start", flush=True)
    # epochs = 0 returns the start itself
    start, _, _ = _decompose(ctx, case, 0, None)
    again, _, _ = _decompose(ctx, case, 0, None)
    for u, v in zip(start, again):
        np.testing.assert_array_equal(u, v)
    # the oracle's draw, written separately from the same definitions
    ref = oracle.random_start(oracle_problem(case))
    for name, g, o in zip("ABCG", start, ref):
        np.testing.assert_allclose(g, o, rtol=2e-7, atol=1e-30, err_msg=name)
    # one epoch from the random start against the oracle from its own draw
    got, loss, _ = _decompose(ctx, case, 1, None)
    orc = oracle.run(oracle_problem(case), *ref, 1)
    for name, g, o in zip("ABCG", got, orc[:4]):
        assert rel_fro(g, o) <= 1e-4, name
    assert abs(loss[0] - orc[4][0]) <= 1e-3 * abs(orc[4][0])
    # another plan seed draws another start
    other = dict(case)
    other["seed"] = case["seed"] + 1
    s2, _, _ = _decompose(ctx, other, 0, None)
    assert not np.allclose(s2[0], start[0])


def test_decompose_errors(ctx):
    import paper_1711_08095_amd as sn
    bad = planted_case(nnz=500, edges=10)
    bad["P"] = 0
    with pytest.raises(sn.SnectError) as e:
        _decompose(ctx, bad, 1, None)
    assert e.value.code == -1
