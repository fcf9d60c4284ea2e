"""Shared set-up for the parity tests: seeded problems, the oracle run and
the HIP run on the same inputs."""
from __future__ import annotations

import numpy as np

import oracle
import snect_synth as synth


def rel_fro(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def planted_case(seed=synth.DATA_SEED, dims=(200, 500, 5), ranks=(5, 5, 2), nnz=20000, edges=2000,
                 lam=0.01, lam_g=0.1, lr=1e-3, cls=1.0, P=8, T=64, plan_seed=synth.PLAN_SEED,
                 init_seed=synth.INIT_SEED, sigma=1.0):
    """Planted Tucker tensor (the tiny workload by default).  Values are the
    oracle's model at the planted factors plus the drawn noise, rounded to
    float32 so that both sides read identical inputs."""
    p = synth.planted(seed=seed, dims=dims, ranks=ranks, nnz=nnz, edges=edges)
    pr0 = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, np.zeros(nnz))
    x = (oracle.model_values(pr0, p.A, p.B, p.C, p.G) + p.noise).astype(np.float32)
    A, B, C, G = synth.normal_init(init_seed, dims, ranks, sigma)
    case = dict(dims=dims, ranks=ranks, i=p.i, j=p.j, k=p.k, x=x, eu=p.eu, ev=p.ev, ew=None,
                lam=lam, lam_g=lam_g, lr=lr, cls=cls, P=P, T=T, seed=plan_seed,
                init=tuple(a.astype(np.float32) for a in (A, B, C, G)))
    return case


def oracle_problem(case) -> oracle.Problem:
    return oracle.Problem(case["dims"], case["ranks"], case["i"], case["j"], case["k"],
                          np.asarray(case["x"], np.float64), case["eu"], case["ev"],
                          None if case["ew"] is None else np.asarray(case["ew"], np.float64),
                          lam=case["lam"], lam_g=case["lam_g"], lr=case["lr"],
                          core_lr_scale=case["cls"], P=case["P"], T=case["T"], seed=case["seed"])


def run_oracle(case, epochs, start_epoch=0, threads=0):
    A, B, C, G = (np.asarray(a, np.float64) for a in case["init"])
    return oracle.run(oracle_problem(case), A, B, C, G, epochs, start_epoch=start_epoch,
                      threads=threads)


def gpu_problem(ctx, case, precision=0):
    import paper_1711_08095_amd as sn
    hyper = sn.Hyper(ranks=case["ranks"], lam=case["lam"], lam_g=case["lam_g"], lr=case["lr"],
                     core_lr_scale=case["cls"], P=case["P"], T=case["T"], precision=precision,
                     seed=case["seed"])
    return sn.Problem(ctx, case["dims"], case["i"], case["j"], case["k"], case["x"], case["eu"],
                      case["ev"], case["ew"], hyper)


def gpu_factors(case, device="cuda"):
    import torch
    return [torch.tensor(np.asarray(a, np.float32), device=device).contiguous() for a in case["init"]]


def run_gpu(ctx, case, epochs, start_epoch=0, precision=0, factors=None, prob=None):
    prob = prob or gpu_problem(ctx, case, precision)
    f = factors if factors is not None else gpu_factors(case)
    loss, rmse = prob.train(*f, epochs=epochs, start_epoch=start_epoch)
    return [t.double().cpu().numpy() for t in f], loss, rmse, prob
