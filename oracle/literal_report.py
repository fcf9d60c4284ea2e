"""Convergence of the stratified schedule against Algorithm 1 read literally,
on the tiny planted tensor (200 x 500 x 5, core 5 x 5 x 2, 20,000 cells,
Erdos-Renyi gene graph with 2,000 edges; lambda = 0.01, lambda_g = 0.1,
eta = 1e-3, N(0,1) init).  Everything runs in the FP64 oracle; the GPU path
reproduces the stratified runs to FP32 rounding.

    python -m oracle.literal_report [--epochs 20]

prints one row per epoch: f_opt and training RMSE of
  literal   -- one core, per-nonzero C and G steps, nonzeros and edges
               interleaved in a seeded random order;
  P1T1      -- the stratified schedule with one block and one-nonzero tiles;
  P8T64     -- the stratified schedule of the parity tests.
"""
import argparse
import time

import numpy as np

import oracle
import snect_synth as synth


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=20)
    args = ap.parse_args()
    p = synth.planted()
    pr0 = oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, np.zeros(len(p.i)))
    x = oracle.model_values(pr0, p.A, p.B, p.C, p.G) + p.noise
    init = synth.normal_init(synth.INIT_SEED, p.dims, p.ranks, 1.0)

    def prob(P, T):
        return oracle.Problem(p.dims, p.ranks, p.i, p.j, p.k, x, p.eu, p.ev, lam=0.01, lam_g=0.1,
                              lr=1e-3, P=P, T=T, seed=synth.PLAN_SEED)

    f0, r0, _ = oracle.loss(prob(1, 1), *init)
    runs = {}
    t = time.perf_counter()
    runs["literal"] = oracle.run_literal(prob(1, 1), *init, args.epochs)[4:]
    runs["P1T1"] = oracle.run(prob(1, 1), *init, args.epochs)[4:]
    runs["P8T64"] = oracle.run(prob(8, 64), *init, args.epochs)[4:]
    names = list(runs)
    print(f"# planted 200x500x5, 20000 nnz; initial f_opt {f0:.6g}, RMSE {r0:.6g} "
          f"({time.perf_counter() - t:.1f}s)")
    print("| epoch | " + " | ".join(f"{n} f_opt | {n} RMSE" for n in names) + " |")
    print("|---|" + "---|---|" * len(names))
    for e in range(args.epochs):
        cells = " | ".join(f"{runs[n][0][e]:.6g} | {runs[n][1][e]:.4f}" for n in names)
        print(f"| {e + 1} | {cells} |")


if __name__ == "__main__":
    main()
