"""Seeded synthetic inputs for SNeCT workloads.

This module only draws random inputs: index sets, values, graphs, factor
initialisations and request streams.  It holds none of the method's
arithmetic (no reconstruction, no loss, no update rule), so both the FP64
oracle and the HIP path can consume what it produces without sharing code.

The paper's data (the PanCan12 tensor of Section 2.1.1 and the PathwayCommons
gene network of Section 2.1.2) is not available; the generators below stand
in for it with the paper's shapes (patient x gene x platform, about
4.5k x 14k x 5) and value types per platform.  Every generator takes an
explicit integer seed and uses numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Seed conventions: data, init and plan seeds per workload index.
DATA_SEED = 1000
INIT_SEED = 2000
PLAN_SEED = 3000


@dataclasses.dataclass
class Problem:
    """A sparse 3-mode tensor, a gene graph and the hyper-parameters."""

    dims: tuple            # (I1, I2, I3)
    ranks: tuple           # (J1, J2, J3)
    i: np.ndarray          # int32[nnz], patient index (0-based)
    j: np.ndarray          # int32[nnz], gene index
    k: np.ndarray          # int32[nnz], platform index
    x: np.ndarray          # float32[nnz] (float64 copy in x64)
    eu: np.ndarray         # int32[E] edge endpoint
    ev: np.ndarray         # int32[E] edge endpoint
    ew: Optional[np.ndarray]  # float32[E] or None (= 1)
    lam: float = 0.01
    lam_g: float = 0.1
    lr: float = 1e-3
    core_lr_scale: float = 1.0
    epochs: int = 10
    strata: int = 8
    tile: int = 64
    seed: int = PLAN_SEED
    name: str = ""
    x64: Optional[np.ndarray] = None  # exact float64 values when planted

    @property
    def nnz(self) -> int:
        return int(self.i.shape[0])


def sample_cells(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    """m distinct integers drawn uniformly without replacement from [0, n)."""
    if m > n:
        raise ValueError("cannot draw more distinct cells than exist")
    if m == 0:
        return np.zeros(0, dtype=np.int64)
    if m * 4 >= n:
        return np.sort(rng.permutation(n)[:m]).astype(np.int64)
    draw = max(int(m * 1.25) + 64, m + 64)
    while True:
        cand = np.unique(rng.integers(0, n, size=draw, dtype=np.int64))
        if cand.shape[0] >= m:
            # a uniformly random m-subset of the distinct draws is a uniformly
            # random m-subset of [0, n) by exchangeability
            pick = rng.permutation(cand.shape[0])[:m]
            return np.sort(cand[pick])
        draw = int(draw * 1.5)


def erdos_renyi_edges(rng: np.random.Generator, n: int, m: int):
    """G(n, M): m distinct undirected pairs u < v, no self-loops."""
    total = n * (n - 1) // 2
    codes = sample_cells(rng, total, m)
    # decode the pair index into (u, v) with u < v (row-major upper triangle)
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    # row r starts at r*n - r*(r+1)/2
    starts = np.array([r * n - r * (r + 1) // 2 for r in range(n)], dtype=np.int64)
    r = np.searchsorted(starts, codes, side="right") - 1
    u[:] = r
    v[:] = codes - starts[r] + r + 1
    perm = rng.permutation(m)
    return u[perm].astype(np.int32), v[perm].astype(np.int32)


def barabasi_albert_edges(rng: np.random.Generator, n: int, m: int):
    """Preferential attachment: a star on m+1 nodes, then each new node links
    to m distinct earlier nodes drawn with probability proportional to
    degree.  Gives m + (n-m-1)*m edges (139,900 for n=14,000, m=10)."""
    us = []
    vs = []
    # initial star: node 0 joined to 1..m
    repeated = []
    for t in range(1, m + 1):
        us.append(0)
        vs.append(t)
        repeated += [0, t]
    rep = np.zeros(2 * (m + (n - m - 1) * m), dtype=np.int64)
    rep[: len(repeated)] = repeated
    rlen = len(repeated)
    for src in range(m + 1, n):
        chosen = set()
        while len(chosen) < m:
            need = m - len(chosen)
            picks = rep[rng.integers(0, rlen, size=need * 2)]
            for t in picks.tolist():
                if t not in chosen:
                    chosen.add(t)
                    if len(chosen) == m:
                        break
        tg = sorted(chosen)
        for t in tg:
            us.append(src)
            vs.append(t)
        rep[rlen: rlen + m] = tg
        rep[rlen + m: rlen + 2 * m] = src
        rlen += 2 * m
    u = np.asarray(us, dtype=np.int32)
    v = np.asarray(vs, dtype=np.int32)
    perm = rng.permutation(u.shape[0])
    return u[perm], v[perm]


def normal_init(seed: int, dims, ranks, sigma: float):
    """i.i.d. N(0, sigma^2) factors and core (float64), drawn in the order
    A, B, C, G."""
    rng = np.random.default_rng(seed)
    I1, I2, I3 = dims
    J1, J2, J3 = ranks
    A = rng.standard_normal((I1, J1)) * sigma
    B = rng.standard_normal((I2, J2)) * sigma
    C = rng.standard_normal((I3, J3)) * sigma
    G = rng.standard_normal((J1, J2, J3)) * sigma
    return A, B, C, G


def default_sigma(x: np.ndarray, ranks) -> float:
    """Init scale (mean(x^2) / (J1 J2 J3))^(1/8): with four i.i.d. N(0, s^2)
    terms per product, the model's value scale then matches the data's."""
    J1, J2, J3 = ranks
    if x.shape[0] == 0:
        return 1.0
    ms = float(np.mean(np.asarray(x, dtype=np.float64) ** 2))
    if ms <= 0.0:
        return 1.0
    return (ms / (J1 * J2 * J3)) ** 0.125


# --------------------------------------------------------------------------
# Planted low-rank tensor (tiny workload): the caller turns the planted
# factors into values with its own reconstruction and adds `noise`.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Planted:
    dims: tuple
    ranks: tuple
    i: np.ndarray
    j: np.ndarray
    k: np.ndarray
    noise: np.ndarray      # float64[nnz]
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    G: np.ndarray
    eu: np.ndarray
    ev: np.ndarray


def planted(seed: int = DATA_SEED, dims=(200, 500, 5), ranks=(5, 5, 2),
            nnz: int = 20000, noise_sd: float = 0.1, edges: int = 2000) -> Planted:
    """Tiny planted Tucker tensor: N(0,1) core and factors, `nnz` distinct
    cells uniform without replacement, N(0, noise_sd^2) noise, and an
    Erdos-Renyi gene graph with `edges` distinct pairs."""
    rng = np.random.default_rng(seed)
    I1, I2, I3 = dims
    J1, J2, J3 = ranks
    G = rng.standard_normal((J1, J2, J3))
    A = rng.standard_normal((I1, J1))
    B = rng.standard_normal((I2, J2))
    C = rng.standard_normal((I3, J3))
    cells = sample_cells(rng, I1 * I2 * I3, nnz)
    cells = cells[rng.permutation(nnz)]
    i = (cells // (I2 * I3)).astype(np.int32)
    j = ((cells // I3) % I2).astype(np.int32)
    k = (cells % I3).astype(np.int32)
    noise = rng.standard_normal(nnz) * noise_sd
    if edges > 0 and I2 > 1:
        eu, ev = erdos_renyi_edges(rng, I2, edges)
    else:
        eu = np.zeros(0, np.int32)
        ev = np.zeros(0, np.int32)
    return Planted(dims, ranks, i, j, k, noise, A, B, C, G, eu, ev)


# --------------------------------------------------------------------------
# PanCan-shaped tensor: per-platform value types of the paper's Table 1.
# --------------------------------------------------------------------------
def pancan_like(seed: int = DATA_SEED + 1, I1: int = 4500, I2: int = 14000,
                nnz: int = 25_000_000, ba_m: int = 10, mut_density: float = 0.03,
                protein_gene_frac: float = 0.02, graph: bool = True):
    """Five platforms over I1 patients x I2 genes:
      k=0 binary mutation, value 1.0 on mut_density of the patient x gene cells;
      k=4 protein-like N(0,1) on all patients x a random protein_gene_frac of genes;
      k=1, k=2 expression / methylation z-scores N(0,1);
      k=3 integer copy number in {-2..2}, P(0)=.5, P(+-1)=.2, P(+-2)=.05;
    the remaining nonzeros split evenly over k=1..3 (the remainder to k=1).
    Returns (i, j, k, x, eu, ev) with x float32 and the COO order shuffled."""
    rng = np.random.default_rng(seed)
    cells2 = I1 * I2
    n0 = int(round(mut_density * cells2))
    ng4 = max(1, int(round(protein_gene_frac * I2)))
    n4 = I1 * ng4
    rest = nnz - n0 - n4
    if rest < 0:
        raise ValueError("nnz too small for the fixed platforms")
    n123 = [rest // 3 + (rest % 3), rest // 3, rest // 3]
    parts_i, parts_j, parts_k, parts_x = [], [], [], []
    # platform 0: mutation present
    c = sample_cells(rng, cells2, n0)
    parts_i.append(c // I2); parts_j.append(c % I2)
    parts_k.append(np.zeros(n0, np.int64)); parts_x.append(np.ones(n0))
    # platforms 1..3
    for kk, cnt in zip((1, 2, 3), n123):
        c = sample_cells(rng, cells2, cnt)
        parts_i.append(c // I2); parts_j.append(c % I2)
        parts_k.append(np.full(cnt, kk, np.int64))
        if kk < 3:
            parts_x.append(rng.standard_normal(cnt))
        else:
            parts_x.append(rng.choice(np.array([-2.0, -1.0, 0.0, 1.0, 2.0]), size=cnt,
                                      p=[0.05, 0.2, 0.5, 0.2, 0.05]))
    # platform 4: protein-like on a gene subset, all patients
    genes4 = np.sort(rng.choice(I2, size=ng4, replace=False))
    ii, jj = np.meshgrid(np.arange(I1), genes4, indexing="ij")
    parts_i.append(ii.ravel()); parts_j.append(jj.ravel())
    parts_k.append(np.full(n4, 4, np.int64)); parts_x.append(rng.standard_normal(n4))
    i = np.concatenate(parts_i).astype(np.int32)
    j = np.concatenate(parts_j).astype(np.int32)
    k = np.concatenate(parts_k).astype(np.int32)
    x = np.concatenate(parts_x).astype(np.float32)
    perm = rng.permutation(i.shape[0])
    i, j, k, x = i[perm], j[perm], k[perm], x[perm]
    if graph:
        eu, ev = barabasi_albert_edges(rng, I2, ba_m)
    else:
        eu = np.zeros(0, np.int32); ev = np.zeros(0, np.int32)
    return i, j, k, x, eu, ev


def pancan_problem(ranks=(10, 10, 5), nnz: int = 25_000_000, I1: int = 4500,
                   I2: int = 14000, epochs: int = 20, strata: int = 128,
                   tile: int = 64, seed: int = DATA_SEED + 1) -> Problem:
    i, j, k, x, eu, ev = pancan_like(seed=seed, I1=I1, I2=I2, nnz=nnz)
    return Problem(dims=(I1, I2, 5), ranks=tuple(ranks), i=i, j=j, k=k, x=x,
                   eu=eu, ev=ev, ew=None, lam=0.01, lam_g=0.1, lr=1e-3,
                   core_lr_scale=1.0, epochs=epochs, strata=strata, tile=tile,
                   seed=PLAN_SEED + 1, name="pancan")


def sweep_specs(seed: int = DATA_SEED + 3, count: int = 16, scale: float = 1.0):
    """Sixteen uneven decompositions: J1, J2 in {5,10,15,20}, J3 in {2,5},
    I1 ~ U[1000, 4500], I2 ~ U[5000, 14000], I3 = 5, nnz ~ U[1M, 10M]
    (times `scale`), lambda_g cycling {0, 0.01, 0.1, 1}."""
    rng = np.random.default_rng(seed)
    specs = []
    lg = [0.0, 0.01, 0.1, 1.0]
    for t in range(count):
        J1 = int(rng.choice([5, 10, 15, 20]))
        J2 = int(rng.choice([5, 10, 15, 20]))
        J3 = int(rng.choice([2, 5]))
        I1 = int(rng.integers(1000, 4501))
        I2 = int(rng.integers(5000, 14001))
        nnz = int(rng.integers(1_000_000, 10_000_001) * scale)
        specs.append(dict(dims=(I1, I2, 5), ranks=(J1, J2, J3), nnz=nnz,
                          lam_g=lg[t % 4], seed=int(rng.integers(1 << 31))))
    return specs


def fold_in_requests(seed: int = DATA_SEED + 4, count: int = 10000, I2: int = 14000,
                     I3: int = 5, rate: float = 2000.0, nnz_lo: int = 2000,
                     nnz_hi: int = 60000):
    """Open-loop Poisson arrivals (seeded exponential gaps) of new-patient
    profiles: nnz ~ U{nnz_lo..nnz_hi} distinct (gene, platform) cells with
    per-platform values as in `pancan_like`.  Returns a list of dicts with
    arrival time (s), j, k (int32) and x (float32)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.integers(nnz_lo, nnz_hi + 1))
        c = sample_cells(rng, I2 * I3, n)
        j = (c // I3).astype(np.int32)
        k = (c % I3).astype(np.int32)
        x = rng.standard_normal(n)
        x[k == 0] = 1.0
        m3 = k == 3
        x[m3] = rng.choice(np.array([-2.0, -1.0, 0.0, 1.0, 2.0]), size=int(m3.sum()),
                           p=[0.05, 0.2, 0.5, 0.2, 0.05])
        out.append(dict(arrival=t, j=j, k=k, x=x.astype(np.float32)))
    return out


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


__all__ = [
    "Problem", "Planted", "planted", "pancan_like", "pancan_problem",
    "sweep_specs", "fold_in_requests", "normal_init", "default_sigma",
    "sample_cells", "erdos_renyi_edges", "barabasi_albert_edges",
    "DATA_SEED", "INIT_SEED", "PLAN_SEED", "ceil_div", "math",
]
