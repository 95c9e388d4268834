"""Seeded synthetic inputs: graphs in CSR form and random removal sets.

This module is shared by the CPU oracle and the HIP path. It holds no part of
the method's arithmetic (no connected components, no pairwise connectivity, no
genetic operator): it only builds the undirected, unweighted graphs the method
runs on (Section III-A, problem definition of PSSO) and uniformly random
k-subsets used as populations to evaluate.

Graph families stand in for the paper's critical-node datasets (Table I: small
BA/ER/forest-fire graphs and a protein network), which are not available here:

* ``barabasi_albert``: preferential attachment, ``m`` edges per new node,
  seeded by a star on ``m + 1`` nodes.
* ``chung_lu``: power-law expected degrees ``w_i ~ (i+1)^(-1/(gamma-1))``
  scaled to a target mean, endpoints of a fixed number of edge draws sampled
  i.i.d. proportional to ``w``; self-loops and repeated pairs dropped.
* ``erdos_renyi``: G(n, p) with ``p = avg_deg / (n - 1)``, drawn as a
  binomial edge count followed by distinct uniform pairs.

Every graph is randomly relabelled with the same seed so that vertex id does not
correlate with degree, and is returned as a symmetric, simple CSR with sorted
neighbour lists (``row_ptr`` int32 [n+1], ``col_idx`` int32 [2m]).
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSRGraph:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype="<i4").tobytes())
        h.update(np.ascontiguousarray(self.col_idx, dtype="<i4").tobytes())
        return h.hexdigest()


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "", meta=None) -> CSRGraph:
    """Symmetric simple CSR from an undirected edge list (self-loops and
    repeated pairs are dropped; neighbour lists come out sorted)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSRGraph(n, row_ptr.astype(np.int32), dst.astype(np.int32), name, dict(meta or {}))


def _relabel(n: int, u: np.ndarray, v: np.ndarray, rng: np.random.Generator):
    perm = rng.permutation(n)
    return perm[u], perm[v]


def barabasi_albert(n: int, m: int, seed: int, relabel: bool = True) -> CSRGraph:
    if not (1 <= m < n):
        raise ValueError("need 1 <= m < n")
    rng = np.random.Generator(np.random.PCG64(seed))
    # seed graph: star with centre 0 and leaves 1..m
    us = [0] * m
    vs = list(range(1, m + 1))
    endpoints = np.empty(2 * m * n, dtype=np.int64)
    endpoints[: 2 * m] = np.array(us + vs, dtype=np.int64)
    ne = 2 * m
    eu = np.empty(m * (n - m - 1), dtype=np.int64)
    ev = np.empty(m * (n - m - 1), dtype=np.int64)
    pos = 0
    for new in range(m + 1, n):
        targets: list[int] = []
        while len(targets) < m:
            # draw a batch; keep the first distinct ones in draw order
            draws = endpoints[rng.integers(0, ne, size=2 * m)]
            for t in draws.tolist():
                if t not in targets:
                    targets.append(t)
                    if len(targets) == m:
                        break
        for t in targets:
            eu[pos] = new
            ev[pos] = t
            pos += 1
            endpoints[ne] = new
            endpoints[ne + 1] = t
            ne += 2
    u = np.concatenate([np.array(us, dtype=np.int64), eu[:pos]])
    v = np.concatenate([np.array(vs, dtype=np.int64), ev[:pos]])
    if relabel:
        u, v = _relabel(n, u, v, rng)
    return csr_from_edges(n, u, v, name=f"ba_n{n}_m{m}_s{seed}", meta=dict(kind="ba", n=n, m=m, seed=seed))


def chung_lu(n: int, gamma: float, mean_deg: float, n_pairs: int, seed: int, relabel: bool = True) -> CSRGraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    w *= mean_deg / w.mean()
    p = w / w.sum()
    u = rng.choice(n, size=n_pairs, p=p)
    v = rng.choice(n, size=n_pairs, p=p)
    if relabel:
        u, v = _relabel(n, u, v, rng)
    return csr_from_edges(n, u, v, name=f"cl_n{n}_g{gamma}_d{mean_deg}_s{seed}",
                          meta=dict(kind="chung_lu", n=n, gamma=gamma, mean_deg=mean_deg, pairs=n_pairs, seed=seed))


def erdos_renyi(n: int, avg_deg: float, seed: int, relabel: bool = True) -> CSRGraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    total = n * (n - 1) // 2
    p = min(1.0, avg_deg / max(1, n - 1))
    target = int(rng.binomial(total, p))
    keys = np.empty(0, dtype=np.int64)
    while keys.shape[0] < target:
        need = target - keys.shape[0]
        a = rng.integers(0, n, size=need + need // 8 + 16)
        b = rng.integers(0, n, size=a.shape[0])
        ok = a != b
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        new = lo * n + hi
        # keep first occurrences in draw order, drop pairs already present
        _, first = np.unique(new, return_index=True)
        new = new[np.sort(first)]
        new = new[~np.isin(new, keys)]
        keys = np.concatenate([keys, new[:need]])
    u = keys // n
    v = keys % n
    if relabel:
        u, v = _relabel(n, u, v, rng)
    return csr_from_edges(n, u, v, name=f"er_n{n}_d{avg_deg}_s{seed}", meta=dict(kind="er", n=n, avg_deg=avg_deg, seed=seed))


# ---------------------------------------------------------------------------
# Named workloads (graph + GA shape).  Rates pc/pm and tournament size are the
# same for every workload: 0.7 / 0.05 per gene and T = 2.
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    graph: CSRGraph
    k: int
    pop: int
    generations: int
    seed: int
    pc: float = 0.7
    pm: float = 0.05
    tournament: int = 2
    offspring: int = 0      # 0 -> pop
    exact_top: int = 0      # 0 -> all offspring evaluated exactly


def ba200() -> CSRGraph:
    return barabasi_albert(200, 3, seed=1)


def ba10k() -> CSRGraph:
    return barabasi_albert(10_000, 3, seed=2)


def chung_lu_200k() -> CSRGraph:
    return chung_lu(200_000, 2.5, 10.0, 1_000_000, seed=3)


def workload(name: str) -> Workload:
    if name == "ba200_k10_p32":
        return Workload(name, ba200(), k=10, pop=32, generations=20, seed=0)
    if name == "ba10k_k100_p256":
        return Workload(name, ba10k(), k=100, pop=256, generations=200, seed=0)
    if name == "cl200k_k2000_p1024":
        return Workload(name, chung_lu_200k(), k=2000, pop=1024, generations=500, seed=0)
    if name == "cl200k_k2000_p1024_screen4096":
        return Workload(name, chung_lu_200k(), k=2000, pop=1024, generations=500, seed=0,
                        offspring=4096, exact_top=512)
    raise KeyError(name)


def batched_instance_sizes(count: int = 64, lo: int = 1000, hi: int = 50_000, seed: int = 4) -> list[int]:
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [int(round(math.exp(t))) for t in x]


def batched_instances(count: int = 64, seed: int = 4, sizes: list[int] | None = None) -> list[Workload]:
    """Uneven multi-instance set: even instances BA(n, 3), odd instances ER
    with mean degree 8; budget 1% of n, population 128, 200 generations,
    instance b seeded with b."""
    if sizes is None:
        sizes = batched_instance_sizes(count, seed=seed)
    out = []
    for b, n in enumerate(sizes):
        g = barabasi_albert(n, 3, seed=1000 + b) if b % 2 == 0 else erdos_renyi(n, 8.0, seed=1000 + b)
        out.append(Workload(f"inst{b}", g, k=max(1, n // 100), pop=128, generations=200, seed=b))
    return out


# ---------------------------------------------------------------------------
# Random removal sets
# ---------------------------------------------------------------------------

def random_population(n: int, k: int, P: int, seed: int, sort_rows: bool = True) -> np.ndarray:
    """P distinct k-subsets of range(n), int32 [P, k]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((P, k), dtype=np.int32)
    for i in range(P):
        row = rng.choice(n, size=k, replace=False)
        out[i] = np.sort(row) if sort_rows else row
    return out


def hub_biased_population(g: CSRGraph, k: int, P: int, seed: int, hub_frac: float = 0.5) -> np.ndarray:
    """P k-subsets where about ``hub_frac`` of each row is drawn from the
    highest-degree 2k vertices and the rest uniformly: the shape GA
    populations take once they start to find hubs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = g.degrees()
    top = np.argsort(-deg, kind="stable")[: 2 * k]
    out = np.empty((P, k), dtype=np.int32)
    nh = int(round(hub_frac * k))
    for i in range(P):
        hubs = rng.choice(top, size=nh, replace=False)
        rest_pool = np.setdiff1d(np.arange(g.n), hubs, assume_unique=False)
        rest = rng.choice(rest_pool, size=k - nh, replace=False)
        out[i] = np.sort(np.concatenate([hubs, rest]))
    return out
