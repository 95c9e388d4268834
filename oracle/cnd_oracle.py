"""ctypes front end of the CPU oracle (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It wraps ``gapa_oracle.c`` (plain C, built into ``liboracle.so``)
and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ST_INIT, ST_SELECT, ST_XOVER, ST_REPAIR, ST_MUTATE = 0, 1, 2, 3, 4

_lib = None
_lock = threading.Lock()


class OracleParams(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("k", C.c_int32), ("pop", C.c_int32), ("offspring", C.c_int32),
        ("tournament", C.c_int32), ("objective", C.c_int32),
        ("seed", C.c_uint64), ("t_pc", C.c_uint64), ("t_pm", C.c_uint64),
    ]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                from . import build_oracle  # builds from source with gcc
                build_oracle.build()
            L = C.CDLL(LIB_PATH)
            i32p = C.POINTER(C.c_int32)
            i64p = C.POINTER(C.c_int64)
            u32p = C.POINTER(C.c_uint32)
            L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
            L.oracle_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, u32p]
            L.oracle_bounded.argtypes = [C.c_uint32, C.c_uint32]
            L.oracle_bounded.restype = C.c_uint32
            L.oracle_threshold.argtypes = [C.c_double]
            L.oracle_threshold.restype = C.c_uint64
            for fn in (L.oracle_pc_bfs, L.oracle_pc_unionfind):
                fn.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, i32p]
                fn.restype = C.c_int64
            L.oracle_components.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, i32p]
            L.oracle_components.restype = C.c_int64
            L.oracle_eval_population.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, C.c_int32, i64p, i32p, C.c_int32]
            L.oracle_eval_population.restype = C.c_int64
            pp = C.POINTER(OracleParams)
            L.oracle_init_individual.argtypes = [pp, C.c_int32, i32p]
            L.oracle_tournament.argtypes = [pp, C.c_int32, C.c_int32, i64p]
            L.oracle_tournament.restype = C.c_int32
            L.oracle_make_child.argtypes = [pp, C.c_int32, C.c_int32, i32p, i64p, i32p, i32p, i32p, i32p]
            L.oracle_ga_init.argtypes = [pp, C.c_int32, i32p, i32p, i32p, i64p, C.c_int32]
            L.oracle_ga_step.argtypes = [pp, C.c_int32, C.c_int32, i32p, i32p, i32p, i64p, i32p, C.c_int32, i32p, i64p, C.c_int32]
            L.oracle_max_threads.restype = C.c_int
            L.oracle_uniform_sym.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int32, C.c_double,
                                             C.POINTER(C.c_double)]
            _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def default_threads() -> int:
    return int(lib().oracle_max_threads())


# --- random numbers ---------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    kk = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, C.c_uint32), _p(kk, C.c_uint32), _p(out, C.c_uint32))
    return out


def draw(seed, slot, ind, gen, stream, attempt=0) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_draw(seed, slot, ind, gen, stream, attempt, _p(out, C.c_uint32))
    return out


def uniform_sym(seed: int, tensor: int, rows: int, cols: int, bound: float) -> np.ndarray:
    """[rows, cols] float64: element (r, c) = bound * (2u - 1), u from the
    first word of draw(seed, slot c, ind r, gen tensor, stream 5)."""
    out = np.zeros((rows, cols), dtype=np.float64)
    lib().oracle_uniform_sym(seed, tensor, rows, cols, bound, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def bounded(w: int, m: int) -> int:
    return int(lib().oracle_bounded(w, m))


def threshold(p: float) -> int:
    return int(lib().oracle_threshold(p))


# --- fitness ----------------------------------------------------------------

def pc(graph, genes, method: str = "bfs") -> tuple[int, int]:
    """(PC, MCN) of the graph with the nodes in ``genes`` removed."""
    g = _i32(genes).ravel()
    mcn = C.c_int32(0)
    fn = lib().oracle_pc_bfs if method == "bfs" else lib().oracle_pc_unionfind
    val = fn(graph.n, _p(graph.row_ptr, C.c_int32), _p(graph.col_idx, C.c_int32),
             _p(g, C.c_int32), int(g.shape[0]), C.byref(mcn))
    if val < 0:
        raise ValueError("gene out of range")
    return int(val), int(mcn.value)


def components(graph, genes) -> tuple[int, int]:
    """(number of connected components of G - S, |V minus S|) for the nodes
    in ``genes`` removed; isolated survivors are components of their own."""
    g = _i32(genes).ravel()
    alive = C.c_int32(0)
    val = lib().oracle_components(graph.n, _p(graph.row_ptr, C.c_int32), _p(graph.col_idx, C.c_int32),
                                  _p(g, C.c_int32), int(g.shape[0]), C.byref(alive))
    if val < 0:
        raise ValueError("gene out of range")
    return int(val), int(alive.value)


def eval_population(graph, genes: np.ndarray, nthreads: int | None = None, want_mcn: bool = False):
    G = _i32(genes)
    P, k = G.shape
    F = np.zeros(P, dtype=np.int64)
    M = np.zeros(P, dtype=np.int32)
    nt = default_threads() if nthreads is None else nthreads
    bad = lib().oracle_eval_population(graph.n, _p(graph.row_ptr, C.c_int32), _p(graph.col_idx, C.c_int32),
                                       _p(G, C.c_int32), P, k, _p(F, C.c_int64), _p(M, C.c_int32), nt)
    if bad:
        raise ValueError(f"gene out of range in row {bad - 1}")
    return (F, M) if want_mcn else F


# --- the paper's dense reachability fitness (SixDST) ---------------------------

def sixdst(graph, genes, hops: int) -> tuple[int, int]:
    """The dense reachability fitness of Sec. III-D (eq. 13-17) for one
    removal set: A_S is the adjacency matrix with every edge of a removed
    node deleted (eq. 13), M = Normalizer((A_S + I)^hops) with the power
    taken as `hops` successive products, each normalised (entries > 0 become
    1; normalising in between leaves the support of the power unchanged).
    Row i of M marks the nodes within `hops` hops of i, itself included; a
    removed node's row is its own unit entry.  Returns
    ((sum(M) - n) / 2, the largest row sum over surviving nodes (0 when
    none survive)).  With hops at least the diameter of every component of
    G[V minus S] the pair is (PC, MCN) exactly (eq. 16-17); the paper's
    choice hops = 6 (eq. 15) is the truncation.  Dense products: for small
    graphs only.  They are taken in float64 (a BLAS product): every entry is
    a count of at most n < 2^53 paths of 0/1 entries, so the float64 product
    is the exact integer product."""
    n = graph.n
    S = np.unique(np.asarray(genes, dtype=np.int64).ravel())
    if S.size and (S.min() < 0 or S.max() >= n):
        raise ValueError("gene out of range")
    if hops < 1:
        raise ValueError("hops must be at least 1")
    A = np.zeros((n, n), dtype=np.int64)
    for v in range(n):
        A[v, graph.col_idx[graph.row_ptr[v]:graph.row_ptr[v + 1]]] = 1
    A[S, :] = 0
    A[:, S] = 0
    step = (A + np.eye(n, dtype=np.int64)).astype(np.float64)
    M = step.copy()
    for _ in range(hops - 1):
        M = ((M @ step) > 0).astype(np.float64)
    M = M.astype(np.int64)
    alive = np.ones(n, dtype=bool)
    alive[S] = False
    rows = M.sum(axis=1)
    total = int(M.sum())
    mcn = int(rows[alive].max()) if alive.any() else 0
    return (total - n) // 2, mcn


# --- genetic algorithm --------------------------------------------------------

OBJECTIVES = {"pc": 0, "mcn": 1, "components": 2}


def make_params(n, k, pop, seed, pc=0.7, pm=0.05, tournament=2, offspring=0, objective="pc") -> OracleParams:
    return OracleParams(n=n, k=k, pop=pop, offspring=offspring or pop, tournament=tournament,
                        objective=OBJECTIVES[objective], seed=seed, t_pc=threshold(pc), t_pm=threshold(pm))


class OracleGA:
    """The GA run on the host: generation 0 at construction, ``step()`` for
    each further generation.  ``pop`` is [P, k] int32 and ``F`` [P] int64,
    ordered by (F, tag).  F is PC; with objective="mcn" the largest
    surviving component (the CND fitness of Sec. III-D); with
    objective="components" |V minus S| minus the number of components of
    G - S, so that minimising F maximises the number of components."""

    def __init__(self, graph, k, pop, seed, pc=0.7, pm=0.05, tournament=2, offspring=0, nthreads=None,
                 objective="pc"):
        self.graph = graph
        self.params = make_params(graph.n, k, pop, seed, pc, pm, tournament, offspring, objective)
        self.nthreads = default_threads() if nthreads is None else nthreads
        self.pop = np.zeros((pop, k), dtype=np.int32)
        self.F = np.zeros(pop, dtype=np.int64)
        rc = lib().oracle_ga_init(C.byref(self.params), graph.n, _p(graph.row_ptr, C.c_int32),
                                  _p(graph.col_idx, C.c_int32), _p(self.pop, C.c_int32), _p(self.F, C.c_int64),
                                  self.nthreads)
        if rc != 0:
            raise RuntimeError("oracle init failed")
        self.generation = 0

    def step(self, pool_idx=None, keep_children=False):
        p = self.params
        g = self.generation + 1
        kids = np.zeros((p.offspring, p.k), dtype=np.int32) if keep_children else None
        kf = np.zeros(p.offspring, dtype=np.int64) if keep_children else None
        if pool_idx is not None:
            pi = _i32(pool_idx)
            pptr, npool = _p(pi, C.c_int32), int(pi.shape[0])
        else:
            pptr, npool = None, 0
        rc = lib().oracle_ga_step(C.byref(p), g, self.graph.n, _p(self.graph.row_ptr, C.c_int32),
                                  _p(self.graph.col_idx, C.c_int32), _p(self.pop, C.c_int32), _p(self.F, C.c_int64),
                                  pptr, npool,
                                  _p(kids, C.c_int32) if kids is not None else None,
                                  _p(kf, C.c_int64) if kf is not None else None, self.nthreads)
        if rc != 0:
            raise RuntimeError("oracle step failed")
        self.generation = g
        return (kids, kf) if keep_children else None


def make_child(params: OracleParams, gen: int, o: int, pop: np.ndarray, F: np.ndarray):
    """One offspring without evaluation: returns (child_sorted, pre_repair,
    pre_mutation, donor_index)."""
    pop = _i32(pop)
    F = np.ascontiguousarray(F, dtype=np.int64)
    k = params.k
    child = np.zeros(k, dtype=np.int32)
    pre_r = np.zeros(k, dtype=np.int32)
    pre_m = np.zeros(k, dtype=np.int32)
    d = C.c_int32(-1)
    rc = lib().oracle_make_child(C.byref(params), gen, o, _p(pop, C.c_int32), _p(F, C.c_int64),
                                 _p(child, C.c_int32), _p(pre_r, C.c_int32), _p(pre_m, C.c_int32), C.byref(d))
    if rc != 0:
        raise RuntimeError("oracle make_child failed")
    return child, pre_r, pre_m, int(d.value)


def init_individual(params: OracleParams, i: int) -> np.ndarray:
    row = np.zeros(params.k, dtype=np.int32)
    if lib().oracle_init_individual(C.byref(params), i, _p(row, C.c_int32)) != 0:
        raise RuntimeError("oracle init_individual failed")
    return row


def tournament(params: OracleParams, gen: int, o: int, F: np.ndarray) -> int:
    F = np.ascontiguousarray(F, dtype=np.int64)
    return int(lib().oracle_tournament(C.byref(params), gen, o, _p(F, C.c_int64)))
