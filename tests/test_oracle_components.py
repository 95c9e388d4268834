"""Pins of the oracle's component count and of the GA objective that
maximises it (CPU only).

The number of connected components NC(G - S) is read off the same component
partition as PC and MCN (Sec. III-D obtains component sizes from the rows of
the reachability matrix); the paper reports only PC and MCN, so this objective
is an extension.  The GA minimises |V minus S| - NC: the size of a spanning
forest of G - S, zero exactly when no surviving edge is left.

Checked against closed forms (complete graph, path, cycle, star, disjoint
cliques, an edgeless graph), SciPy's connected components, and the forest
identity on trees: an induced subgraph of a tree is a forest, so
|V minus S| - NC equals its edge count.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as cg

from oracle import cnd_oracle as O
from paper_2412_20980_amd import inputs


def complete(n):
    u, v = np.triu_indices(n, 1)
    return inputs.csr_from_edges(n, u, v)


def path(n):
    return inputs.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))


def cycle(n):
    return inputs.csr_from_edges(n, np.arange(n), (np.arange(n) + 1) % n)


def star(n):
    return inputs.csr_from_edges(n, np.zeros(n - 1, dtype=int), np.arange(1, n))


def scipy_components(g, S):
    alive = np.ones(g.n, bool)
    alive[np.asarray(S, dtype=int)] = False
    idx = np.nonzero(alive)[0]
    if idx.size == 0:
        return 0
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    return int(cg.connected_components(A[idx][:, idx], directed=False)[0])


def test_closed_forms():
    assert O.components(complete(12), [0, 5, 7]) == (1, 9)
    assert O.components(complete(5), [0, 1, 2, 3, 4]) == (0, 0)
    # a path cut at interior nodes: one component per non-empty segment
    assert O.components(path(10), [3, 6]) == (3, 8)
    assert O.components(path(10), [0, 1, 9]) == (1, 7)
    assert O.components(path(10), [1, 3, 5, 7]) == (5, 6)
    # a cycle minus j separated nodes falls into j arcs
    assert O.components(cycle(12), [0, 4, 8]) == (3, 9)
    assert O.components(cycle(12), []) == (1, 12)
    # a star without its centre: every leaf alone
    assert O.components(star(9), [0]) == (8, 8)
    assert O.components(star(9), [3]) == (1, 8)
    # no edges: every survivor alone
    empty = inputs.csr_from_edges(7, np.zeros(0, int), np.zeros(0, int))
    assert O.components(empty, [2, 4]) == (5, 5)


def test_disjoint_cliques():
    sizes = [4, 6, 3, 5]
    u, v, off = [], [], 0
    for s in sizes:
        a, b = np.triu_indices(s, 1)
        u.append(a + off)
        v.append(b + off)
        off += s
    g = inputs.csr_from_edges(off, np.concatenate(u), np.concatenate(v))
    assert O.components(g, []) == (4, 18)
    # emptying the second clique removes its component
    assert O.components(g, list(range(4, 10))) == (3, 12)
    # repeated genes are one removal
    assert O.components(g, [0, 0, 1]) == (4, 16)


def test_matches_scipy():
    rng = np.random.default_rng(5)
    for gen, seed in ((lambda s: inputs.erdos_renyi(400, 1.5, seed=s), 1),
                      (lambda s: inputs.barabasi_albert(300, 2, seed=s), 2),
                      (lambda s: inputs.chung_lu(500, 2.5, 3.0, 800, seed=s), 3)):
        g = gen(seed)
        for _ in range(6):
            S = rng.choice(g.n, size=int(rng.integers(0, g.n // 4)), replace=False)
            nc, alive = O.components(g, S)
            assert alive == g.n - S.size
            assert nc == scipy_components(g, S)


def test_forest_identity_on_trees():
    # BA with m = 1 is a tree; G - S is then a forest whose edge count is
    # |V minus S| - NC
    g = inputs.barabasi_albert(500, 1, seed=9)
    assert g.m == g.n - 1
    rng = np.random.default_rng(1)
    for _ in range(10):
        S = rng.choice(g.n, size=40, replace=False)
        dead = np.zeros(g.n, bool)
        dead[S] = True
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        surviving_edges = int(np.sum(~dead[src] & ~dead[g.col_idx])) // 2
        nc, alive = O.components(g, S)
        assert alive - nc == surviving_edges


def test_invariants_against_pc():
    g = inputs.erdos_renyi(300, 2.0, seed=4)
    rng = np.random.default_rng(2)
    for _ in range(10):
        S = rng.choice(g.n, size=30, replace=False)
        nc, alive = O.components(g, S)
        pc, mcn = O.pc(g, S)
        assert 1 <= nc <= alive
        # the largest component and nc - 1 others of size >= 1
        assert mcn + (nc - 1) <= alive
        assert (pc == 0) == (nc == alive)


def test_out_of_range_gene():
    with pytest.raises(ValueError):
        O.components(path(5), [5])


def test_ga_objective_is_survivors_minus_components():
    g = inputs.erdos_renyi(300, 3.0, seed=21)
    ga = O.OracleGA(g, 15, 24, 7, 0.7, 0.1, 2, 40, objective="components")
    best = []
    for _ in range(8):
        for row, f in zip(ga.pop, ga.F):
            nc, alive = O.components(g, row)
            assert f == alive - nc
        assert np.all(np.diff(ga.F) >= 0)
        best.append(int(ga.F[0]))
        ga.step()
    assert all(b >= a for a, b in zip(best[1:], best[:-1]))
    # a different objective moves the search elsewhere
    other = O.OracleGA(g, 15, 24, 7, 0.7, 0.1, 2, 40)
    for _ in range(3):
        other.step()
    assert not np.array_equal(other.pop, ga.pop)
