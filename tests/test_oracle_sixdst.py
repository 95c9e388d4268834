"""The oracle's dense reachability fitness (Sec. III-D, eq. 13-17) against
closed forms and the exact components.

Pairs within h hops on a path of n nodes: sum_{d=1..min(h, n-1)} (n - d); the
largest h-hop neighbourhood (itself included) of a path node: min(n, 2h + 1).
On a cycle of n nodes with 2h < n: n h pairs and 2h + 1.  One hop: the
surviving edges.  With h at least the diameter the pair is (PC, MCN) of the
components (BFS)."""
import numpy as np
import pytest

from oracle import cnd_oracle as O
from paper_2412_20980_amd import inputs


class _G:
    def __init__(self, n, adj):
        self.n = n
        rp, ci = [0], []
        for v in range(n):
            ci += sorted(adj[v])
            rp.append(len(ci))
        self.row_ptr = np.array(rp, dtype=np.int32)
        self.col_idx = np.array(ci, dtype=np.int32)


def path(n):
    return _G(n, [[u for u in (v - 1, v + 1) if 0 <= u < n] for v in range(n)])


def cycle(n):
    return _G(n, [[(v - 1) % n, (v + 1) % n] for v in range(n)])


@pytest.mark.parametrize("n,h", [(20, 6), (20, 1), (7, 6), (13, 3), (30, 12)])
def test_path_closed_form(n, h):
    pairs = sum(n - d for d in range(1, min(h, n - 1) + 1))
    assert O.sixdst(path(n), [], h) == (pairs, min(n, 2 * h + 1))


@pytest.mark.parametrize("n,h", [(33, 6), (15, 3), (40, 1)])
def test_cycle_closed_form(n, h):
    assert 2 * h < n
    assert O.sixdst(cycle(n), [], h) == (n * h, 2 * h + 1)


def test_removed_node_splits_the_path():
    # node 10 of a 20-node path removed: paths of 10 and 9 nodes
    assert O.sixdst(path(20), [10], 25) == (45 + 36, 10)
    # six hops: within each piece, pairs at distance <= 6
    left = sum(10 - d for d in range(1, 7))
    right = sum(9 - d for d in range(1, 7))
    assert O.sixdst(path(20), [10], 6) == (left + right, 10)


def test_one_hop_counts_surviving_edges():
    g = inputs.erdos_renyi(80, 4.0, seed=3)
    rng = np.random.default_rng(1)
    for _ in range(5):
        S = rng.choice(g.n, size=10, replace=False)
        alive = np.ones(g.n, bool)
        alive[S] = False
        edges = sum(1 for v in range(g.n) for u in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
                    if v < u and alive[v] and alive[u])
        deg = [sum(1 for u in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]] if alive[u]) for v in range(g.n)]
        pc1, mcn1 = O.sixdst(g, S, 1)
        assert pc1 == edges
        assert mcn1 == 1 + max(d for d, a in zip(deg, alive) if a)


def test_enough_hops_give_the_components():
    rng = np.random.default_rng(2)
    for g in [inputs.barabasi_albert(60, 1, seed=4), inputs.erdos_renyi(70, 2.0, seed=5)]:
        for _ in range(4):
            S = rng.choice(g.n, size=rng.integers(0, 15), replace=False)
            assert O.sixdst(g, S, g.n) == O.pc(g, S)


def test_hops_are_monotone_and_everything_removed():
    g = inputs.barabasi_albert(50, 2, seed=6)
    vals = [O.sixdst(g, [0, 1], h) for h in range(1, 8)]
    assert all(a[0] <= b[0] and a[1] <= b[1] for a, b in zip(vals, vals[1:]))
    assert O.sixdst(path(5), range(5), 6) == (0, 0)
