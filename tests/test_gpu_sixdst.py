"""The paper's dense reachability fitness (Sec. III-D, eq. 13-17) on the
matrix cores, through the C ABI, against the oracle: exact integers.

Truncated hop counts (the paper's 6, and others) against the oracle's
definition on small graphs whose node counts are not multiples of the
64-node tile; hop counts at least the diameter against the exact
components (the bit-parallel path and the oracle's BFS) at n = 2000 with
enough individuals to need two workspace chunks."""
import numpy as np
import pytest

from oracle import cnd_oracle as O
from paper_2412_20980_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2412_20980_amd import gapa
    return gapa


@pytest.mark.parametrize("name,hops", [("ba150", 6), ("ba150", 1), ("er200", 6), ("er200", 3), ("tree130", 7),
                                       ("tree130", 2), ("er64", 5)])
def test_truncated_hops_match_oracle(gp, name, hops):
    g = {"ba150": lambda: inputs.barabasi_albert(150, 2, seed=1), "er200": lambda: inputs.erdos_renyi(200, 3.0, seed=2),
         "tree130": lambda: inputs.barabasi_albert(130, 1, seed=3), "er64": lambda: inputs.erdos_renyi(64, 2.5, seed=4)}[name]()
    print(f"{name} hops={hops}", flush=True)
    graph = gp.Graph.from_csr(g)
    rng = np.random.default_rng(hops)
    k = max(1, g.n // 20)
    genes = np.stack([rng.choice(g.n, size=k, replace=False) for _ in range(12)]).astype(np.int32)
    pc, mcn = graph.sixdst(genes, hops)
    for i in range(len(genes)):
        assert (int(pc[i]), int(mcn[i])) == O.sixdst(g, genes[i], hops), i


@pytest.mark.parametrize("hops", [6, 3])
def test_multi_tile_truncated_hops_match_oracle(gp, hops):
    """n = 1100: 9 x 9 product tiles of 128, so most tiles are off the
    diagonal and written twice (mirrored); every row of a population of
    removal sets is compared with the oracle's definition.  A sparse random
    graph (mean degree 2.5) keeps many pairs beyond both hop counts, so the
    truncation shows in every value."""
    g = inputs.erdos_renyi(1100, 2.5, seed=21)
    graph = gp.Graph.from_csr(g)
    genes = inputs.random_population(g.n, 30, 10, seed=22)
    # one row that removes the hubs, where truncation matters least
    order = np.argsort(-np.diff(g.row_ptr), kind="stable")
    genes[0] = np.sort(order[:30]).astype(np.int32)
    print(f"n=1100 hops={hops}, 10 rows", flush=True)
    pc, mcn = graph.sixdst(genes, hops)
    for i in range(len(genes)):
        assert (int(pc[i]), int(mcn[i])) == O.sixdst(g, genes[i], hops), i


def test_enough_hops_give_the_components(gp):
    import torch
    g = inputs.barabasi_albert(2000, 2, seed=5)
    graph = gp.Graph.from_csr(g)
    genes = inputs.random_population(g.n, 20, 200, seed=6)
    print("n=2000, 200 individuals, hops = n", flush=True)
    pc, mcn = graph.sixdst(genes, g.n)
    F, M = graph.eval(genes, want_mcn=True)
    assert np.array_equal(pc, F) and np.array_equal(mcn, M)
    for i in range(0, 200, 40):
        assert (int(pc[i]), int(mcn[i])) == O.pc(g, genes[i])
    # device pointers, the paper's six hops: pairs within six hops never exceed PC
    d = torch.from_numpy(genes).cuda()
    pc6, mcn6 = gp.gapa_sixdst_eval(graph.handle, d, 6)
    assert bool((pc6.cpu() <= torch.from_numpy(F)).all()) and bool((mcn6.cpu() <= torch.from_numpy(M)).all())


def test_errors(gp):
    g = inputs.barabasi_albert(100, 2, seed=7)
    graph = gp.Graph.from_csr(g)
    genes = np.array([[1, 2, 3]], dtype=np.int32)
    with pytest.raises(gp.GapaError) as e:
        graph.sixdst(genes, 0)
    assert e.value.code == gp.GAPA_E_INVALID_ARG
    with pytest.raises(gp.GapaError) as e:
        graph.sixdst(np.array([[1, 100]], dtype=np.int32), 6)
    assert e.value.code == gp.GAPA_E_BAD_GENE
    big = gp.Graph.from_csr(inputs.erdos_renyi(9000, 2.0, seed=8), trust=True)
    with pytest.raises(gp.GapaError) as e:
        big.sixdst(genes, 6)
    assert e.value.code == gp.GAPA_E_INVALID_ARG
    # everything removed: no pairs, no surviving row
    pc, mcn = graph.sixdst(np.arange(100, dtype=np.int32)[None, :], 6)
    assert int(pc[0]) == 0 and int(mcn[0]) == 0


def test_tiny_graphs_empty_rows_and_huge_hop_counts(gp):
    class G:  # CSR of a path on n nodes
        def __init__(self, n):
            self.n = n
            adj = [[u for u in (v - 1, v + 1) if 0 <= u < n] for v in range(n)]
            self.row_ptr = np.array([0] + list(np.cumsum([len(a) for a in adj])), dtype=np.int32)
            self.col_idx = np.array([u for a in adj for u in a], dtype=np.int32)
            self.nnz = int(self.row_ptr[-1])
    for n in (1, 2, 3, 130):
        g = G(n)
        graph = gp.Graph(g.n, g.row_ptr, g.col_idx)
        empty = np.zeros((3, 0), dtype=np.int32)
        for hops in (1, 6, 10 ** 9):
            pc, mcn = graph.sixdst(empty, hops)
            ref = O.sixdst(g, [], min(hops, n))
            assert all((int(pc[i]), int(mcn[i])) == ref for i in range(3)), (n, hops)
        if n > 1:
            pc, mcn = graph.sixdst(np.array([[n // 2]], dtype=np.int32), 10 ** 9)
            assert (int(pc[0]), int(mcn[0])) == O.pc(g, [n // 2])
