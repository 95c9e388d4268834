"""GPU parity of the component-count objective against the CPU oracle,
through the C ABI.

With GAPA_MAXIMISE_COMPONENTS the fitness of a removal set S is
|V minus S| - NC(G - S) (the size of a spanning forest of G - S); the pass
sums |C| - 1 over the same components it uses for PC.  Every value must equal
the oracle's plain BFS count exactly, for single passes, several chunks on
concurrent lanes, the union-find algorithm, device pointers, the degenerate
cases, a sample of the 200k-node workload, whole GA trajectories and a batch.
"""
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


def expected(g, pop):
    out = np.zeros(len(pop), dtype=np.int64)
    for i, row in enumerate(pop):
        nc, alive = O.components(g, row)
        out[i] = alive - nc
    return out


def ragged_population(n, P, seed, kmax):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, kmax + 1))
    return inputs.random_population(n, k, P, seed=seed)


@pytest.mark.parametrize("unionfind", [False, True])
@pytest.mark.parametrize("P", [1, 37, 1024, 1500, 2500])
def test_eval_matches_oracle(gp, unionfind, P):
    # ER at mean degree 1.5 leaves many isolated nodes and small trees; BA(2)
    # one large component; Chung-Lu hubs
    graphs = [inputs.erdos_renyi(3000, 1.5, seed=41), inputs.barabasi_albert(2000, 2, seed=42),
              inputs.chung_lu(4000, 2.5, 4.0, 8000, seed=43)]
    for j, g in enumerate(graphs):
        pop = ragged_population(g.n, P, seed=100 * j + P, kmax=g.n // 8)
        graph = gp.Graph.from_csr(g, unionfind=unionfind)
        got, mcn = graph.eval(pop, want_mcn=True, objective="components")
        assert np.array_equal(got, expected(g, pop)), (j, P)
        # the largest component is unchanged by the objective
        assert np.array_equal(mcn, O.eval_population(g, pop, want_mcn=True)[1]), (j, P)
        # and PC is still what the default objective returns
        assert np.array_equal(graph.eval(pop), O.eval_population(g, pop)), (j, P)


def test_device_pointers(gp):
    import torch
    g = inputs.erdos_renyi(2500, 2.0, seed=44)
    pop = inputs.random_population(g.n, 60, 700, seed=45)
    graph = gp.Graph.from_csr(g)
    d = torch.from_numpy(pop).cuda()
    F = torch.empty(pop.shape[0], dtype=torch.int64, device="cuda")
    gp.gapa_eval_population(graph.handle, d, fitness=F, flags=gp.GAPA_MAXIMISE_COMPONENTS)
    torch.cuda.synchronize()
    assert np.array_equal(F.cpu().numpy(), expected(g, pop))


def test_degenerate_cases(gp):
    # no genes: |V| - NC(G)
    g = inputs.erdos_renyi(1200, 1.2, seed=46)
    empty = np.zeros((5, 0), dtype=np.int32)
    got = gp.Graph.from_csr(g).eval(empty, objective="components")
    nc, alive = O.components(g, [])
    assert np.all(got == alive - nc)
    # every node of a path removed but the ends; a star without its centre;
    # an edgeless graph; a single node; repeated genes
    path = inputs.csr_from_edges(300, np.arange(299), np.arange(1, 300))
    star = inputs.csr_from_edges(300, np.zeros(299, dtype=int), np.arange(1, 300))
    edgeless = inputs.csr_from_edges(50, np.zeros(0, int), np.zeros(0, int))
    one = inputs.csr_from_edges(1, np.zeros(0, int), np.zeros(0, int))
    cases = [(path, np.arange(1, 299, dtype=np.int32)[None, :]),
             (star, np.array([[0, 0, 0]], dtype=np.int32)),
             (star, np.array([[5, 9, 9]], dtype=np.int32)),
             (edgeless, np.array([[1, 2, 3]], dtype=np.int32)),
             (one, np.zeros((3, 0), dtype=np.int32)),
             (one, np.zeros((2, 1), dtype=np.int32))]
    for unionfind in (False, True):
        for cg, pop in cases:
            got = gp.Graph.from_csr(cg, unionfind=unionfind).eval(pop, objective="components")
            assert np.array_equal(got, expected(cg, pop)), (cg.n, pop[:, :4], unionfind)
    # forest sizes of the two closed forms: the path's ends are apart (0),
    # a star without its centre has no edge left (0), with two leaves removed
    # it is one tree of 298 nodes (297)
    assert gp.Graph.from_csr(path).eval(np.arange(1, 299, dtype=np.int32)[None, :], objective="components")[0] == 0
    assert gp.Graph.from_csr(star).eval(np.array([[0]], dtype=np.int32), objective="components")[0] == 0
    assert gp.Graph.from_csr(star).eval(np.array([[5, 9]], dtype=np.int32), objective="components")[0] == 297


def test_full_size_sample(gp, cl200k):
    """The 200k-node workload at P = 1024 in the benchmark's launch shape; a
    sample of rows against the oracle, all rows against the tree identity's
    bound (0 <= fitness <= survivors - 1)."""
    pop = np.concatenate([inputs.hub_biased_population(cl200k, 2000, 512, seed=47, hub_frac=1.0),
                          inputs.random_population(cl200k.n, 2000, 512, seed=48)])
    got = gp.Graph.from_csr(cl200k, trust=True).eval(pop, objective="components")
    idx = np.arange(0, 1024, 127)
    assert np.array_equal(got[idx], expected(cl200k, pop[idx]))
    assert np.all(got >= 0) and np.all(got <= cl200k.n - 2000 - 1)


@pytest.mark.parametrize("replay", [False, True])
def test_ga_trajectory_matches_oracle(gp, replay):
    g = inputs.erdos_renyi(1500, 2.0, seed=49)
    graph = gp.Graph.from_csr(g)
    ga = gp.GA(graph, 30, 40, 9, 0.7, 0.1, 2, 60, replay=replay, objective="components")
    oga = O.OracleGA(g, 30, 40, 9, 0.7, 0.1, 2, 60, objective="components")
    for gen in range(6):
        pop, F = ga.population()
        assert np.array_equal(F, oga.F) and np.array_equal(pop, oga.pop), gen
        ga.step(1)
        oga.step()
    csrs = [inputs.barabasi_albert(400, 2, seed=50), inputs.erdos_renyi(900, 1.8, seed=51)]
    params = [dict(k=8, pop=16, seed=1, objective="components"),
              dict(k=20, pop=32, seed=2, offspring=48, objective="components")]
    bt = gp.Batch([gp.Graph.from_csr(c) for c in csrs], params, replay=replay)
    ogas = [O.OracleGA(c, p["k"], p["pop"], p["seed"], 0.7, 0.05, 2, p.get("offspring", 0), objective="components")
            for c, p in zip(csrs, params)]
    for _ in range(5):
        bt.step(1)
        for o in ogas:
            o.step()
    for b, o in enumerate(ogas):
        pop, F = bt.population(b)
        assert np.array_equal(F, o.F) and np.array_equal(pop, o.pop), b


def test_rejected_combinations(gp):
    g = inputs.erdos_renyi(500, 2.0, seed=52)
    graph = gp.Graph.from_csr(g)
    with pytest.raises(gp.GapaError):
        gp.gapa_ga_create(graph.handle, 10, 16, 1, flags=gp.GAPA_MINIMISE_MCN | gp.GAPA_MAXIMISE_COMPONENTS)
    with pytest.raises(gp.GapaError):
        ga = gp.GA(graph, 10, 16, 1, offspring=32, objective="components")
        ga.attach_surrogate(screen=8, batch=16, buffer=128)
    with pytest.raises(ValueError):
        graph.eval(np.zeros((1, 1), dtype=np.int32), objective="mcn")
