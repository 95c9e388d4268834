"""The allocation-free batched fitness (gapa_eval_population_noalloc) through
the C ABI: the same fitness and MCN as gapa_eval_population on the same
device genes, on two calls in a row (the second smaller, on another graph,
after the first left its contents in the shared scratch), and the oracle on a
sample.  Errors: host pointers, a graph too large for the scratch, a bad
gene."""
import ctypes as C

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


def both(gp, graph, genes, flags):
    import torch
    d = torch.from_numpy(genes).cuda()
    P = genes.shape[0]
    f_ref = torch.empty(P, dtype=torch.int64, device="cuda")
    m_ref = torch.zeros(P, dtype=torch.int32, device="cuda")
    gp.gapa_eval_population(graph.handle, d, fitness=f_ref, mcn=m_ref, flags=flags | gp.GAPA_WANT_MCN)
    f = torch.full((P,), -1, dtype=torch.int64, device="cuda")
    m = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    gp.gapa_eval_population_noalloc(graph.handle, d, fitness=f, mcn=m, flags=flags | gp.GAPA_WANT_MCN)
    torch.cuda.synchronize()
    return f.cpu().numpy(), m.cpu().numpy(), f_ref.cpu().numpy(), m_ref.cpu().numpy()


def test_noalloc_matches_eval_population_on_two_calls(gp, cl200k):
    # call 1: the 200k-node graph, 300 hub-biased rows (chunks of 32 at this
    # size: ten passes, the last one ragged)
    g1 = gp.Graph.from_csr(cl200k, trust=True)
    genes1 = inputs.hub_biased_population(cl200k, 2000, 300, seed=5, hub_frac=0.8)
    print("noalloc call 1: n=200000, P=300, k=2000", flush=True)
    f, m, f_ref, m_ref = both(gp, g1, genes1, 0)
    assert np.array_equal(f, f_ref) and np.array_equal(m, m_ref)
    for i in (0, 151, 299):
        assert (int(f[i]), int(m[i])) == O.pc(cl200k, genes1[i])
    # call 2: smaller, another graph, the component-count measure
    ba = inputs.barabasi_albert(3000, 2, seed=6)
    g2 = gp.Graph.from_csr(ba)
    genes2 = inputs.random_population(ba.n, 30, 70, seed=7)
    print("noalloc call 2: n=3000, P=70, k=30", flush=True)
    f, m, f_ref, m_ref = both(gp, g2, genes2, gp.GAPA_TRUST_INPUT | gp.GAPA_MAXIMISE_COMPONENTS)
    assert np.array_equal(f, f_ref) and np.array_equal(m, m_ref)
    for i in (0, 69):
        nc, alive = O.components(ba, genes2[i])
        assert int(f[i]) == alive - nc
    # and the PC measure again on the same graph after it
    f, m, f_ref, m_ref = both(gp, g2, genes2[:5], 0)
    assert np.array_equal(f, f_ref) and np.array_equal(m, m_ref)


def test_noalloc_errors(gp):
    import torch
    from paper_2412_20980_amd import gapa
    ba = inputs.barabasi_albert(500, 2, seed=8)
    graph = gp.Graph.from_csr(ba)
    genes = torch.from_numpy(inputs.random_population(ba.n, 10, 4, seed=9)).cuda()
    fit = torch.empty(4, dtype=torch.int64, device="cuda")
    L = gapa.lib()
    # host pointers are refused
    h = np.zeros((4, 10), dtype=np.int32)
    hf = np.zeros(4, dtype=np.int64)
    assert L.gapa_eval_population_noalloc(graph.handle, h.ctypes.data, 4, 10, hf.ctypes.data, None, 0, None) == \
        gapa.GAPA_E_INVALID_ARG
    # a gene out of range is reported (checked on the device)
    bad = genes.clone()
    bad[2, 3] = ba.n
    with pytest.raises(gp.GapaError) as e:
        gp.gapa_eval_population_noalloc(graph.handle, bad, fitness=fit)
    assert e.value.code == gp.GAPA_E_BAD_GENE
    # a path of 400k nodes needs more than the fixed scratch at 32 rows a pass
    n = 400_000
    deg = np.full(n, 2, dtype=np.int64)
    deg[0] = deg[-1] = 1
    row_ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    col = np.empty(row_ptr[-1], dtype=np.int32)
    col[row_ptr[1:n]] = np.arange(0, n - 1)      # node v >= 1: left neighbour v - 1 first
    col[row_ptr[1:n] - 1] = np.arange(1, n)      # node v <= n - 2: right neighbour v + 1 last
    big = gp.Graph(n, row_ptr, col, trust=True)
    gbig = torch.zeros((2, 3), dtype=torch.int32, device="cuda")
    fbig = torch.empty(2, dtype=torch.int64, device="cuda")
    with pytest.raises(gp.GapaError) as e:
        gp.gapa_eval_population_noalloc(big.handle, gbig, fitness=fbig, flags=gp.GAPA_TRUST_INPUT)
    assert e.value.code == gp.GAPA_E_INVALID_ARG and "scratch" in str(e.value)
    # the scratch is still usable afterwards
    f = gp.gapa_eval_population_noalloc(graph.handle, genes, fitness=fit)
    assert np.array_equal(f.cpu().numpy(), O.eval_population(ba, genes.cpu().numpy()))
