"""The seeded synthetic inputs are reproducible: every graph the tests and the
benchmark use hashes to the value stored by tests/golden/make_golden.py."""
import json
import os

import numpy as np

from paper_2412_20980_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def manifest():
    with open(os.path.join(HERE, "golden", "graphs_manifest.json")) as f:
        return json.load(f)


def test_named_graph_hashes(ba200, ba10k, cl200k):
    m = manifest()
    for name, g in (("ba200", ba200), ("ba10k", ba10k), ("chung_lu_200k", cl200k)):
        assert g.sha256() == m[name]["sha256"], name
    assert ba200.m == 591 and ba10k.m == 29_991
    assert cl200k.n == 200_000 and 990_000 < cl200k.m < 1_000_000


def test_batched_instance_hashes_sample():
    m = manifest()
    sizes = inputs.batched_instance_sizes()
    assert sizes == m["batched_sizes"]
    assert all(1000 <= s <= 50_000 for s in sizes)
    for b in (0, 1, 5, 62, 63):
        n = sizes[b]
        g = inputs.barabasi_albert(n, 3, seed=1000 + b) if b % 2 == 0 else inputs.erdos_renyi(n, 8.0, seed=1000 + b)
        assert g.sha256() == m["batched"][b]["sha256"]


def test_csr_is_symmetric_simple_sorted(ba10k):
    g = ba10k
    rp, ci = g.row_ptr.astype(np.int64), g.col_idx.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == ci.shape[0] and np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(src != ci)
    for v in range(0, g.n, 97):
        nb = ci[rp[v]:rp[v + 1]]
        assert np.all(np.diff(nb) > 0)
    fwd = set(zip(src.tolist(), ci.tolist()))
    assert all((b, a) in fwd for a, b in list(fwd)[:5000])


def test_random_population_rows():
    pop = inputs.random_population(100, 10, 20, seed=3)
    assert pop.shape == (20, 10) and pop.dtype == np.int32
    assert np.all(np.diff(pop, axis=1) > 0)
