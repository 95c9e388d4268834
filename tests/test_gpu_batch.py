"""Batched GAs and HIP-graph replay, through the C ABI.

A batch advances many independent GA instances (each with its own graph,
budget, population, offspring count, tournament size, rates and seed) with
shared launches: one operator launch, one bit-parallel fitness pass over the
disjoint union of the instance graphs, one elitism launch per generation.
Every instance must follow exactly the oracle GA it would follow alone:
population rows and int64 fitness, in order, at every generation.  Replay
records one generation as a HIP graph and replays it; the trajectories must
not change (each replay is checked against the oracle, with host
synchronisation and eager work between replays)."""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import cnd_oracle as O
from paper_2412_20980_amd import inputs

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2412_20980_amd import gapa
    return gapa


def state_hash(pop, F):
    h = hashlib.sha256()
    h.update(pop.astype("<i4").tobytes())
    h.update(F.astype("<i8").tobytes())
    return h.hexdigest()[:32]


def oracle_for(g, p):
    return O.OracleGA(g, p["k"], p["pop"], p["seed"], p.get("pc", 0.7), p.get("pm", 0.05), p.get("tournament", 2),
                      p.get("offspring", 0))


def lockstep_batch(gp, csrs, params, gens, replay, graphs=None):
    print(f"batch of {len(csrs)}: n={[g.n for g in csrs]} replay={replay} gens={gens}", flush=True)
    graphs = graphs or [gp.Graph.from_csr(g) for g in csrs]
    bt = gp.Batch(graphs, params, replay=replay)
    ogas = [oracle_for(g, p) for g, p in zip(csrs, params)]
    for gen in range(gens + 1):
        for b, oga in enumerate(ogas):
            pop, F = bt.population(b)
            assert np.array_equal(F, oga.F), f"instance {b}: fitness differs at generation {gen}"
            assert np.array_equal(pop, oga.pop), f"instance {b}: population differs at generation {gen}"
        if gen < gens:
            bt.step(1)
            for oga in ogas:
                oga.step()
    for b, oga in enumerate(ogas):
        genes, f, gcount = bt.best(b)
        assert gcount == gens and f == oga.F[0] and np.array_equal(genes, oga.pop[0])
    return bt


def uneven_instances():
    csrs = [inputs.erdos_renyi(60, 3.0, seed=11), inputs.barabasi_albert(300, 2, seed=12),
            inputs.erdos_renyi(1000, 4.0, seed=13), inputs.barabasi_albert(2500, 3, seed=14),
            inputs.erdos_renyi(90, 2.0, seed=15), inputs.barabasi_albert(700, 1, seed=16)]
    params = [dict(k=5, pop=8, seed=1, pc=0.5, pm=0.3),
              dict(k=30, pop=32, seed=2, tournament=3, offspring=7),
              dict(k=10, pop=100, seed=3, pc=0.9, pm=0.2, offspring=128),
              dict(k=25, pop=128, seed=(1 << 40) + 4),
              dict(k=40, pop=5, seed=5, tournament=5, pc=1.0, pm=1.0, offspring=60),
              dict(k=70, pop=64, seed=6, pc=0.6, pm=0.1, offspring=33)]
    return csrs, params


@pytest.mark.parametrize("replay", [False, True])
def test_uneven_batch_matches_oracle_per_instance(gp, replay):
    csrs, params = uneven_instances()
    lockstep_batch(gp, csrs, params, 6, replay)


def test_wide_slots_and_repeated_graph(gp):
    """An instance with 600 individuals (1024 slots per instance), the same
    graph handle used by several instances with different seeds."""
    g1 = inputs.barabasi_albert(400, 2, seed=21)
    g2 = inputs.erdos_renyi(1500, 3.0, seed=22)
    graphs1 = gp.Graph.from_csr(g1)
    graphs2 = gp.Graph.from_csr(g2)
    csrs = [g1, g2, g1, g1]
    params = [dict(k=12, pop=600, seed=31, offspring=300), dict(k=40, pop=20, seed=32),
              dict(k=12, pop=20, seed=33, offspring=1000), dict(k=3, pop=1, seed=34)]
    lockstep_batch(gp, csrs, params, 4, True, graphs=[graphs1, graphs2, graphs1, graphs1])


def test_single_instance_batch_equals_ga(gp, ba200):
    W = inputs.workload("ba200_k10_p32")
    graph = gp.Graph.from_csr(ba200)
    p = dict(k=W.k, pop=W.pop, seed=W.seed, pc=W.pc, pm=W.pm, tournament=W.tournament)
    bt = lockstep_batch(gp, [ba200], [p], 8, True, graphs=[graph])
    ga = gp.GA(graph, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament)
    ga.step(8)
    pop_b, F_b = bt.population(0)
    pop_g, F_g = ga.population()
    assert np.array_equal(pop_b, pop_g) and np.array_equal(F_b, F_g)


@pytest.mark.parametrize("lam", [0, 50, 2000])
def test_ga_replay_matches_oracle(gp, lam):
    """A single GA with graph replay (lambda > 1024: several fitness chunks
    inside the recorded generation)."""
    g = inputs.erdos_renyi(800, 3.0, seed=41)
    print(f"replay GA lambda={lam}", flush=True)
    graph = gp.Graph.from_csr(g)
    ga = gp.GA(graph, 40, 64, 42, 0.7, 0.1, 2, lam, replay=True)
    oga = O.OracleGA(g, 40, 64, 42, 0.7, 0.1, 2, lam)
    for gen in range(7):
        pop, F = ga.population()
        assert np.array_equal(F, oga.F) and np.array_equal(pop, oga.pop), f"generation {gen}"
        # eager work on the device between replays
        graph.eval(pop[:3])
        ga.step(1)
        oga.step()


def test_replay_on_side_stream_and_timing_fallback(gp, ba10k):
    import torch
    W = inputs.workload("ba10k_k100_p256")
    graph = gp.Graph.from_csr(ba10k)
    s = torch.cuda.Stream()
    ga = gp.GA(graph, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament, replay=True, stream=s)
    ga.step(3, stream=s)
    ga.set_timing(1)  # timing runs generations eagerly
    ga.step(2, stream=s)
    times = ga.kernel_times()
    assert times["ga_offspring"][0] == 2 and times["elitism"][0] == 2
    ga.set_timing(0)
    ga.step(5, stream=s)
    oga = O.OracleGA(ba10k, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament)
    for _ in range(10):
        oga.step()
    pop, F = ga.population()
    assert np.array_equal(F, oga.F) and np.array_equal(pop, oga.pop)


def test_batch_timing_and_errors(gp):
    csrs, params = uneven_instances()
    graphs = [gp.Graph.from_csr(g) for g in csrs]
    bt = gp.Batch(graphs, params, replay=False)
    bt.set_timing(1)
    bt.step(2)
    t = bt.kernel_times()
    assert t["fitness_pass"][0] == 2 and t["ga_offspring"][0] == 2
    with pytest.raises(gp.GapaError) as e:
        gp.gapa_batch_best(bt.handle, len(csrs), 1)
    assert e.value.code == gp.GAPA_E_INVALID_ARG
    bad = [dict(p) for p in params]
    bad[2]["pop"] = 1025
    with pytest.raises(gp.GapaError) as e:
        gp.Batch(graphs, bad)
    assert e.value.code == gp.GAPA_E_INVALID_ARG
    bad = [dict(p) for p in params]
    bad[1]["k"] = csrs[1].n  # k > n / 2
    with pytest.raises(gp.GapaError) as e:
        gp.Batch(graphs, bad)
    assert e.value.code == gp.GAPA_E_INVALID_ARG


def test_batched_instances_match_golden(gp):
    """The 64-instance workload (log-uniform sizes in [1000, 50000], BA and
    ER graphs, k = n / 100, P = 128, 200 generations): every instance's
    per-generation state hash against the oracle's stored trajectory."""
    with open(os.path.join(HERE, "golden", "trajectories.json")) as f:
        traj = json.load(f)
    if "batched" not in traj:
        pytest.skip("no stored batched trajectories")
    ws = inputs.batched_instances()
    ref = traj["batched"]
    assert len(ref) == len(ws)
    graphs = []
    for w, r in zip(ws, ref):
        assert w.graph.sha256() == r["graph_sha256"]
        graphs.append(gp.Graph.from_csr(w.graph, trust=True))
    params = [dict(k=w.k, pop=w.pop, seed=w.seed, pc=w.pc, pm=w.pm, tournament=w.tournament) for w in ws]
    gens = ref[0]["generations"]
    print(f"batched golden: {len(ws)} instances, {gens} generations", flush=True)
    bt = gp.Batch(graphs, params, replay=True)
    for gen in range(gens + 1):
        for b, r in enumerate(ref):
            pop, F = bt.population(b)
            assert state_hash(pop, F) == r["hash"][gen], f"instance {b} differs at generation {gen}"
        if gen < gens:
            bt.step(1)
    for b, r in enumerate(ref):
        _, f, _ = bt.best(b)
        assert f == r["best"][gens]


@pytest.fixture(scope="module")
def cl200k_small_pop():
    g = inputs.chung_lu_200k()
    genes = inputs.hub_biased_population(g, 2000, 200, seed=3)
    return g, genes, O.eval_population(g, genes)


@pytest.mark.parametrize("tune", [dict(sweep_grid=16, band_scan=1, sweeps=0, band_blocks=16),
                                  dict(sweep_grid=65535, band_scan=1 << 20, sweeps=32, band_blocks=65535),
                                  dict(sweep_grid=300, band_scan=5, sweeps=1, band_blocks=77)])
def test_launch_shapes_never_change_results(gp, cl200k_small_pop, tune):
    g, genes, ref = cl200k_small_pop
    print(f"tuning {tune}", flush=True)
    graph = gp.Graph.from_csr(g, trust=True)
    graph.set_tuning(**tune)
    assert graph.get_tuning() == tune
    assert np.array_equal(graph.eval(genes), ref)


def test_autotuned_batch_and_retuned_replay_keep_trajectories(gp):
    csrs, params = uneven_instances()
    graphs = [gp.Graph.from_csr(g) for g in csrs]
    bt = gp.Batch(graphs, params, replay=True)
    ogas = [oracle_for(g, p) for g, p in zip(csrs, params)]
    for gen in range(1, 7):
        bt.step(1)
        for o in ogas:
            o.step()
        if gen == 2:
            best = bt.autotune(reps=1)
            print(f"autotuned {best}", flush=True)
        for b, o in enumerate(ogas):
            pop, F = bt.population(b)
            assert np.array_equal(F, o.F) and np.array_equal(pop, o.pop), (b, gen)
    # a replayed single GA whose graph is retuned mid-run
    g = inputs.erdos_renyi(900, 3.0, seed=51)
    graph = gp.Graph.from_csr(g)
    ga = gp.GA(graph, 30, 48, 5, 0.7, 0.1, 2, 100, replay=True)
    oga = O.OracleGA(g, 30, 48, 5, 0.7, 0.1, 2, 100)
    for gen in range(1, 7):
        if gen == 4:
            graph.set_tuning(sweep_grid=128, band_scan=8, sweeps=1, band_blocks=64)
        ga.step(1)
        oga.step()
        pop, F = ga.population()
        assert np.array_equal(F, oga.F) and np.array_equal(pop, oga.pop), gen


def test_multi_generation_recordings_match_oracle(gp):
    """Several generations recorded as one HIP graph: a step call of that
    many generations from the same buffer parity is one launch, and the
    trajectory stays the oracle's (an odd count ends on the other parity,
    where the next call falls back to one-generation replays)."""
    g = inputs.erdos_renyi(800, 3.0, seed=43)
    graph = gp.Graph.from_csr(g)
    ga = gp.GA(graph, 40, 64, 43, 0.7, 0.1, 2, 1500, replay=True)
    oga = O.OracleGA(g, 40, 64, 43, 0.7, 0.1, 2, 1500)
    with pytest.raises(gp.GapaError) as e:
        ga.record(4)  # nothing run yet: buffers not sized
    assert e.value.code == gp.GAPA_E_STATE
    ga.step(1)
    oga.step()
    with pytest.raises(gp.GapaError) as e:
        ga.record(0)
    assert e.value.code == gp.GAPA_E_INVALID_ARG
    ga.record(4)
    ga.record(5)
    for n in (4, 4, 5, 5, 3):
        print(f"step({n})", flush=True)
        ga.step(n)
        for _ in range(n):
            oga.step()
        pop, F = ga.population()
        assert np.array_equal(F, oga.F) and np.array_equal(pop, oga.pop), n
        graph.eval(pop[:2])  # eager work between launches
    csrs, params = uneven_instances()
    bt = gp.Batch([gp.Graph.from_csr(c) for c in csrs], params, replay=True)
    ogas = [oracle_for(c, p) for c, p in zip(csrs, params)]
    bt.step(1)
    bt.record(6)
    for _ in range(2):
        bt.step(6)
    for o in ogas:
        for _ in range(13):
            o.step()
    for b, o in enumerate(ogas):
        pop, F = bt.population(b)
        assert np.array_equal(F, o.F) and np.array_equal(pop, o.pop), b
