"""Learned screening surrogate on the GPU, through the C ABI, against the
surrogate oracle.

Integer work is exact: initial weights (Philox, float32) bit for bit;
screening decisions equal the oracle's selection applied to the device's own
float32 predictions; the GA trajectory equals the oracle's replay given the
device's screened indices, generation by generation, up to the full-size
workload (200k nodes, 4096 children screened to 512).  The judge's
statistics equal the oracle's on the device's predictions and label
standardisation.  Floating-point work is compared at tolerances derived from
the network's precision (bfloat16 weights, activations and activation
gradients; float32 accumulation, pre-activations, loss and optimiser): the
forward pass and, element by element, the gradients against the oracle
computing with the same bfloat16 roundings in float64, one Adam step against
the oracle's formula on the device's gradients, replayed training against
Adam's bound on how far two runs can drift.  A last test shows what the
trained network gains over random screening at the same exact-evaluation
budget."""
import numpy as np
import pytest

from oracle import cnd_oracle as O
from oracle import surrogate_oracle as S
from paper_2412_20980_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2412_20980_amd import gapa
    return gapa


def make_ga(gp, g, k=20, pop=32, seed=7, lam=128, **surr):
    graph = gp.Graph.from_csr(g)
    ga = gp.GA(graph, k, pop, seed, 0.7, 0.05, 2, lam)
    opts = dict(screen=32, batch=64, train_steps=2, warmup_gens=2, buffer=4096, fallback_gens=3)
    opts.update(surr)
    ga.attach_surrogate(**opts)
    return graph, ga


def weights(ga, n):
    return {name: ga.surrogate_tensor(name, n=n).astype(np.float64) for name in S.TENSORS}


def test_initial_weights_bit_exact(gp):
    g = inputs.barabasi_albert(700, 3, seed=1)
    _, ga = make_ga(gp, g, seed=(1 << 33) + 5)
    ref = S.init_params((1 << 33) + 5, g.n)
    got = weights(ga, g.n)
    for name in S.TENSORS:
        assert np.array_equal(got[name], ref[name]), name


def random_weights(rng, n):
    # float32 values with the scale of a trained model, biases non-zero
    return {"E": rng.normal(0, 0.05, (n, 64)), "W1": rng.normal(0, 0.2, (256, 64)), "b1": rng.normal(0, 0.1, 256),
            "W2": rng.normal(0, 0.08, (256, 256)), "b2": rng.normal(0, 0.1, 256), "w3": rng.normal(0, 0.1, 256),
            "b3": rng.normal(0, 0.5, 1)}


def set_weights(ga, p):
    for name in S.TENSORS:
        ga.set_surrogate_tensor(name, p[name])
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


@pytest.mark.parametrize("P", [1, 63, 200])
def test_forward_matches_oracle(gp, P):
    import torch
    g = inputs.barabasi_albert(900, 3, seed=2)
    _, ga = make_ga(gp, g)
    p = set_weights(ga, random_weights(np.random.default_rng(P), g.n))
    sets = inputs.random_population(g.n, 20, P, seed=P)
    y = ga.predict(torch.from_numpy(sets).cuda()).cpu().numpy().astype(np.float64)
    ref_b = S.forward(p, sets, bf16_ops=True)["yhat"]
    ref = S.forward(p, sets)["yhat"]
    scale = 1.0 + np.max(np.abs(ref_b))
    assert np.max(np.abs(y - ref_b)) <= 2e-3 * scale
    assert np.max(np.abs(y - ref)) <= 3e-2 * scale


def test_gradients_match_oracle(gp):
    """Element by element.  A bfloat16 operand that rounds differently on the
    two sides (their float32 and float64 sums differ in the last bits and
    straddle a rounding boundary) moves an entry by at most one bfloat16 step
    (2^-8 relative) of the terms it enters, and float32 accumulation adds
    about 2^-24 per term: every entry agrees within 2^-6 of the tensor's
    largest entry, and nearly all within a bfloat16 step of their own size."""
    import torch
    g = inputs.barabasi_albert(900, 3, seed=3)
    _, ga = make_ga(gp, g, batch=64)
    p = set_weights(ga, random_weights(np.random.default_rng(5), g.n))
    sets = inputs.random_population(g.n, 20, 64, seed=9)
    target = np.random.default_rng(6).normal(size=64).astype(np.float32)
    ga.train_batch(torch.from_numpy(sets).cuda(), torch.from_numpy(target).cuda(), keep_grads=True)
    loss_ref, ref, _ = S.loss_and_grads(p, sets, target.astype(np.float64), bf16_ops=True)
    for name in S.TENSORS:
        got = ga.surrogate_tensor(name, grad=True, n=g.n).astype(np.float64)
        scale = np.max(np.abs(ref[name]))
        err = np.abs(got - ref[name])
        close = np.mean(err <= 2.0 ** -8 * np.abs(ref[name]) + 2.0 ** -12 * scale)
        print(f"{name}: max err / max |ref| = {err.max() / scale:.2e}, within a bf16 step: {close:.4f}", flush=True)
        assert err.max() <= 2.0 ** -6 * scale, name
        assert close >= 0.99, name
    # rows of E outside every set get no gradient
    used = np.zeros(g.n, bool)
    used[sets.ravel()] = True
    assert not ga.surrogate_tensor("E", grad=True, n=g.n)[~used].any()
    # the step's loss (the mean squared error of the same forward pass)
    loss = ga.surrogate_stats()["loss"]
    print(f"loss device {loss:.6f} oracle {loss_ref:.6f}", flush=True)
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref


def test_judge_statistics_match_oracle(gp):
    """The judge's Spearman correlation and mean relative error on explicit
    predictions and exact fitness (ties on both sides, more children than the
    judge looks at, a pool that permutes the predictions) equal the oracle's
    to rounding."""
    import torch
    rng = np.random.default_rng(3)
    for m, lam, use_pool in ((1, 1, False), (7, 20, True), (544, 4096, True), (1024, 1024, False),
                             (3000, 4096, True)):
        yhat = rng.normal(size=lam).astype(np.float32)
        yhat[rng.integers(0, lam, size=lam // 4)] = np.float32(0.5)
        F = rng.integers(0, 10 ** 10, size=m).astype(np.int64)
        F[: m // 3] = F[0]
        pool = rng.permutation(lam)[:m].astype(np.int32) if use_pool else np.arange(m, dtype=np.int32)
        mu, sd = 20.0, 1.5
        rho, rel = gp.gapa_surrogate_judge(torch.from_numpy(yhat).cuda(), torch.from_numpy(F).cuda(), mu, sd,
                                           pool=torch.from_numpy(pool).cuda() if use_pool else None)
        rho_ref, rel_ref = S.judge_stats(yhat[pool].astype(np.float64), F, mu, sd)
        assert abs(rho - rho_ref) <= 1e-9, (m, rho, rho_ref)
        assert abs(rel - rel_ref) <= 1e-9 * max(1.0, rel_ref), (m, rel, rel_ref)
    with pytest.raises(gp.GapaError) as e:
        gp.gapa_surrogate_judge(torch.zeros(4, device="cuda"), torch.zeros(4, dtype=torch.int64, device="cuda"),
                                0.0, 0.0)
    assert e.value.code == gp.GAPA_E_INVALID_ARG


def test_generation_training_moves_exactly_the_sampled_rows(gp):
    """A generation's training builds its batches' membership bits straight
    from the sampled rows (ascending): Adam is lazy on the embeddings, so the
    rows it moves are exactly the nodes of the batches the oracle samples for
    that generation, and every other row keeps its value bit for bit (also at
    sizes that are not multiples of the kernels' 256-node ranges)."""
    for n, k, batch in ((1500, 20, 64), (1031, 37, 32)):
        g = inputs.barabasi_albert(n, 1, seed=n)
        _, ga = make_ga(gp, g, k=k, batch=batch, buffer=1024)
        before = ga.surrogate_tensor("E", n=g.n).copy()
        ga.step(1)
        after = ga.surrogate_tensor("E", n=g.n)
        moved = np.any(after != before, axis=1)
        sga = S.SurrogateGA(g, k, 32, 7, 128, batch=batch, steps=2, warmup=2, buffer=1024, bf16_ops=True)
        sga.step()
        count = min(sga.appended, sga.cap)
        touched = np.zeros(g.n, bool)
        for t in range(2):
            touched[sga.buf_sets[S.sample_batch(7, 1, t, batch, count)].ravel()] = True
        print(f"n={n}: {touched.sum()} rows touched, {moved.sum()} moved", flush=True)
        assert np.array_equal(moved, touched)


def test_adam_step_matches_formula(gp):
    import torch
    g = inputs.barabasi_albert(600, 3, seed=4)
    _, ga = make_ga(gp, g, k=15, batch=32)
    p = set_weights(ga, random_weights(np.random.default_rng(8), g.n))
    sets = inputs.random_population(g.n, 15, 32, seed=3)
    target = np.linspace(-1, 1, 32).astype(np.float32)
    ga.train_batch(torch.from_numpy(sets).cuda(), torch.from_numpy(target).cuda(), keep_grads=True)
    grads = {name: ga.surrogate_tensor(name, grad=True, n=g.n).astype(np.float64) for name in S.TENSORS}
    q = {k: v.copy() for k, v in p.items()}
    S.Adam(q, lr=1e-3).step(q, grads, rows=S.batch_rows(sets))
    got = weights(ga, g.n)
    for name in S.TENSORS:
        assert np.max(np.abs(got[name] - q[name])) <= 2e-6, name


def run_replayed(gp, g, gens, **kw):
    """Device GA with a surrogate next to the oracle replaying its screening
    decisions; checks the screening, the judge's statistics and the state
    every generation."""
    lam, k, pop, seed = kw.pop("lam", 128), kw.pop("k", 20), kw.pop("pop", 32), kw.pop("seed", 7)
    _, ga = make_ga(gp, g, k=k, pop=pop, seed=seed, lam=lam, **kw)
    opts = dict(screen=32, batch=64, train_steps=2, warmup_gens=2, buffer=4096)
    opts.update({k2: v for k2, v in kw.items() if k2 in opts})
    sga = S.SurrogateGA(g, k, pop, seed, lam, batch=opts["batch"], steps=opts["train_steps"],
                        warmup=opts["warmup_gens"], buffer=opts["buffer"], bf16_ops=True)
    screened = 0
    losses = []
    for gen in range(1, gens + 1):
        ga.step(1)
        st = ga.surrogate_stats()
        evaluated = ga.last_pool()
        assert st["generation"] == gen and st["evaluated"] == len(evaluated)
        pool, extra = evaluated[:st["pooled"]], evaluated[st["pooled"]:]
        yhat = None
        if st["screened"]:
            screened += 1
            yhat = ga.last_predictions()
            assert len(yhat) == lam
            # the selection is exact given the device's float32 predictions
            assert np.array_equal(pool, S.screen(yhat.astype(np.float64), opts["screen"]))
            # the judge's unbiased extra sample
            assert len(extra) == min(32, lam - opts["screen"])
            assert np.array_equal(extra, S.judge_extra(seed, gen, lam, pool, len(extra)))
        else:
            assert np.array_equal(pool, np.arange(lam)) and len(extra) == 0
        kids, kf, _ = sga.step(pool, extra)
        pop_d, F_d = ga.population()
        assert np.array_equal(F_d, sga.ga.F), f"fitness differs at generation {gen}"
        assert np.array_equal(pop_d, sga.ga.pop), f"population differs at generation {gen}"
        if yhat is not None:
            # the predictions of generation g are in the label standardisation
            # of generation g - 2's training (none before it: mean 0, spread 1)
            mu_ref, sd_ref = sga.label_stats.get(gen - 2, (0.0, 1.0))
            mu, sd = st["label_mean"], st["label_spread"]
            assert abs(mu - mu_ref) <= 1e-12 * max(1.0, abs(mu_ref)) and abs(sd - sd_ref) <= 1e-9 * sd_ref, gen
            F_eval = np.concatenate([kf[pool], O.eval_population(g, kids[extra])]) if len(extra) else kf[pool]
            rho_ref, rel_ref = S.judge_stats(yhat[evaluated].astype(np.float64), F_eval, mu, sd)
            assert abs(st["spearman"] - rho_ref) <= 1e-9, (gen, st["spearman"], rho_ref)
            assert abs(st["rel_err"] - rel_ref) <= 1e-9 * max(1.0, rel_ref), (gen, st["rel_err"], rel_ref)
        if gen >= 3:
            # the loss of the last step of generation g - 2's training
            losses.append((st["loss"], sga.losses[(gen - 2) * opts["train_steps"] - 1]))
    for gen, (dev, ref) in enumerate(losses, start=3):
        print(f"generation {gen}: loss device {dev:.6f} oracle {ref:.6f}", flush=True)
    return ga, sga, screened, losses


def test_screened_trajectory_replays_exactly(gp):
    # a tree (BA with one edge per node): removals split it, so labels vary
    g = inputs.barabasi_albert(1500, 1, seed=5)
    ga, sga, screened, losses = run_replayed(gp, g, 8, fallback_gens=0)
    assert screened == 6
    st = ga.surrogate_stats()
    assert st["train_steps"] == 16
    # The device model and the oracle's float64 replay of its training stay
    # close.  Adam moves a coordinate by at most lr (1 - b1) / sqrt(1 - b2) per
    # step whatever its gradient (Kingma and Ba 2015, Sec. 2.1), so
    # coordinates whose gradient is near zero (its sign set by rounding) can
    # step apart on the two sides: after T steps no coordinate is further apart
    # than twice T such steps, the weight matrices as a whole stay within 2 %
    # and the predictions they make stay aligned.
    import torch
    got, ref = weights(ga, g.n), sga.params
    T, lr = 16, 1e-3
    bound = 2 * T * lr * (1 - 0.9) / np.sqrt(1 - 0.999)
    for name in S.TENSORS:
        d = np.abs(got[name] - ref[name])
        rel = np.linalg.norm(got[name] - ref[name]) / max(np.linalg.norm(ref[name]), 1e-30)
        print(f"{name}: max |diff| {d.max():.2e} (bound {bound:.2e}), relative norm {rel:.3e}", flush=True)
        assert d.max() <= bound, name
    for name in ("W1", "W2", "w3"):
        assert np.linalg.norm(got[name] - ref[name]) <= 2e-2 * np.linalg.norm(ref[name]), name
    sets = inputs.random_population(g.n, 20, 256, seed=11)
    y_dev = ga.predict(torch.from_numpy(sets).cuda()).cpu().numpy().astype(np.float64)
    y_ref = S.forward(ref, sets, bf16_ops=True)["yhat"]
    assert np.corrcoef(y_dev, y_ref)[0, 1] > 0.98
    assert np.linalg.norm(y_dev - y_ref) <= 0.1 * np.linalg.norm(y_ref - y_ref.mean()) + 1e-3 * len(sets)
    # training losses on the same batches: equal at the first step, within a
    # few percent as the weights drift apart
    for dev, r in losses:
        assert abs(dev - r) <= 0.05 * r + 1e-4


def test_full_size_screened_generations_replay_exactly(gp, cl200k):
    """The surrogate workload at its size: 200k nodes, k = 2000, population
    1024, 4096 children per generation, 512 screened for exact evaluation
    (plus the judge's 32), training batches of 1024.  Two full generations,
    then three screened ones: screening, the judge's sample and statistics,
    fitness and populations checked every generation."""
    W = inputs.workload("cl200k_k2000_p1024_screen4096")
    print("full-size surrogate replay: 2 full + 3 screened generations", flush=True)
    ga, sga, screened, _ = run_replayed(gp, cl200k, 5, k=W.k, pop=W.pop, lam=W.offspring, seed=W.seed,
                                        screen=W.exact_top, batch=1024, train_steps=2, warmup_gens=2,
                                        buffer=16384, fallback_gens=0)
    assert screened == 3
    assert ga.surrogate_stats()["evaluated"] == W.exact_top + 32


def test_fallback_to_full_generations(gp):
    """An unreachable correlation threshold forces full generations.  The
    decision for generation g comes from the judge of generation g - 2, and a
    generation launched before a forced one does not count: with one warm-up
    generation, generations 2, 3, 5 and 6 are screened and 4 and 7 are full."""
    g = inputs.erdos_renyi(1200, 4.0, seed=6)
    ga, _, screened, _ = run_replayed(gp, g, 7, min_rho=2.0, fallback_gens=1, warmup_gens=1)
    st = ga.surrogate_stats()
    assert screened == 4 and st["fallbacks"] == 2


def test_binding_rejects_rows_of_the_wrong_width(gp):
    import torch
    g = inputs.barabasi_albert(300, 2, seed=9)
    _, ga = make_ga(gp, g, k=15, batch=32)
    with pytest.raises(ValueError):
        ga.predict(torch.zeros((4, 14), dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        ga.train_batch(torch.zeros((32, 16), dtype=torch.int32, device="cuda"),
                       torch.zeros(32, dtype=torch.float32, device="cuda"))


def test_attach_rejects_bad_parameters(gp, ba200):
    graph = gp.Graph.from_csr(ba200)
    ga = gp.GA(graph, 10, 16, 1, offspring=64)
    for bad in (dict(screen=0), dict(screen=65), dict(batch=48), dict(batch=2048), dict(buffer=16), dict(lr=0.0)):
        opts = dict(screen=16, batch=32, buffer=256)
        opts.update(bad)
        with pytest.raises(gp.GapaError) as e:
            ga.attach_surrogate(**opts)
        assert e.value.code == gp.GAPA_E_INVALID_ARG, bad
    ga.step(1)
    with pytest.raises(gp.GapaError):
        ga.attach_surrogate(screen=16, batch=32, buffer=256)  # not at generation 0
    ga2 = gp.GA(graph, 10, 16, 1, offspring=64)
    with pytest.raises(gp.GapaError) as e:
        ga2.surrogate_stats()
    assert e.value.code == gp.GAPA_E_STATE


def best_after(gp, g, gens, seed, random_screen):
    graph = gp.Graph.from_csr(g, trust=True)
    ga = gp.GA(graph, 100, 128, seed, 0.7, 0.05, 2, 1024)
    ga.attach_surrogate(screen=128, batch=256, train_steps=4, warmup_gens=5, buffer=16384, fallback_gens=0,
                        random_screen=random_screen)
    ga.step(gens)
    rho = ga.surrogate_stats()["spearman"]
    return ga.best()[1], rho


def test_trained_screening_beats_random_screening(gp):
    """Same seeds, same operators, the same number of exact evaluations per
    generation (128 of 1024 children): screening by the trained network must
    reach a lower pairwise connectivity than screening at random, and its
    predictions must rank the evaluated children (positive correlation)."""
    g = inputs.chung_lu(20000, 2.5, 10.0, 100_000, seed=7)
    wins, rhos = 0, []
    for seed in (1, 2, 3):
        print(f"surrogate vs random, seed {seed}", flush=True)
        f_s, rho = best_after(gp, g, 40, seed, False)
        f_r, _ = best_after(gp, g, 40, seed, True)
        print(f"  best PC surrogate {f_s} random {f_r} rho {rho:.3f}", flush=True)
        wins += f_s < f_r
        rhos.append(rho)
    assert wins >= 2
    assert np.mean(rhos) > 0.3
