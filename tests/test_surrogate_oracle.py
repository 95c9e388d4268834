"""Pins of the surrogate oracle (CPU only).

The oracle's model, gradients, optimiser and screening are checked against
things other than themselves: bfloat16 rounding against torch's conversion,
the backward pass against central finite differences and float64 autograd,
Adam against its closed-form first step and torch.optim.Adam, the forward
pass in its linear regime against a closed form, screening and Spearman's
correlation against brute force and scipy."""
import math

import numpy as np
import pytest
import torch

from oracle import cnd_oracle as O
from oracle import surrogate_oracle as S
from paper_2412_20980_amd import inputs


def tiny_params(rng, n=7, D=3, H=5):
    return {"E": rng.normal(size=(n, D)), "W1": rng.normal(size=(H, D)), "b1": rng.normal(size=H) * 0.1,
            "W2": rng.normal(size=(H, H)), "b2": rng.normal(size=H) * 0.1, "w3": rng.normal(size=H),
            "b3": rng.normal(size=1)}


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, size=2000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8, -3.5]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert S.bf16(1.0 + 2.0 ** -8) == 1.0
    assert S.bf16(1.0 + 2.0 ** -7 + 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_init_values_and_ranges():
    seed, n, D, H = 11, 300, 64, 256
    p = S.init_params(seed, n, D, H)
    b = S.init_bounds(D, H)
    assert p["E"].shape == (n, D) and p["W1"].shape == (H, D) and p["W2"].shape == (H, H) and p["w3"].shape == (H,)
    for k in ("E", "W1", "W2", "w3"):
        assert np.all(np.abs(p[k]) < b[k])
        # float32 values
        assert np.array_equal(p[k], p[k].astype(np.float32).astype(np.float64))
    assert not p["b1"].any() and not p["b2"].any() and not p["b3"].any()
    # element (r, c) of tensor t comes from draw(seed, c, r, t, stream 5)
    for (t, name, r, c) in ((0, "E", 17, 5), (1, "W1", 200, 63), (2, "W2", 3, 255)):
        w = int(O.draw(seed, c, r, t, S.ST_SURR_INIT)[0])
        u = (w + 0.5) / 2 ** 32
        assert p[name][r, c] == np.float64(np.float32(b[name] * (2 * u - 1)))
    w = int(O.draw(seed, 7, 0, 3, S.ST_SURR_INIT)[0])
    assert p["w3"][7] == np.float64(np.float32(b["w3"] * (2 * ((w + 0.5) / 2 ** 32) - 1)))
    # uniform: mean and variance of the 19200 values of E
    e = p["E"].ravel()
    assert abs(e.mean()) < 4 * 0.05 / math.sqrt(3 * e.size)
    assert abs(e.var() - 0.05 ** 2 / 3) < 0.05 * 0.05 ** 2 / 3


def test_embedding_sum_brute_force():
    rng = np.random.default_rng(1)
    E = rng.normal(size=(20, 4))
    sets = rng.integers(0, 20, size=(6, 5))
    x = S.embed(E, sets)
    for i in range(6):
        acc = np.zeros(4)
        for v in sets[i]:
            acc += E[v]
        assert np.allclose(x[i], acc, rtol=0, atol=1e-12)


def test_forward_linear_regime_closed_form():
    """With every pre-activation positive the network is the affine map
    w3 (W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(2)
    p = {"E": rng.uniform(0.1, 1, size=(10, 3)), "W1": rng.uniform(0.1, 1, size=(4, 3)), "b1": np.full(4, 0.2),
         "W2": rng.uniform(0.1, 1, size=(4, 4)), "b2": np.full(4, 0.3), "w3": rng.normal(size=4), "b3": np.array([0.7])}
    sets = rng.integers(0, 10, size=(5, 3))
    x = S.embed(p["E"], sets)
    A = p["w3"] @ p["W2"] @ p["W1"]
    c = p["w3"] @ (p["W2"] @ p["b1"] + p["b2"]) + 0.7
    assert np.allclose(S.forward(p, sets)["yhat"], x @ A + c, rtol=1e-12)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(3)
    p = tiny_params(rng)
    sets = rng.integers(0, 7, size=(4, 3))
    target = rng.normal(size=4)
    _, g, _ = S.loss_and_grads(p, sets, target)
    h = 1e-6
    for k in S.TENSORS:
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k][i] += h
            lp = S.loss_and_grads(q, sets, target)[0]
            q[k][i] -= 2 * h
            lm = S.loss_and_grads(q, sets, target)[0]
            num = (lp - lm) / (2 * h)
            assert abs(num - g[k][i]) <= 1e-6 * max(1.0, abs(num)), (k, i, num, g[k][i])


def test_gradients_match_float64_autograd():
    rng = np.random.default_rng(4)
    p = tiny_params(rng, n=30, D=8, H=16)
    sets = rng.integers(0, 30, size=(12, 6))
    target = rng.normal(size=12)
    loss, g, _ = S.loss_and_grads(p, sets, target)
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    x = t["E"][torch.tensor(sets)].sum(dim=1)
    h1 = torch.relu(x @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    yhat = h2 @ t["w3"] + t["b3"]
    tl = torch.mean((yhat - torch.tensor(target)) ** 2)
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12
    for k in S.TENSORS:
        assert np.allclose(g[k], t[k].grad.numpy(), rtol=1e-10, atol=1e-12), k


def test_bf16_mode_stays_close_to_the_definition():
    g = inputs.barabasi_albert(500, 3, seed=5)
    p = S.init_params(3, g.n)
    sets = inputs.random_population(g.n, 20, 64, seed=6)
    a = S.forward(p, sets)["yhat"]
    b = S.forward(p, sets, bf16_ops=True)["yhat"]
    assert np.max(np.abs(a - b)) < 2e-2 * (1 + np.max(np.abs(a)))
    target = np.linspace(-1, 1, 64)
    _, ga, _ = S.loss_and_grads(p, sets, target)
    _, gb, _ = S.loss_and_grads(p, sets, target, bf16_ops=True)
    # bfloat16 operands (8-bit significands) move the first-layer gradients
    # by several percent (ReLU masks flip near zero, sums cancel); the device
    # is compared against the bf16-mode oracle, where the roundings agree
    for k in S.TENSORS:
        na, nb = np.linalg.norm(ga[k]), np.linalg.norm(gb[k])
        assert np.linalg.norm(ga[k] - gb[k]) <= 0.12 * na, k
        assert ga[k].ravel() @ gb[k].ravel() >= 0.99 * na * nb, k


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    p = tiny_params(rng)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    q = {k: v.copy() for k, v in p.items()}
    opt = S.Adam(q, lr=1e-3)
    opt.step(q, g)
    for k in p:
        assert np.allclose(q[k], p[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=0, atol=1e-15)


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    p = tiny_params(rng)
    q = {k: v.copy() for k, v in p.items()}
    opt = S.Adam(q, lr=1e-3)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    topt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        g = {k: rng.normal(size=v.shape) for k, v in p.items()}
        opt.step(q, g)
        for k, t in tp.items():
            t.grad = torch.tensor(g[k])
        topt.step()
    for k in p:
        assert np.allclose(q[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15), k


def test_lazy_adam_on_embeddings_matches_torch_sparse_adam():
    """Rows outside the batch keep weights and moments; the others follow
    torch.optim.SparseAdam (the lazy variant for sparse gradients)."""
    rng = np.random.default_rng(13)
    p = tiny_params(rng, n=12, D=3, H=4)
    q = {k: v.copy() for k, v in p.items()}
    opt = S.Adam(q, lr=1e-3)
    E = torch.tensor(p["E"], dtype=torch.float64, requires_grad=True)
    topt = torch.optim.SparseAdam([E], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    seen = set()
    for step in range(4):
        sets = rng.integers(0, 12, size=(3, 2))
        rows = S.batch_rows(sets)
        seen.update(rows.tolist())
        g = {k: rng.normal(size=v.shape) for k, v in p.items()}
        g["E"][np.setdiff1d(np.arange(12), rows)] = 0.0
        opt.step(q, g, rows=rows)
        E.grad = torch.sparse_coo_tensor(torch.tensor(rows)[None, :], torch.tensor(g["E"][rows]), (12, 3))
        topt.step()
    # SparseAdam adds eps to sqrt(v) before the bias correction (eps scaled
    # by sqrt(1 - b2^t)): ~1e-10 here; a wrong row set would differ by ~1e-3
    assert np.allclose(q["E"], E.detach().numpy(), rtol=0, atol=1e-8)
    never = np.setdiff1d(np.arange(12), sorted(seen))
    assert never.size > 0 and np.array_equal(q["E"][never], p["E"][never])
    assert np.all(opt.m["E"][never] == 0) and np.all(opt.v["E"][never] == 0)


def test_screen_brute_force_with_ties():
    rng = np.random.default_rng(9)
    yhat = rng.integers(0, 20, size=300).astype(np.float64)  # many ties
    got = S.screen(yhat, 50)
    ranked = sorted(range(300), key=lambda i: (yhat[i], i))[:50]
    assert np.array_equal(got, np.sort(ranked))


def test_spearman_matches_scipy():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(10)
    a = rng.integers(0, 30, size=200).astype(float)
    b = a + rng.normal(size=200) * 5
    assert abs(S.spearman(a, b) - spearmanr(a, b).correlation) < 1e-12
    assert abs(S.spearman(a, -a) + 1.0) < 1e-12


def test_labels_and_standardisation():
    F = np.array([0, 1, 10 ** 10])
    assert np.array_equal(S.label(F), np.log1p(F.astype(float)))
    mu, sd = S.standardise(np.array([1.0, 3.0]))
    assert mu == 2.0 and abs(sd - 1.0) < 1e-12
    # equal labels: the floor keeps the spread at 1e-6, targets stay zero
    assert S.standardise(np.array([5.0, 5.0])) == (5.0, 1e-6)


def test_batch_sampling_uses_stream_six():
    idx = S.sample_batch(5, 3, 2, 64, 1000)
    assert idx.min() >= 0 and idx.max() < 1000
    w = int(O.draw(5, 10, 2, 3, S.ST_SURR_SAMPLE)[0])
    assert idx[10] == (w * 1000) >> 32


def test_replayed_ga_without_screening_is_the_plain_ga():
    g = inputs.barabasi_albert(300, 2, seed=12)
    sga = S.SurrogateGA(g, 10, 16, 4, offspring=40, D=8, H=16, batch=32, steps=1, warmup=100, buffer=256)
    ga = O.OracleGA(g, 10, 16, 4, offspring=40)
    for _ in range(4):
        sga.step()
        ga.step()
        assert np.array_equal(sga.ga.pop, ga.pop) and np.array_equal(sga.ga.F, ga.F)
    assert sga.appended == 4 * 40 and len(sga.losses) == 4


def test_bf16_mode_is_the_mixed_precision_network():
    """The oracle's bfloat16 mode against torch autograd in float64 given only
    where the network keeps bfloat16 values: the weight copies (E, W1, W2, w3)
    and activations (x, h1, h2) are rounded in the forward pass (gradients
    pass to the float32 masters unchanged), the activation gradients (of z1,
    z2 and x) are rounded in the backward pass; sums, biases, pre-activations
    and the loss stay wide.  Autograd derives the chain rule itself."""
    rng = np.random.default_rng(14)
    n, B, k = 40, 16, 5
    p = {"E": rng.normal(0, 0.3, (n, 8)), "W1": rng.normal(0, 0.4, (16, 8)), "b1": rng.normal(0, 0.1, 16),
         "W2": rng.normal(0, 0.3, (16, 16)), "b2": rng.normal(0, 0.1, 16), "w3": rng.normal(0, 0.3, 16),
         "b3": rng.normal(0, 0.1, 1)}
    sets = np.stack([rng.choice(n, size=k, replace=False) for _ in range(B)])
    target = rng.normal(size=B)

    def rt(x):  # torch's own bfloat16 conversion (through float32)
        return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    class Value(torch.autograd.Function):  # rounded value, gradient passed through
        @staticmethod
        def forward(ctx, x):
            return rt(x)

        @staticmethod
        def backward(ctx, g):
            return g

    class Grad(torch.autograd.Function):  # value passed through, gradient rounded
        @staticmethod
        def forward(ctx, x):
            return x.clone()

        @staticmethod
        def backward(ctx, g):
            return rt(g)

    t = {kk: torch.tensor(v, dtype=torch.float64, requires_grad=True) for kk, v in p.items()}
    x = Grad.apply(Value.apply(Value.apply(t["E"])[torch.tensor(sets)].sum(dim=1)))
    z1 = Grad.apply(x @ Value.apply(t["W1"]).T + t["b1"])
    h1 = Value.apply(torch.relu(z1))
    z2 = Grad.apply(h1 @ Value.apply(t["W2"]).T + t["b2"])
    h2 = Value.apply(torch.relu(z2))
    yhat = h2 @ Value.apply(t["w3"]) + t["b3"]
    loss_t = torch.mean((yhat - torch.tensor(target)) ** 2)
    loss_t.backward()
    loss, g, f = S.loss_and_grads(p, sets, target, bf16_ops=True)
    assert abs(loss - loss_t.item()) <= 1e-12
    assert np.allclose(f["yhat"], yhat.detach().numpy(), rtol=1e-12, atol=1e-12)
    for kk in S.TENSORS:
        assert np.allclose(g[kk], t[kk].grad.numpy(), rtol=1e-10, atol=1e-12), kk


def test_judge_sample_is_evenly_spaced():
    assert np.array_equal(S.judge_sample(10), np.arange(10))
    assert np.array_equal(S.judge_sample(1024), np.arange(1024))
    for m in (1025, 3000, 4096, 10 ** 6):
        idx = S.judge_sample(m)
        gaps = np.diff(idx)
        assert len(idx) == 1024 and idx[0] == 0 and idx[-1] < m
        assert gaps.min() >= m // 1024 and gaps.max() <= -(-m // 1024)
        # spread over the whole range: the last entry is within one gap of the end
        assert m - idx[-1] <= -(-m // 1024)


def test_judge_statistics_pins():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(15)
    F = rng.integers(0, 10 ** 9, size=3000)
    F[:500] = F[0]  # ties
    mu, sd = 15.0, 2.0
    # exact predictions: zero relative error and, over the judged sample,
    # Spearman equal to scipy's on the same values
    y_exact = (np.log1p(F.astype(np.float64)) - mu) / sd
    rho, rel = S.judge_stats(y_exact, F, mu, sd)
    assert abs(rho - 1.0) < 1e-12 and rel < 1e-9
    # predicting 2 PC + 1 everywhere: relative error (PC + 1) / max(PC, 1)
    y2 = (np.log(2.0 * F.astype(np.float64) + 2.0) - mu) / sd
    idx = S.judge_sample(len(F))
    _, rel2 = S.judge_stats(y2, F, mu, sd)
    f = F[idx].astype(np.float64)
    assert abs(rel2 - np.mean((f + 1.0) / np.maximum(f, 1.0))) < 1e-9 * rel2
    # a noisy predictor: scipy's Spearman on the judged entries
    y = y_exact + rng.normal(size=3000)
    rho3, _ = S.judge_stats(y, F, mu, sd)
    assert abs(rho3 - spearmanr(y[idx], F[idx]).correlation) < 1e-12


def test_judge_extra_selection():
    """The judge's extra sample: the `count` non-pooled children with the
    smallest (stream-7 key, index), checked against an independent ranking
    (numpy lexsort over all keys), and its frequency is uniform over the
    non-pooled children across generations."""
    seed, lam = 9, 200
    rng = np.random.default_rng(16)
    pool = np.sort(rng.choice(lam, size=64, replace=False))
    for gen, count in ((3, 32), (4, 1), (5, 136)):
        got = S.judge_extra(seed, gen, lam, pool, count)
        keys = np.array([int(O.draw(seed, o, 1, gen, 7)[0]) for o in range(lam)], dtype=np.int64)
        keys[pool] = np.iinfo(np.int64).max  # pooled children never qualify
        order = np.lexsort((np.arange(lam), keys))
        assert np.array_equal(got, np.sort(order[:count]))
        assert not np.intersect1d(got, pool).size and np.all(np.diff(got) > 0)
    # count = every child outside the pool: exactly those
    assert np.array_equal(S.judge_extra(seed, 6, lam, pool, lam - 64), np.setdiff1d(np.arange(lam), pool))
    # uniform over the 136 non-pooled children: chi-square over 300 generations
    hits = np.zeros(lam)
    gens = 300
    for gen in range(1, gens + 1):
        hits[S.judge_extra(seed, gen, lam, pool, 8)] += 1
    free = np.setdiff1d(np.arange(lam), pool)
    assert not hits[pool].any()
    expected = gens * 8 / len(free)
    chi2 = float(((hits[free] - expected) ** 2 / expected).sum())
    # 135 degrees of freedom: mean 135, sd ~16.4; 6 sd above is far in the tail
    assert chi2 < 135 + 6 * math.sqrt(2 * 135)
