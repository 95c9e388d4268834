"""Pins of the oracle's genetic algorithm (CPU only).

The paper fixes the operators' algebra (Section III-B: crossover mask eq. 3-4
and blend eq. 6, mutation mask eq. 7-8 and blend eq. 9, elitism eq. 10-11) but
prints no trajectory; the GA is pinned here by those identities, by
invariants, by special cases and by an independent Python transcription.
"""
import hashlib
import itertools

import numpy as np
import pytest

from oracle import cnd_oracle as O
from oracle import miniref
from paper_2412_20980_amd import inputs


def check_population(g, pop, F, k):
    P = pop.shape[0]
    assert pop.shape == (P, k)
    assert np.all(pop >= 0) and np.all(pop < g.n)
    assert np.all(np.diff(pop, axis=1) > 0), "rows sorted, genes distinct"
    assert np.all(np.diff(F) >= 0), "population ordered by fitness"
    for i in range(0, P, max(1, P // 8)):
        assert F[i] == O.pc(g, pop[i])[0]


def test_mini_reference_trajectory_ba200(ba200):
    W = inputs.workload("ba200_k10_p32")
    ga = O.OracleGA(ba200, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament)
    mg = miniref.MiniGA(ba200, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament)
    assert ga.pop.tolist() == mg.pop and ga.F.tolist() == mg.F
    best = [int(ga.F[0])]
    for _ in range(W.generations):
        ga.step()
        mg.step()
        assert ga.pop.tolist() == mg.pop and ga.F.tolist() == mg.F
        check_population(ba200, ga.pop, ga.F, W.k)
        best.append(int(ga.F[0]))
    assert all(b1 <= b0 for b0, b1 in zip(best, best[1:])), "elitism never loses the best"
    assert best[-1] < best[0]


@pytest.mark.parametrize("n,k,P,T,pc,pm,lam,seed", [
    (60, 5, 8, 2, 0.5, 0.3, 0, 3),
    (40, 20, 5, 3, 0.9, 0.2, 7, 4),     # k = n/2, odd tournament, lambda > P
    (90, 12, 6, 5, 0.7, 0.05, 3, 5),    # T = 5 spans two SELECT draws, lambda < P
    (30, 1, 4, 1, 1.0, 1.0, 0, (1 << 40) + 9),  # 64-bit seed, certain coins
    (50, 7, 1, 2, 0.7, 0.5, 0, 6),      # P = 1
])
def test_mini_reference_small_configs(n, k, P, T, pc, pm, lam, seed):
    g = inputs.erdos_renyi(n, 3.0, seed=n)
    ga = O.OracleGA(g, k, P, seed, pc, pm, T, lam)
    mg = miniref.MiniGA(g, k, P, seed, pc, pm, T, lam)
    for gen in range(6):
        assert ga.pop.tolist() == mg.pop and ga.F.tolist() == mg.F, gen
        ga.step()
        mg.step()
        check_population(g, ga.pop, ga.F, k)


def test_pooled_subset_matches_mini_reference():
    g = inputs.barabasi_albert(120, 2, seed=8)
    ga = O.OracleGA(g, 8, 10, 1, 0.7, 0.1, 2, 40)
    mg = miniref.MiniGA(g, 8, 10, 1, 0.7, 0.1, 2, 40)
    rng = np.random.default_rng(0)
    for _ in range(4):
        pool = np.sort(rng.choice(40, size=12, replace=False))
        kids, kf = ga.step(pool_idx=pool, keep_children=True)
        mkids = mg.step(pool_idx=pool.tolist())
        assert kids.tolist() == mkids
        assert ga.pop.tolist() == mg.pop and ga.F.tolist() == mg.F
        assert np.all(kf[np.setdiff1d(np.arange(40), pool)] == -1)


def test_crossover_and_mutation_blend_identities(ba10k):
    """Before repair the child is eq. 6: RC*donor + (1-RC)*base with
    RC_j = [w0 < T_pc]; the mutation mask RM_j = [w1 < T_pm] (eq. 8) marks
    exactly the slots that change after repair (eq. 9)."""
    W = inputs.workload("ba10k_k100_p256")
    ga = O.OracleGA(ba10k, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament, nthreads=8)
    p = ga.params
    for o in range(0, 256, 17):
        child, pre_r, pre_m, d = O.make_child(p, 1, o, ga.pop, ga.F)
        base, donor = ga.pop[o % p.pop], ga.pop[d]
        w = np.array([O.draw(p.seed, j, o, 1, O.ST_XOVER) for j in range(p.k)], dtype=np.uint64)
        RC = w[:, 0] < p.t_pc
        RM = w[:, 1] < p.t_pm
        assert np.array_equal(pre_r, np.where(RC, donor, base))
        # repair rewrites exactly the slots whose value already sits at a lower slot
        dups = {j for j in range(p.k) if pre_r[j] in pre_r[:j]}
        assert set(np.nonzero(pre_m != pre_r)[0].tolist()) == dups
        assert len(set(pre_m.tolist())) == p.k
        # mutation changes exactly the masked slots (the replacement is a non-member)
        sorted_child_set = set(child.tolist())
        assert len(sorted_child_set) == p.k
        mutated_out = set(pre_m[RM].tolist()) - sorted_child_set
        assert len(mutated_out) <= int(RM.sum())
        assert set(pre_m[~RM].tolist()) <= sorted_child_set


def test_tournament_is_min_position_on_sorted_population(ba10k):
    W = inputs.workload("ba10k_k100_p256")
    ga = O.OracleGA(ba10k, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament, nthreads=8)
    p = ga.params
    for o in range(256):
        w = O.draw(p.seed, 0, o, 1, O.ST_SELECT)
        a, b = O.bounded(int(w[0]), p.pop), O.bounded(int(w[1]), p.pop)
        assert O.tournament(p, 1, o, ga.F) == min(a, b)


def test_rates_match_pc_and_pm():
    # over many (offspring, slot) coins the crossover and mutation fractions
    # are binomial(pc) and binomial(pm)
    p = O.make_params(10_000, 100, 256, seed=0, pc=0.7, pm=0.05)
    w = np.array([O.draw(0, j, o, 1, O.ST_XOVER) for o in range(50) for j in range(100)], dtype=np.uint64)
    N = w.shape[0]
    fx = (w[:, 0] < p.t_pc).mean()
    fm = (w[:, 1] < p.t_pm).mean()
    assert abs(fx - 0.7) < 4 * np.sqrt(0.7 * 0.3 / N)
    assert abs(fm - 0.05) < 4 * np.sqrt(0.05 * 0.95 / N)


def test_no_variation_is_a_fixed_point(ba200):
    # pc = pm = 0: every child copies its base row, ties keep the parents
    ga = O.OracleGA(ba200, 10, 32, 0, pc=0.0, pm=0.0)
    pop0, F0 = ga.pop.copy(), ga.F.copy()
    for _ in range(5):
        kids, _ = ga.step(keep_children=True)
        assert np.array_equal(kids, pop0[np.arange(32) % 32])
        assert np.array_equal(ga.pop, pop0) and np.array_equal(ga.F, F0)


def test_full_crossover_copies_donor(ba200):
    ga = O.OracleGA(ba200, 10, 32, 0, pc=1.0, pm=0.0)
    p = ga.params
    for o in range(32):
        child, pre_r, _, d = O.make_child(p, 1, o, ga.pop, ga.F)
        assert np.array_equal(child, ga.pop[d]) and np.array_equal(pre_r, ga.pop[d])


def test_mutation_draws_are_uniform_over_non_members():
    # one gene, certain mutation: the replacement is uniform over the other
    # n - 1 nodes (eq. 9's replacement genes, read as uniform non-members)
    g = inputs.erdos_renyi(12, 3.0, seed=1)
    p = O.make_params(12, 1, 1, seed=3, pc=0.0, pm=1.0)
    pop = np.array([[4]], dtype=np.int32)
    F = np.array([O.pc(g, pop[0])[0]], dtype=np.int64)
    counts = np.zeros(12, dtype=np.int64)
    trials = 3300
    for gen in range(1, trials + 1):
        child, pre_r, pre_m, _ = O.make_child(p, gen, 0, pop, F)
        assert pre_r[0] == 4 and pre_m[0] == 4
        counts[child[0]] += 1
    assert counts[4] == 0
    expected = trials / 11
    chi2 = (((counts - expected) ** 2 / expected)[np.arange(12) != 4]).sum()
    assert chi2 < 29.6  # 0.999 quantile, 10 dof


def test_init_rows_are_distinct_uniform_subsets():
    p = O.make_params(50, 10, 1, seed=9)
    seen = np.zeros(50, dtype=np.int64)
    for i in range(400):
        row = O.init_individual(p, i)
        assert np.all(np.diff(row) > 0)
        seen[row] += 1
    expected = 400 * 10 / 50
    chi2 = ((seen - expected) ** 2 / expected).sum()
    assert chi2 < 85.4  # 0.999 quantile, 49 dof


def test_ga_never_beats_brute_force_optimum():
    g = inputs.erdos_renyi(14, 3.0, seed=21)
    k = 3
    opt = min(O.pc(g, list(S))[0] for S in itertools.combinations(range(g.n), k))
    ga = O.OracleGA(g, k, 12, 2, 0.7, 0.2)
    for _ in range(40):
        ga.step()
        assert ga.F[0] >= opt
    assert ga.F[0] == opt  # a 364-subset space: 40 generations of 12 find it


def test_oracle_trajectory_hashes_stable(ba200):
    """The oracle's C1-shaped trajectory is deterministic across runs and
    thread counts."""
    W = inputs.workload("ba200_k10_p32")

    def run(nt):
        ga = O.OracleGA(ba200, W.k, W.pop, W.seed, W.pc, W.pm, W.tournament, nthreads=nt)
        h = hashlib.sha256()
        for _ in range(W.generations):
            ga.step()
            h.update(ga.pop.tobytes())
            h.update(ga.F.tobytes())
        return h.hexdigest()

    assert run(1) == run(8)


def test_oracle_state_is_complete_for_resume():
    """Checkpoint/resume on the oracle: the GA state is the ordered population,
    its fitness and the generation number (every draw is keyed by them), so a
    fresh GA given a copy of that state continues exactly like the original."""
    g = inputs.barabasi_albert(400, 2, seed=5)
    a = O.OracleGA(g, 12, 20, 3, 0.7, 0.1, 2, 30)
    for _ in range(6):
        a.step()
    b = O.OracleGA(g, 12, 20, 3, 0.7, 0.1, 2, 30)
    b.pop[:], b.F[:], b.generation = a.pop.copy(), a.F.copy(), a.generation
    for _ in range(5):
        a.step()
        b.step()
        assert np.array_equal(a.pop, b.pop) and np.array_equal(a.F, b.F)
