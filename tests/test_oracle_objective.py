"""The oracle GA with the MCN objective (the largest surviving component,
the CND fitness of Sec. III-D) instead of PC.

Pins: every individual's fitness equals the MCN of its row computed by the
plain BFS; rows are ordered by (fitness, tag); the best MCN never rises over
the generations (elitism keeps the parents); the default objective is PC and
keeps the stored PC trajectories (tested elsewhere) unchanged."""
import numpy as np

from oracle import cnd_oracle as O
from paper_2412_20980_amd import inputs


def test_fitness_is_the_bfs_mcn_of_each_row():
    g = inputs.erdos_renyi(300, 3.0, seed=21)
    ga = O.OracleGA(g, 15, 24, 7, 0.7, 0.1, 2, 40, objective="mcn")
    best = []
    for gen in range(8):
        for row, f in zip(ga.pop, ga.F):
            assert f == O.pc(g, row)[1]
        assert np.all(np.diff(ga.F) >= 0)
        best.append(int(ga.F[0]))
        ga.step()
    assert all(b >= a for a, b in zip(best[1:], best[:-1]))


def test_objectives_differ_and_default_is_pc():
    g = inputs.barabasi_albert(200, 3, seed=1)
    a = O.OracleGA(g, 10, 16, 3)
    b = O.OracleGA(g, 10, 16, 3, objective="pc")
    c = O.OracleGA(g, 10, 16, 3, objective="mcn")
    for _ in range(3):
        a.step()
        b.step()
        c.step()
    assert np.array_equal(a.F, b.F) and np.array_equal(a.pop, b.pop)
    for row, f in zip(a.pop, a.F):
        assert f == O.pc(g, row)[0]
    assert not np.array_equal(a.F, c.F)
