"""Pure-Python mini reference of the CND genetic algorithm (test
infrastructure only, small cases).

A second, independent transcription of the same method as ``gapa_oracle.c``:
Python integers for Philox4x32-10, a dictionary-of-sets BFS for pairwise
connectivity, and lists for the genetic operators.  It exists so that a slip
in the C oracle's transcription (a wrong stream, slot or tie-break) shows up as
a disagreement on small workloads.  Section and equation references are to the
paper (Section III-B genetic operators, eq. 2-11).
"""
from __future__ import annotations

M32 = 0xFFFFFFFF
ST_INIT, ST_SELECT, ST_XOVER, ST_REPAIR, ST_MUTATE = 0, 1, 2, 3, 4


def philox4x32_10(ctr, key):
    """Salmon et al. (SC'11): ten rounds of two 32x32->64 multiplications with
    a Weyl-sequence key schedule."""
    c0, c1, c2, c3 = (int(x) & M32 for x in ctr)
    k0, k1 = (int(x) & M32 for x in key)
    for _ in range(10):
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c3 ^ k1) & M32, p0 & M32
        k0 = (k0 + 0x9E3779B9) & M32
        k1 = (k1 + 0xBB67AE85) & M32
    return (c0, c1, c2, c3)


def draw(seed, slot, ind, gen, stream, attempt=0):
    return philox4x32_10((slot, ind, gen, (stream << 24) | attempt), (seed & M32, seed >> 32))


def bounded(w, m):
    return (w * m) >> 32


def threshold(p):
    if not p > 0:
        return 0
    if p >= 1:
        return 1 << 32
    return int(p * 4294967296.0)


def pc_bfs(n, adj, removed):
    """Pairwise connectivity and largest component of G - removed."""
    removed = set(removed)
    seen = set()
    pc = 0
    mcn = 0
    for s in range(n):
        if s in removed or s in seen:
            continue
        seen.add(s)
        frontier = [s]
        size = 0
        while frontier:
            size += len(frontier)
            nxt = []
            for v in frontier:
                for u in adj[v]:
                    if u not in removed and u not in seen:
                        seen.add(u)
                        nxt.append(u)
            frontier = nxt
        pc += size * (size - 1) // 2
        mcn = max(mcn, size)
    return pc, mcn


def adjacency(graph):
    rp = graph.row_ptr.tolist()
    ci = graph.col_idx.tolist()
    return [ci[rp[v]:rp[v + 1]] for v in range(graph.n)]


class MiniGA:
    def __init__(self, graph, k, pop, seed, pc=0.7, pm=0.05, tournament=2, offspring=0):
        self.n = graph.n
        self.adj = adjacency(graph)
        self.k, self.P, self.seed, self.T = k, pop, seed, tournament
        self.L = offspring or pop
        self.t_pc, self.t_pm = threshold(pc), threshold(pm)
        rows = [self._init_row(i) for i in range(pop)]
        fit = [self.fitness(r) for r in rows]
        order = sorted(range(pop), key=lambda i: (fit[i], i))
        self.pop = [rows[i] for i in order]
        self.F = [fit[i] for i in order]
        self.generation = 0

    def fitness(self, row):
        return pc_bfs(self.n, self.adj, row)[0]

    def _uniform_outside(self, members, slot, ind, gen, stream):
        t = 0
        while True:
            u = bounded(draw(self.seed, slot, ind, gen, stream, t)[0], self.n)
            if u not in members:
                return u
            t += 1

    def _init_row(self, i):
        row, members = [], set()
        for j in range(self.k):
            u = self._uniform_outside(members, j, i, 0, ST_INIT)
            row.append(u)
            members.add(u)
        return sorted(row)

    def _donor(self, gen, o):
        best = None
        for c in range(self.T):
            w = draw(self.seed, c // 4, o, gen, ST_SELECT)
            a = bounded(w[c % 4], self.P)
            if best is None or (self.F[a], a) < (self.F[best], best):
                best = a
        return best

    def child(self, gen, o):
        base = self.pop[o % self.P]
        donor = self.pop[self._donor(gen, o)]
        kid, mut = [], []
        for j in range(self.k):
            w = draw(self.seed, j, o, gen, ST_XOVER)
            kid.append(donor[j] if w[0] < self.t_pc else base[j])
            mut.append(w[1] < self.t_pm)
        members, dups = set(), []
        for j, v in enumerate(kid):
            if v in members:
                dups.append(j)
            else:
                members.add(v)
        for j in dups:
            u = self._uniform_outside(members, j, o, gen, ST_REPAIR)
            kid[j] = u
            members.add(u)
        for j in range(self.k):
            if mut[j]:
                u = self._uniform_outside(members, j, o, gen, ST_MUTATE)
                members.discard(kid[j])
                members.add(u)
                kid[j] = u
        return sorted(kid)

    def step(self, pool_idx=None):
        g = self.generation + 1
        kids = [self.child(g, o) for o in range(self.L)]
        pool = list(range(self.L)) if pool_idx is None else list(pool_idx)
        entries = [(self.F[r], r, self.pop[r]) for r in range(self.P)]
        entries += [(self.fitness(kids[o]), self.P + o, kids[o]) for o in pool]
        entries.sort(key=lambda e: (e[0], e[1]))
        self.pop = [e[2] for e in entries[: self.P]]
        self.F = [e[0] for e in entries[: self.P]]
        self.generation = g
        return kids
