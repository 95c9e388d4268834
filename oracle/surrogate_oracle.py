"""Oracle of the learned screening surrogate (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module; it shares no code with the HIP library.

The surrogate is an extension, not part of the paper: the paper's GA
evaluates every offspring exactly (Section III-B/C).  Here a small network
predicts the fitness of each offspring of a large pool so that only the most
promising fraction is evaluated exactly; the exact evaluator stays the judge
(the GA state only ever holds exact fitness values).

Model, for a removed-node set S (an individual) over node embeddings E [n, D]:

    x(S) = sum_{v in S} E[v]                                   (D)
    z1 = W1 x + b1,  h1 = relu(z1)                             (H)
    z2 = W2 h1 + b2, h2 = relu(z2)                             (H)
    yhat = w3 . h2 + b3

trained on y = ln(1 + PC(S)) standardised by the mean and spread of the
labels held in the replay buffer, with the mean squared error and Adam
(Kingma and Ba, ICLR 2015, Algorithm 1: bias-corrected first and second
moment estimates; lazy on the embedding table, whose gradient is sparse).  Everything here is float64.  With ``bf16=True`` the
forward and backward passes round the operands of every product to bfloat16
(through float32, round to nearest even) exactly where the device kernels
do, so that the device can be compared tightly; without it they are the
plain definition.

Random numbers (initial weights, training batches) come from Philox4x32-10
through the C oracle: stream 5 for initial weights (``cnd_oracle.uniform_sym``)
and stream 6 for batch sampling.
"""
from __future__ import annotations

import math

import numpy as np

from . import cnd_oracle as O

ST_SURR_INIT = 5
ST_SURR_SAMPLE = 6
TENSORS = ("E", "W1", "b1", "W2", "b2", "w3", "b3")


# --- numerics helpers ---------------------------------------------------------

def bf16(x) -> np.ndarray:
    """Round to bfloat16 through float32 (round to nearest, ties to even),
    returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def relu(x):
    return np.maximum(x, 0.0)


# --- parameters ---------------------------------------------------------------

def init_bounds(D: int, H: int) -> dict:
    """Uniform ranges of the initial weights: E in (-0.05, 0.05); W1, W2 in
    (-sqrt(6 / fan_in), +sqrt(6 / fan_in)) (He et al. 2015, uniform variant,
    for layers followed by ReLU); w3 in (-sqrt(3 / fan_in), +sqrt(3 / fan_in));
    biases zero."""
    return {"E": 0.05, "W1": math.sqrt(6.0 / D), "W2": math.sqrt(6.0 / H), "w3": math.sqrt(3.0 / H)}


def init_params(seed: int, n: int, D: int = 64, H: int = 256) -> dict:
    """Initial parameters as the float32 values the device stores (held in
    float64).  Tensor ids of the Philox draws: E 0, W1 1, W2 2, w3 3."""
    b = init_bounds(D, H)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    return {
        "E": f32(O.uniform_sym(seed, 0, n, D, b["E"])),
        "W1": f32(O.uniform_sym(seed, 1, H, D, b["W1"])),
        "b1": np.zeros(H),
        "W2": f32(O.uniform_sym(seed, 2, H, H, b["W2"])),
        "b2": np.zeros(H),
        "w3": f32(O.uniform_sym(seed, 3, 1, H, b["w3"]))[0],
        "b3": np.zeros(1),
    }


# --- forward / backward -------------------------------------------------------

def membership(sets: np.ndarray, n: int):
    """The B x n matrix of a batch of sets: entry (b, v) counts the
    occurrences of v in row b (a sparse matrix, so that sums over the rows of
    the embedding table cost O(B k D) at any n)."""
    from scipy.sparse import csr_matrix
    S = np.asarray(sets, dtype=np.int64)
    B, k = S.shape
    rows = np.repeat(np.arange(B, dtype=np.int64), k)
    return csr_matrix((np.ones(B * k), (rows, S.ravel())), shape=(B, n))


def embed(E: np.ndarray, sets: np.ndarray) -> np.ndarray:
    """x(S) for each row of sets [B, k]: the sum of the rows of E, i.e. the
    membership matrix times E."""
    return np.asarray(membership(sets, E.shape[0]) @ E)


def forward(p: dict, sets: np.ndarray, bf16_ops: bool = False) -> dict:
    r = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    x = embed(r(p["E"]), sets)
    xb = r(x)
    z1 = xb @ r(p["W1"]).T + p["b1"]
    h1 = r(relu(z1))
    z2 = h1 @ r(p["W2"]).T + p["b2"]
    h2 = r(relu(z2))
    yhat = h2 @ r(p["w3"]) + p["b3"][0]
    return {"x": xb, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "yhat": yhat}


def loss_and_grads(p: dict, sets: np.ndarray, target: np.ndarray, bf16_ops: bool = False):
    """Mean squared error over the batch and its gradient for every
    parameter (backpropagation through the model above; dE[v] sums dx over
    the samples whose set holds v, once per occurrence)."""
    r = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    f = forward(p, sets, bf16_ops)
    B = sets.shape[0]
    err = f["yhat"] - target
    loss = float(np.mean(err * err))
    dy = 2.0 * err / B
    g = {}
    g["w3"] = f["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, r(p["w3"])) * (f["z2"] > 0)
    dz2b = r(dz2)
    g["W2"] = dz2b.T @ f["h1"]
    g["b2"] = dz2b.sum(axis=0)
    dh1 = dz2b @ r(p["W2"])
    dz1 = dh1 * (f["z1"] > 0)
    dz1b = r(dz1)
    g["W1"] = dz1b.T @ f["x"]
    g["b1"] = dz1b.sum(axis=0)
    dx = r(dz1b @ r(p["W1"]))
    # dE = M^T dx with M the membership matrix: row v sums dx over the
    # samples whose set holds v, once per occurrence
    g["E"] = np.asarray(membership(sets, p["E"].shape[0]).T @ dx)
    return loss, g, f


# --- Adam ---------------------------------------------------------------------

class Adam:
    """Kingma and Ba (2015), Algorithm 1:
    m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
    theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
    dense for every tensor except the embedding table when `rows` is given:
    there it is lazy, as for sparse gradients (torch.optim.SparseAdam): only
    the listed rows (the nodes present in the batch) update their moments and
    weights, with the global step count t."""

    def __init__(self, params: dict, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def _update(self, params, grads, k, sel):
        m, v, g = self.m[k], self.v[k], grads[k]
        m[sel] = self.b1 * m[sel] + (1.0 - self.b1) * g[sel]
        v[sel] = self.b2 * v[sel] + (1.0 - self.b2) * g[sel] ** 2
        params[k][sel] = params[k][sel] - self.lr * (m[sel] / self.c1) / (np.sqrt(v[sel] / self.c2) + self.eps)

    def step(self, params: dict, grads: dict, rows=None):
        self.t += 1
        self.c1 = 1.0 - self.b1 ** self.t
        self.c2 = 1.0 - self.b2 ** self.t
        for k in params:
            if k == "E" and rows is not None:
                self._update(params, grads, k, np.asarray(rows, dtype=np.int64))
            else:
                self._update(params, grads, k, slice(None))


def batch_rows(sets) -> np.ndarray:
    """Nodes present in a batch of sets (the rows of E a lazy step touches)."""
    return np.unique(np.asarray(sets, dtype=np.int64))


# --- labels, screening, judge statistics -----------------------------------------

def label(F) -> np.ndarray:
    """Training label of an exact fitness: ln(1 + PC)."""
    return np.log1p(np.asarray(F, dtype=np.float64))


SPREAD_FLOOR = 1e-6


def standardise(labels: np.ndarray):
    """Mean and spread of the buffered labels: sqrt(variance + 1e-12), the
    population variance floored so that a buffer of (nearly) equal labels
    gives targets near zero instead of amplified rounding noise (1e-6 in
    ln(1 + PC) is far below the differences that rank individuals)."""
    mu = float(np.mean(labels))
    var = float(np.mean((labels - mu) ** 2))
    return mu, math.sqrt(var + SPREAD_FLOOR ** 2)


def screen(yhat: np.ndarray, m: int) -> np.ndarray:
    """The m offspring with the smallest predictions (ties: smaller index
    first), returned in ascending index order."""
    order = np.lexsort((np.arange(len(yhat)), np.asarray(yhat)))
    return np.sort(order[:m])


def average_ranks(a: np.ndarray) -> np.ndarray:
    """Ranks 1..m; tied values share the mean of their ranks."""
    a = np.asarray(a, dtype=np.float64)
    less = (a[None, :] < a[:, None]).sum(axis=1)
    equal = (a[None, :] == a[:, None]).sum(axis=1)
    return less + (equal + 1) / 2.0


def spearman(a, b) -> float:
    """Spearman's rank correlation: Pearson's correlation of the average
    ranks."""
    ra, rb = average_ranks(a), average_ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = math.sqrt(float((ra * ra).sum() * (rb * rb).sum()))
    return float((ra * rb).sum() / den) if den > 0 else 0.0


JUDGE_MAX = 1024


def judge_sample(m: int, cap: int = JUDGE_MAX) -> np.ndarray:
    """Entries of m evaluated children the judge looks at: all of them when
    m <= cap, else cap of them evenly spaced (entry i is floor(i m / cap))."""
    J = min(m, cap)
    return np.array([(i * m) // J for i in range(J)], dtype=np.int64)


def judge_stats(yhat, F, mu: float, sd: float, cap: int = JUDGE_MAX):
    """The judge of a generation over its evaluated children (yhat: their
    predictions on the standardised scale, F: their exact PC, same order):
    Spearman's correlation between prediction and PC, and the mean relative
    error of the predicted PC expm1(yhat sd + mu) (the label is ln(1 + PC)),
    relative to max(PC, 1); both over judge_sample(len(F))."""
    idx = judge_sample(len(F), cap)
    y = np.asarray(yhat, dtype=np.float64)[idx]
    f = np.asarray(F, dtype=np.int64)[idx]
    rel = np.abs(np.expm1(y * sd + mu) - f.astype(np.float64)) / np.maximum(f.astype(np.float64), 1.0)
    return spearman(y, f.astype(np.float64)), float(rel.mean())


def sample_batch(seed: int, gen: int, step: int, B: int, count: int) -> np.ndarray:
    """Buffer entries of training step `step` of generation `gen`: entry j is
    bounded(w, count), w the first word of draw(seed, slot j, ind step, gen,
    stream 6)."""
    return np.array([O.bounded(int(O.draw(seed, j, step, gen, ST_SURR_SAMPLE)[0]), count) for j in range(B)],
                    dtype=np.int64)


# --- the surrogate-screened GA, replayed ------------------------------------------

class SurrogateGA:
    """The GA of ``cnd_oracle.OracleGA`` with learned screening, replayed:
    each generation takes the screened offspring indices (the device's
    decisions: they depend on floating-point predictions) and reproduces the
    integer state exactly, while it trains its own float64 copy of the model
    on the same data.

    Per generation g: the operators make `offspring` children; the pool (all
    of them during the first `warmup` generations, else the given indices)
    is evaluated exactly; elitism keeps the P best of parents and pool; the
    pool's (set, label) pairs enter a ring buffer of `buffer` entries in pool
    order; then `steps` Adam steps run, each on `batch` entries sampled with
    stream 6, against labels standardised over the buffer."""

    def __init__(self, graph, k, pop, seed, offspring, pc=0.7, pm=0.05, tournament=2, D=64, H=256, lr=1e-3,
                 batch=1024, steps=4, warmup=10, buffer=65536, bf16_ops=False, nthreads=None):
        self.ga = O.OracleGA(graph, k, pop, seed, pc, pm, tournament, offspring, nthreads)
        self.seed, self.k = seed, k
        self.batch, self.steps, self.warmup, self.cap = batch, steps, warmup, buffer
        self.bf16_ops = bf16_ops
        self.params = init_params(seed, graph.n, D, H)
        self.opt = Adam(self.params, lr)
        self.buf_sets = np.zeros((buffer, k), dtype=np.int32)
        self.buf_y = np.zeros(buffer)
        self.appended = 0
        self.losses = []
        self.label_stats = {}  # generation -> (mean, spread) its training standardised with

    @property
    def generation(self):
        return self.ga.generation

    def append(self, sets, F):
        for row, f in zip(sets, F):
            slot = self.appended % self.cap
            self.buf_sets[slot] = row
            self.buf_y[slot] = label(f)
            self.appended += 1

    def train(self, gen):
        count = min(self.appended, self.cap)
        mu, sd = standardise(self.buf_y[:count])
        self.label_stats[gen] = (mu, sd)
        for t in range(self.steps):
            idx = sample_batch(self.seed, gen, t, self.batch, count)
            sets = self.buf_sets[idx]
            loss, g, _ = loss_and_grads(self.params, sets, (self.buf_y[idx] - mu) / sd, self.bf16_ops)
            self.opt.step(self.params, g, rows=batch_rows(sets))
            self.losses.append(loss)
        return mu, sd

    def step(self, pool=None, extra=None):
        """One generation.  pool: the children that enter elitism (all during
        warm-up or when None); extra: children evaluated for the judge only
        (they join the buffer after the pool)."""
        gen = self.ga.generation + 1
        p = self.ga.params
        if gen <= self.warmup or pool is None:
            pool = np.arange(p.offspring)
        pool = np.asarray(pool, dtype=np.int32)
        kids, kf = self.ga.step(pool_idx=pool, keep_children=True)
        self.append(kids[pool], kf[pool])
        if extra is not None and len(extra):
            extra = np.asarray(extra, dtype=np.int64)
            self.append(kids[extra], O.eval_population(self.ga.graph, kids[extra]))
        self.train(gen)
        return kids, kf, pool


def judge_extra(seed: int, gen: int, lam: int, pool, count: int) -> np.ndarray:
    """The judge's unbiased sample of a screened generation: the `count`
    children outside the pool with the smallest (first word of draw(seed, o,
    1, gen, stream 7), o), ascending."""
    chosen = set(int(x) for x in pool)
    keys = [(int(O.draw(seed, o, 1, gen, 7)[0]), o) for o in range(lam) if o not in chosen]
    return np.sort(np.array([o for _, o in sorted(keys)[:count]], dtype=np.int64))
