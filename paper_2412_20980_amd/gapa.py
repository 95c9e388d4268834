"""Python binding of libgapa.so (include/gapa.h): argument marshalling only.

Every step of fitness evaluation and of the genetic algorithm runs in the HIP
library; this module converts numpy arrays / torch tensors to pointers and
status codes to exceptions.  There is no fallback: if the library is not
built, importing the binding raises.

PyTorch, when installed, is imported before the library is loaded so that the
process maps a single HIP runtime (torch's); torch tensors on the GPU can then
be passed directly (GAPA_DEVICE_PTRS) together with torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # load torch's HIP runtime first, so libgapa binds to the same one
    import torch  # noqa: F401
    _HAVE_TORCH = True
except Exception:  # pragma: no cover - torch is part of the image
    torch = None
    _HAVE_TORCH = False

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgapa.so")

GAPA_OK = 0
GAPA_E_INVALID_ARG = 1
GAPA_E_BAD_GRAPH = 2
GAPA_E_BAD_GENE = 3
GAPA_E_NO_DEVICE = 4
GAPA_E_DEVICE = 5
GAPA_E_OOM = 6
GAPA_E_STATE = 7

GAPA_DEVICE_PTRS = 1 << 0
GAPA_TRUST_INPUT = 1 << 1
GAPA_WANT_MCN = 1 << 2
GAPA_UNIONFIND = 1 << 3
GAPA_GRAPH_REPLAY = 1 << 4
GAPA_MINIMISE_MCN = 1 << 5
GAPA_MAXIMISE_COMPONENTS = 1 << 6
GAPA_SCREEN_RANDOM = 1 << 0
SURROGATE_TENSORS = ("E", "W1", "b1", "W2", "b2", "w3", "b3")

EXPORTED = (
    "gapa_graph_create", "gapa_graph_destroy", "gapa_eval_population",
    "gapa_ga_create", "gapa_generation_step", "gapa_best", "gapa_get_population", "gapa_ga_destroy",
    "gapa_graph_set_timing", "gapa_graph_kernel_times", "gapa_ga_set_timing", "gapa_ga_kernel_times",
    "gapa_graph_fitness_stats", "gapa_ga_fitness_stats", "gapa_last_error", "gapa_version",
    "gapa_batch_create", "gapa_batch_step", "gapa_batch_best", "gapa_batch_get_population",
    "gapa_batch_set_timing", "gapa_batch_kernel_times", "gapa_batch_destroy",
    "gapa_surrogate_attach", "gapa_surrogate_stats", "gapa_surrogate_last_pool", "gapa_surrogate_predict",
    "gapa_surrogate_train_batch", "gapa_surrogate_tensor", "gapa_surrogate_last_predictions",
    "gapa_graph_get_tuning", "gapa_graph_set_tuning", "gapa_ga_autotune", "gapa_batch_autotune",
    "gapa_ga_record", "gapa_batch_record", "gapa_sixdst_eval", "gapa_ga_save", "gapa_ga_load",
    "gapa_ga_params", "gapa_batch_get_tuning", "gapa_batch_set_tuning", "gapa_surrogate_judge",
    "gapa_eval_population_noalloc", "gapa_best_async",
)


class GapaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gapa error {code}: {msg}")
        self.code = code


class gapa_params(C.Structure):
    _fields_ = [
        ("k", C.c_int32), ("pop", C.c_int32), ("tournament", C.c_int32), ("offspring", C.c_int32),
        ("seed", C.c_uint64), ("pc", C.c_double), ("pm", C.c_double),
        ("flags", C.c_uint32), ("reserved", C.c_int32),
    ]


class gapa_surrogate_params(C.Structure):
    _fields_ = [
        ("emb_dim", C.c_int32), ("hidden", C.c_int32), ("screen", C.c_int32), ("batch", C.c_int32),
        ("train_steps", C.c_int32), ("warmup_gens", C.c_int32), ("buffer", C.c_int32), ("fallback_gens", C.c_int32),
        ("lr", C.c_float), ("min_rho", C.c_float), ("flags", C.c_uint32), ("reserved", C.c_int32),
    ]


class gapa_surrogate_report(C.Structure):
    _fields_ = [
        ("generation", C.c_int64), ("evaluated", C.c_int32), ("pooled", C.c_int32), ("screened", C.c_int32),
        ("reserved", C.c_int32), ("spearman", C.c_double),
        ("rel_err", C.c_double), ("loss", C.c_double), ("fallbacks", C.c_int32), ("train_steps", C.c_int32),
        ("label_mean", C.c_double), ("label_spread", C.c_double),
    ]


class gapa_tuning(C.Structure):
    _fields_ = [("sweep_grid", C.c_int32), ("band_scan", C.c_int32), ("sweeps", C.c_int32),
                ("band_blocks", C.c_int32)]


class gapa_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2412_20980_amd.build_lib`")
    L = C.CDLL(LIB_PATH)
    vp, i32p, i64p = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.gapa_graph_create.argtypes = [C.c_int32, C.c_int64, vp, vp, C.c_uint32, C.POINTER(vp)]
    L.gapa_graph_destroy.argtypes = [vp]
    L.gapa_eval_population.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, C.c_uint32, vp]
    L.gapa_eval_population_noalloc.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, C.c_uint32, vp]
    L.gapa_ga_create.argtypes = [vp, C.POINTER(gapa_params), vp, C.POINTER(vp)]
    L.gapa_generation_step.argtypes = [vp, C.c_int32, vp]
    L.gapa_best.argtypes = [vp, vp, i64p, i64p]
    L.gapa_best_async.argtypes = [vp, vp, vp]
    L.gapa_get_population.argtypes = [vp, vp, vp]
    L.gapa_ga_destroy.argtypes = [vp]
    L.gapa_batch_create.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(gapa_params), vp, C.POINTER(vp)]
    L.gapa_batch_step.argtypes = [vp, C.c_int32, vp]
    L.gapa_batch_best.argtypes = [vp, C.c_int32, vp, i64p, i64p]
    L.gapa_batch_get_population.argtypes = [vp, C.c_int32, vp, vp]
    L.gapa_batch_destroy.argtypes = [vp]
    L.gapa_ga_record.argtypes = [vp, C.c_int32]
    L.gapa_ga_save.argtypes = [vp, C.c_char_p]
    L.gapa_ga_load.argtypes = [vp, C.c_char_p, vp, C.POINTER(vp)]
    L.gapa_ga_params.argtypes = [vp, C.POINTER(gapa_params), C.POINTER(C.c_int64)]
    L.gapa_sixdst_eval.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, C.c_uint32, vp]
    L.gapa_batch_record.argtypes = [vp, C.c_int32]
    L.gapa_graph_get_tuning.argtypes = [vp, C.POINTER(gapa_tuning)]
    L.gapa_graph_set_tuning.argtypes = [vp, C.POINTER(gapa_tuning)]
    L.gapa_ga_autotune.argtypes = [vp, C.c_int32, vp, C.POINTER(gapa_tuning)]
    L.gapa_batch_autotune.argtypes = [vp, C.c_int32, vp, C.POINTER(gapa_tuning)]
    L.gapa_batch_get_tuning.argtypes = [vp, C.POINTER(gapa_tuning)]
    L.gapa_batch_set_tuning.argtypes = [vp, C.POINTER(gapa_tuning)]
    L.gapa_surrogate_attach.argtypes = [vp, C.POINTER(gapa_surrogate_params), vp]
    L.gapa_surrogate_stats.argtypes = [vp, C.POINTER(gapa_surrogate_report)]
    L.gapa_surrogate_last_pool.argtypes = [vp, vp, C.c_int32, i32p]
    L.gapa_surrogate_judge.argtypes = [vp, vp, vp, C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_double), vp]
    L.gapa_surrogate_predict.argtypes = [vp, vp, C.c_int32, vp, vp]
    L.gapa_surrogate_last_predictions.argtypes = [vp, vp, C.c_int32, i32p]
    L.gapa_surrogate_train_batch.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, vp]
    L.gapa_surrogate_tensor.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int64, C.c_int32]
    for f in (L.gapa_graph_set_timing, L.gapa_ga_set_timing, L.gapa_batch_set_timing):
        f.argtypes = [vp, C.c_int32]
    for f in (L.gapa_graph_kernel_times, L.gapa_ga_kernel_times, L.gapa_batch_kernel_times):
        f.argtypes = [vp, C.POINTER(gapa_kernel_time), C.c_int32, i32p]
    for f in (L.gapa_graph_fitness_stats, L.gapa_ga_fitness_stats):
        f.argtypes = [vp, i64p]
    L.gapa_last_error.restype = C.c_char_p
    L.gapa_version.restype = C.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != GAPA_OK:
        raise GapaError(rc, lib().gapa_last_error().decode())


def gapa_version() -> str:
    return lib().gapa_version().decode()


def _is_dev_tensor(x) -> bool:
    return _HAVE_TORCH and isinstance(x, torch.Tensor) and x.is_cuda


def _stream_ptr(stream):
    if stream is None:
        if _HAVE_TORCH and torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return C.c_void_p(None)
    if _HAVE_TORCH and isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


# ----------------------------------------------------------------- graph ----

def gapa_graph_create(n: int, row_ptr, col_idx, flags: int = 0) -> C.c_void_p:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().gapa_graph_create(n, ci.shape[0], rp.ctypes.data, ci.ctypes.data if ci.size else None, flags,
                                   C.byref(h)))
    return h


def gapa_graph_destroy(h):
    _check(lib().gapa_graph_destroy(h))


def gapa_eval_population(h, genes, fitness=None, mcn=None, flags: int = 0, stream=None):
    """genes: numpy [P, k] int32 (host) or a torch int32 CUDA tensor (device;
    fitness/mcn must then be torch CUDA tensors too).  Returns fitness (and mcn
    when requested)."""
    if _is_dev_tensor(genes):
        assert genes.dtype == torch.int32 and genes.is_contiguous() and genes.dim() == 2
        P, k = genes.shape
        if fitness is None:
            fitness = torch.empty(P, dtype=torch.int64, device=genes.device)
        if flags & GAPA_WANT_MCN and mcn is None:
            mcn = torch.zeros(P, dtype=torch.int32, device=genes.device)
        _check(lib().gapa_eval_population(h, genes.data_ptr(), P, k, fitness.data_ptr(),
                                          mcn.data_ptr() if mcn is not None else None,
                                          flags | GAPA_DEVICE_PTRS, _stream_ptr(stream)))
    else:
        G = np.ascontiguousarray(genes, dtype=np.int32)
        if G.ndim == 1:
            G = G[None, :]
        P, k = G.shape
        if fitness is None:
            fitness = np.zeros(P, dtype=np.int64)
        if flags & GAPA_WANT_MCN and mcn is None:
            mcn = np.zeros(P, dtype=np.int32)
        _check(lib().gapa_eval_population(h, G.ctypes.data, P, k, fitness.ctypes.data,
                                          mcn.ctypes.data if mcn is not None else None,
                                          flags & ~GAPA_DEVICE_PTRS, _stream_ptr(stream)))
    return (fitness, mcn) if flags & GAPA_WANT_MCN else fitness


def gapa_eval_population_noalloc(h, genes, fitness=None, mcn=None, flags: int = 0, stream=None):
    """The allocation-free batched fitness: genes a torch int32 CUDA tensor
    [P, k]; fitness (and mcn with GAPA_WANT_MCN) torch CUDA tensors, made here
    when not given (torch's allocation, not the library's)."""
    assert _is_dev_tensor(genes) and genes.dtype == torch.int32 and genes.is_contiguous() and genes.dim() == 2
    P, k = genes.shape
    if fitness is None:
        fitness = torch.empty(P, dtype=torch.int64, device=genes.device)
    if flags & GAPA_WANT_MCN and mcn is None:
        mcn = torch.zeros(P, dtype=torch.int32, device=genes.device)
    _check(lib().gapa_eval_population_noalloc(h, genes.data_ptr(), P, k, fitness.data_ptr(),
                                              mcn.data_ptr() if mcn is not None else None,
                                              flags | GAPA_DEVICE_PTRS, _stream_ptr(stream)))
    return (fitness, mcn) if flags & GAPA_WANT_MCN else fitness


def gapa_surrogate_judge(yhat, fitness, label_mean: float, label_spread: float, pool=None, stream=None):
    """The judge's (Spearman, mean relative error) of predictions yhat (float32
    device tensor, indexed by pool, an int32 device tensor, or directly)
    against the exact fitness of the same children (int64 device tensor)."""
    assert _is_dev_tensor(yhat) and yhat.dtype == torch.float32 and yhat.is_contiguous()
    assert _is_dev_tensor(fitness) and fitness.dtype == torch.int64 and fitness.is_contiguous()
    m = fitness.numel()
    if pool is not None:
        assert _is_dev_tensor(pool) and pool.dtype == torch.int32 and pool.is_contiguous() and pool.numel() == m
    elif yhat.numel() < m:
        raise ValueError("yhat needs one entry per fitness value when no pool is given")
    out = (C.c_double * 2)()
    _check(lib().gapa_surrogate_judge(yhat.data_ptr(), pool.data_ptr() if pool is not None else None,
                                      fitness.data_ptr(), m, float(label_mean), float(label_spread), out,
                                      _stream_ptr(stream)))
    return out[0], out[1]


def gapa_sixdst_eval(h, genes, hops: int, pc=None, mcn=None, flags: int = 0, stream=None):
    """Dense reachability fitness (pc, mcn) of each row of genes: numpy
    [P, k] int32 (host) or a torch int32 CUDA tensor (device; pc and mcn are
    then torch CUDA tensors too)."""
    if _is_dev_tensor(genes):
        assert genes.dtype == torch.int32 and genes.is_contiguous() and genes.dim() == 2
        P, k = genes.shape
        pc = torch.empty(P, dtype=torch.int64, device=genes.device) if pc is None else pc
        mcn = torch.empty(P, dtype=torch.int32, device=genes.device) if mcn is None else mcn
        _check(lib().gapa_sixdst_eval(h, genes.data_ptr(), P, k, hops, pc.data_ptr(), mcn.data_ptr(),
                                      flags | GAPA_DEVICE_PTRS, _stream_ptr(stream)))
    else:
        G = np.ascontiguousarray(genes, dtype=np.int32)
        if G.ndim == 1:
            G = G[None, :]
        P, k = G.shape
        pc = np.zeros(P, dtype=np.int64) if pc is None else pc
        mcn = np.zeros(P, dtype=np.int32) if mcn is None else mcn
        _check(lib().gapa_sixdst_eval(h, G.ctypes.data, P, k, hops, pc.ctypes.data, mcn.ctypes.data,
                                      flags & ~GAPA_DEVICE_PTRS, _stream_ptr(stream)))
    return pc, mcn


def _fitness_stats(fn, h) -> dict:
    out = (C.c_int64 * 4)()
    _check(fn(h, out))
    return {"chunk": out[0], "pending_nodes": out[1], "leftover_pairs": out[2], "changing_sweeps": out[3]}


def _kernel_times(fn, h) -> dict:
    cap = 64
    arr = (gapa_kernel_time * cap)()
    cnt = C.c_int32(0)
    _check(fn(h, arr, cap, C.byref(cnt)))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(cnt.value, cap))}


class Graph:
    """A CSR graph resident on the current HIP device."""

    def __init__(self, n: int, row_ptr, col_idx, trust: bool = False, unionfind: bool = False):
        self.n = int(n)
        flags = (GAPA_TRUST_INPUT if trust else 0) | (GAPA_UNIONFIND if unionfind else 0)
        self.handle = gapa_graph_create(self.n, row_ptr, col_idx, flags)

    @classmethod
    def from_csr(cls, g, trust: bool = False, unionfind: bool = False) -> "Graph":
        return cls(g.n, g.row_ptr, g.col_idx, trust, unionfind)

    def eval(self, genes, want_mcn: bool = False, trust: bool = False, stream=None, objective: str = "pc"):
        """PC of each row (objective="components": survivors minus components)."""
        if objective not in ("pc", "components"):
            raise ValueError(f"objective must be 'pc' or 'components', not {objective!r}")
        flags = (GAPA_WANT_MCN if want_mcn else 0) | (GAPA_TRUST_INPUT if trust else 0) | _objective_flag(objective)
        return gapa_eval_population(self.handle, genes, flags=flags, stream=stream)

    def sixdst(self, genes, hops: int = 6, trust: bool = False, stream=None):
        """(pc, mcn) of the dense reachability fitness with `hops` hops."""
        return gapa_sixdst_eval(self.handle, genes, hops, flags=GAPA_TRUST_INPUT if trust else 0, stream=stream)

    def set_timing(self, on: bool = True):
        _check(lib().gapa_graph_set_timing(self.handle, int(on)))

    def kernel_times(self) -> dict:
        return _kernel_times(lib().gapa_graph_kernel_times, self.handle)

    def fitness_stats(self) -> dict:
        return _fitness_stats(lib().gapa_graph_fitness_stats, self.handle)

    def get_tuning(self) -> dict:
        t = gapa_tuning()
        _check(lib().gapa_graph_get_tuning(self.handle, C.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    def set_tuning(self, sweep_grid=4096, band_scan=32, sweeps=3, band_blocks=8192):
        t = gapa_tuning(sweep_grid=sweep_grid, band_scan=band_scan, sweeps=sweeps, band_blocks=band_blocks)
        _check(lib().gapa_graph_set_tuning(self.handle, C.byref(t)))

    def close(self):
        if self.handle:
            gapa_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -------------------------------------------------------------------- GA ----

def make_params(k, pop, seed, pc=0.7, pm=0.05, tournament=2, offspring=0, flags=0) -> gapa_params:
    return gapa_params(k=k, pop=pop, tournament=tournament, offspring=offspring, seed=seed, pc=pc, pm=pm,
                       flags=flags, reserved=0)


def gapa_ga_create(graph_handle, k, pop, seed, pc=0.7, pm=0.05, tournament=2, offspring=0, stream=None, flags=0):
    p = make_params(k, pop, seed, pc, pm, tournament, offspring, flags)
    h = C.c_void_p()
    _check(lib().gapa_ga_create(graph_handle, C.byref(p), _stream_ptr(stream), C.byref(h)))
    return h


def gapa_generation_step(h, n_generations: int = 1, stream=None):
    _check(lib().gapa_generation_step(h, n_generations, _stream_ptr(stream)))


def gapa_best(h, k: int):
    genes = np.zeros(k, dtype=np.int32)
    f = C.c_int64(0)
    g = C.c_int64(0)
    _check(lib().gapa_best(h, genes.ctypes.data, C.byref(f), C.byref(g)))
    return genes, int(f.value), int(g.value)


def gapa_get_population(h, P: int, k: int):
    genes = np.zeros((P, k), dtype=np.int32)
    F = np.zeros(P, dtype=np.int64)
    _check(lib().gapa_get_population(h, genes.ctypes.data, F.ctypes.data))
    return genes, F


def gapa_ga_destroy(h):
    _check(lib().gapa_ga_destroy(h))


_OBJECTIVE_FLAGS = {"pc": 0, "mcn": GAPA_MINIMISE_MCN, "components": GAPA_MAXIMISE_COMPONENTS}


def _objective_flag(objective: str) -> int:
    if objective not in _OBJECTIVE_FLAGS:
        raise ValueError(f"objective must be one of {sorted(_OBJECTIVE_FLAGS)}, not {objective!r}")
    return _OBJECTIVE_FLAGS[objective]


class GA:
    """The GA on one graph; generation 0 is drawn and evaluated at creation.
    replay=True records one generation as a HIP graph and replays it;
    objective="mcn" minimises the largest surviving component instead of PC;
    objective="components" maximises the number of components (fitness =
    survivors minus components, minimised)."""

    def __init__(self, graph: Graph, k, pop, seed, pc=0.7, pm=0.05, tournament=2, offspring=0, stream=None,
                 replay: bool = False, objective: str = "pc"):
        self.graph = graph
        self.k, self.pop = int(k), int(pop)
        flags = (GAPA_GRAPH_REPLAY if replay else 0) | _objective_flag(objective)
        self.handle = gapa_ga_create(graph.handle, k, pop, seed, pc, pm, tournament, offspring, stream, flags)

    def step(self, n: int = 1, stream=None):
        gapa_generation_step(self.handle, n, stream)

    def save(self, path: str):
        """Checkpoint: parameters, graph identity, generation, population."""
        _check(lib().gapa_ga_save(self.handle, os.fsencode(path)))

    @classmethod
    def load(cls, graph: Graph, path: str, stream=None) -> "GA":
        """A GA resumed from a checkpoint taken on the same graph."""
        h = C.c_void_p()
        _check(lib().gapa_ga_load(graph.handle, os.fsencode(path), _stream_ptr(stream), C.byref(h)))
        ga = cls.__new__(cls)
        ga.graph = graph
        ga.handle = h
        t = gapa_params()
        _check(lib().gapa_ga_params(h, C.byref(t), None))
        ga.k, ga.pop = int(t.k), int(t.pop)
        return ga

    def generation(self) -> int:
        g = C.c_int64()
        _check(lib().gapa_ga_params(self.handle, None, C.byref(g)))
        return int(g.value)

    def best(self):
        return gapa_best(self.handle, self.k)

    def best_async(self, out, index: int = 0, stream=None):
        """Enqueue a copy of the current best fitness into out[index] (an int64
        torch tensor in device or pinned host memory) without waiting."""
        assert out.dtype == torch.int64 and out.is_contiguous() and 0 <= index < out.numel()
        assert out.is_cuda or out.is_pinned()
        _check(lib().gapa_best_async(self.handle, out.data_ptr() + 8 * index, _stream_ptr(stream)))

    def population(self):
        return gapa_get_population(self.handle, self.pop, self.k)

    def set_timing(self, on: bool = True):
        _check(lib().gapa_ga_set_timing(self.handle, int(on)))

    def kernel_times(self) -> dict:
        return _kernel_times(lib().gapa_ga_kernel_times, self.handle)

    def fitness_stats(self) -> dict:
        return _fitness_stats(lib().gapa_ga_fitness_stats, self.handle)

    def record(self, n: int):
        """Record n generations as one HIP graph (replay mode); a later step(n)
        from the same buffer parity is one launch."""
        _check(lib().gapa_ga_record(self.handle, n))

    def autotune(self, reps: int = 3, stream=None) -> dict:
        t = gapa_tuning()
        _check(lib().gapa_ga_autotune(self.handle, reps, _stream_ptr(stream), C.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    # --- learned screening surrogate ---
    def attach_surrogate(self, screen: int, batch: int = 1024, train_steps: int = 4, warmup_gens: int = 10,
                         buffer: int = 65536, fallback_gens: int = 3, lr: float = 1e-3, min_rho: float = 0.3,
                         random_screen: bool = False, stream=None):
        sp = gapa_surrogate_params(emb_dim=64, hidden=256, screen=screen, batch=batch, train_steps=train_steps,
                                   warmup_gens=warmup_gens, buffer=buffer, fallback_gens=fallback_gens, lr=lr,
                                   min_rho=min_rho, flags=GAPA_SCREEN_RANDOM if random_screen else 0, reserved=0)
        _check(lib().gapa_surrogate_attach(self.handle, C.byref(sp), _stream_ptr(stream)))

    def surrogate_stats(self) -> dict:
        r = gapa_surrogate_report()
        _check(lib().gapa_surrogate_stats(self.handle, C.byref(r)))
        return {f: getattr(r, f) for f, _ in r._fields_}

    def last_pool(self) -> np.ndarray:
        cnt = C.c_int32(0)
        _check(lib().gapa_surrogate_last_pool(self.handle, None, 0, C.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.int32)
        if cnt.value:
            _check(lib().gapa_surrogate_last_pool(self.handle, out.ctypes.data, cnt.value, C.byref(cnt)))
        return out

    def last_predictions(self) -> np.ndarray:
        cnt = C.c_int32(0)
        _check(lib().gapa_surrogate_last_predictions(self.handle, None, 0, C.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.float32)
        if cnt.value:
            _check(lib().gapa_surrogate_last_predictions(self.handle, out.ctypes.data, cnt.value, C.byref(cnt)))
        return out

    def predict(self, genes, stream=None):
        """genes: torch int32 CUDA tensor [P, k]; returns float32 predictions."""
        assert _is_dev_tensor(genes) and genes.dtype == torch.int32 and genes.is_contiguous()
        if genes.dim() != 2 or genes.shape[1] != self.k:
            raise ValueError(f"genes must be [P, {self.k}] (the GA's budget), got {tuple(genes.shape)}")
        y = torch.empty(genes.shape[0], dtype=torch.float32, device=genes.device)
        _check(lib().gapa_surrogate_predict(self.handle, genes.data_ptr(), genes.shape[0], y.data_ptr(),
                                            _stream_ptr(stream)))
        return y

    def train_batch(self, genes, target, keep_grads: bool = True, stream=None):
        assert _is_dev_tensor(genes) and _is_dev_tensor(target)
        if genes.dtype != torch.int32 or not genes.is_contiguous() or genes.dim() != 2 or genes.shape[1] != self.k:
            raise ValueError(f"genes must be a contiguous int32 [B, {self.k}] tensor (the GA's budget)")
        if target.dtype != torch.float32 or not target.is_contiguous() or target.numel() != genes.shape[0]:
            raise ValueError("target must be a contiguous float32 tensor with one entry per row")
        _check(lib().gapa_surrogate_train_batch(self.handle, genes.data_ptr(), target.data_ptr(), genes.shape[0],
                                                int(keep_grads), _stream_ptr(stream)))

    def surrogate_tensor(self, name: str, grad: bool = False, n: int | None = None) -> np.ndarray:
        which = SURROGATE_TENSORS.index(name)
        n = self.graph.n if n is None else n
        shape = {"E": (n, 64), "W1": (256, 64), "b1": (256,), "W2": (256, 256), "b2": (256,), "w3": (256,),
                 "b3": (1,)}[name]
        out = np.zeros(shape, dtype=np.float32)
        _check(lib().gapa_surrogate_tensor(self.handle, which, int(grad), out.ctypes.data, out.size, 0))
        return out

    def set_surrogate_tensor(self, name: str, value):
        which = SURROGATE_TENSORS.index(name)
        arr = np.ascontiguousarray(value, dtype=np.float32)
        _check(lib().gapa_surrogate_tensor(self.handle, which, 0, arr.ctypes.data, arr.size, 1))

    def close(self):
        if self.handle:
            gapa_ga_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- batch ----

def gapa_batch_create(graph_handles, params, stream=None):
    """graph_handles: sequence of graph handles; params: sequence of
    gapa_params (one per instance)."""
    count = len(graph_handles)
    hs = (C.c_void_p * count)(*[h.value if isinstance(h, C.c_void_p) else h for h in graph_handles])
    ps = (gapa_params * count)(*params)
    out = C.c_void_p()
    _check(lib().gapa_batch_create(count, hs, ps, _stream_ptr(stream), C.byref(out)))
    return out


def gapa_batch_step(h, n_generations: int = 1, stream=None):
    _check(lib().gapa_batch_step(h, n_generations, _stream_ptr(stream)))


def gapa_batch_best(h, idx: int, k: int):
    genes = np.zeros(k, dtype=np.int32)
    f = C.c_int64(0)
    g = C.c_int64(0)
    _check(lib().gapa_batch_best(h, idx, genes.ctypes.data, C.byref(f), C.byref(g)))
    return genes, int(f.value), int(g.value)


def gapa_batch_get_population(h, idx: int, P: int, k: int):
    genes = np.zeros((P, k), dtype=np.int32)
    F = np.zeros(P, dtype=np.int64)
    _check(lib().gapa_batch_get_population(h, idx, genes.ctypes.data, F.ctypes.data))
    return genes, F


def gapa_batch_destroy(h):
    _check(lib().gapa_batch_destroy(h))


class Batch:
    """Independent GAs, one per (graph, parameters) pair, advanced together;
    instance b evolves exactly as GA(graphs[b], **params[b]) would."""

    def __init__(self, graphs, params, stream=None, replay: bool = True):
        """graphs: sequence of Graph; params: sequence of dicts with keys k,
        pop, seed and optionally pc, pm, tournament, offspring, objective
        ("pc" or "mcn", the same for every instance)."""
        self.graphs = list(graphs)
        self.params = [dict(p) for p in params]
        flags = GAPA_GRAPH_REPLAY if replay else 0
        ps = [make_params(flags=flags | _objective_flag(p.get("objective", "pc")),
                          **{key: v for key, v in p.items() if key != "objective"}) for p in self.params]
        self.handle = gapa_batch_create([g.handle for g in self.graphs], ps, stream)

    def __len__(self):
        return len(self.graphs)

    def step(self, n: int = 1, stream=None):
        gapa_batch_step(self.handle, n, stream)

    def best(self, idx: int):
        return gapa_batch_best(self.handle, idx, self.params[idx]["k"])

    def population(self, idx: int):
        p = self.params[idx]
        return gapa_batch_get_population(self.handle, idx, p["pop"], p["k"])

    def set_timing(self, level: int = 1):
        _check(lib().gapa_batch_set_timing(self.handle, int(level)))

    def record(self, n: int):
        _check(lib().gapa_batch_record(self.handle, n))

    def autotune(self, reps: int = 3, stream=None) -> dict:
        t = gapa_tuning()
        _check(lib().gapa_batch_autotune(self.handle, reps, _stream_ptr(stream), C.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    def kernel_times(self) -> dict:
        return _kernel_times(lib().gapa_batch_kernel_times, self.handle)

    def get_tuning(self) -> dict:
        t = gapa_tuning()
        _check(lib().gapa_batch_get_tuning(self.handle, C.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    def set_tuning(self, sweep_grid=4096, band_scan=32, sweeps=3, band_blocks=8192):
        t = gapa_tuning(sweep_grid=sweep_grid, band_scan=band_scan, sweeps=sweeps, band_blocks=band_blocks)
        _check(lib().gapa_batch_set_tuning(self.handle, C.byref(t)))

    def close(self):
        if self.handle:
            gapa_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
