"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/smnn.h declares, and rejects bad arguments on the host
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smnn.h")


def _lib():
    from paper_2410_06074_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libsmnn.so not built (run python -m paper_2410_06074_amd.build)")
    return L


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smnn_[a-z_]+)\s*\(", src)) - {"smnn_status", "smnn_mode"})


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("smnn_plan_create", "smnn_plan_destroy", "smnn_plan_sizes", "smnn_forward",
                     "smnn_backward", "smnn_status_string", "smnn_plan_query", "smnn_autotune",
                     "smnn_trace_enable", "smnn_trace_read"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings():
    L = _lib()
    lib = L.lib()
    assert lib.smnn_status_string(0) == b"ok"
    assert b"workspace" in lib.smnn_status_string(3)


def _desc(**kw):
    from paper_2410_06074_amd import _lib as L
    d = L.PlanDesc()
    d.order, d.n_init, d.n_inst, d.steps, d.steps_uniform = 2, 2, 4, None, 100
    d.mode, d.refine_steps, d.chunk, d.chunk_upper, d.block, d.max_blocks = 1, -1, 0, 0, 0, 0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value", [("order", 0), ("order", 5), ("n_init", 4), ("n_init", -1),
                                         ("n_inst", 0), ("steps_uniform", 0), ("mode", 3), ("refine_steps", 5),
                                         ("block", 96), ("block", 512), ("max_blocks", -1),
                                         ("init_points", -1), ("init_points", 1 << 29)])
def test_invalid_plan_descriptions_rejected_on_host(field, value):
    L = _lib()
    lib = L.lib()
    h = ctypes.c_void_p()
    st = lib.smnn_plan_create(ctypes.byref(_desc(**{field: value})), ctypes.byref(h))
    assert st == 1 and not h.value


def test_unsupported_chunk_rejected():
    L = _lib()
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.smnn_plan_create(ctypes.byref(_desc(chunk=7)), ctypes.byref(h)) == 2


def test_null_arguments_rejected():
    L = _lib()
    lib = L.lib()
    assert lib.smnn_plan_create(None, None) == 1
    assert lib.smnn_plan_destroy(None) == 1
    assert lib.smnn_plan_sizes(None, None, None, None) == 1
    assert lib.smnn_plan_query(None, 1) == -1
    fwd = [None] * 8 + [0, None, 0, None, None]
    assert lib.smnn_forward(*fwd) == 1
    bwd = [None] * 8 + [0] + [None] * 7 + [0, None, None]
    assert lib.smnn_backward(*bwd) == 1
    assert lib.smnn_autotune(None, None, None, None, None, None, None, 1, None, None, None, 0, None) == 1
    assert lib.smnn_trace_enable(None, 4) == 1
    assert lib.smnn_trace_read(None, None, 0) == -1


def test_levels_geometry_matches_partition_rule():
    # The partition (smnn_levels.h): chunks of L nodes, separators are the last
    # node of every chunk but an instance's last, and become the next level.
    def levels(T, L, Lu=None):
        out, n = [], list(T)
        while True:
            Lc = L if not out or Lu is None else Lu
            g = [(x + Lc - 1) // Lc for x in n]
            out.append((sum(n), sum(g)))
            nxt = [gi - 1 if x > Lc else 0 for x, gi in zip(n, g)]
            if not any(nxt):
                return out
            n = nxt
    assert levels([10000], 8) == [(10000, 1250), (1249, 157), (156, 20), (19, 3), (2, 1)]
    assert levels([1, 8, 9], 8) == [(18, 4), (1, 1)]
    assert levels([10000], 4, 8) == [(10000, 2500), (2499, 313), (312, 39), (38, 5), (4, 1)]
