"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grrmhd.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(grrmhd_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1312_6127_amd import grrmhd as G

    if not os.path.exists(G.LIBPATH):
        import __graft_entry__

        __graft_entry__.build()
    return G.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n


def test_default_params_match_binding_defaults(L):
    from paper_1312_6127_amd import grrmhd as G
    from paper_1312_6127_amd import inputs as I

    p = G.Params()
    L.grrmhd_default_params(C.byref(p))
    q = G.params(I.default_params())
    for name, _ in G.Params._fields_:
        a, b = getattr(p, name), getattr(q, name)
        if hasattr(a, "__len__"):
            assert list(a) == list(b), name
        elif name not in ("rho_floor", "u_floor"):
            assert a == b, name


def test_invalid_parameters_are_rejected_before_any_device_work(L):
    from paper_1312_6127_amd import grrmhd as G
    from paper_1312_6127_amd import inputs as I

    bad = [dict(gam=1.0), dict(ng=3, n=(8, 1, 1)), dict(n=(0, 1, 1)), dict(max_iter=0),
           dict(metric="ks", a=1.5, n=(8, 8, 1)), dict(bc_lo=("polar", "periodic", "periodic"))]
    for kw in bad:
        p = G.params(I.default_params(**kw))
        h = C.c_void_p()
        rc = L.grrmhd_init_grid(C.byref(p), 0, None, C.byref(h))
        assert rc == -1, kw
        assert L.grrmhd_last_error()
    p = G.params(I.default_params(metric="ks"))
    assert L.grrmhd_implicit_source(C.byref(p), 10, *([None] * 11), 0, None) == -1
    p = G.params(I.default_params())
    assert L.grrmhd_implicit_source(C.byref(p), 0, *([None] * 11), 0, None) == 0
    assert L.grrmhd_step(None, *([None] * 5), 0, None, None, None, 0) == -1
    # execution forms: bad mode, block and workspace are refused on the host
    ex = L.grrmhd_implicit_source_ex
    args = [C.c_void_p(256)] * 10
    assert ex(C.byref(p), 10, *args, 7, 64, 4, C.c_void_p(256), 1 << 20, None) == -1
    assert b"mode" in L.grrmhd_last_error()
    assert ex(C.byref(p), 10, *args, G.PERSISTENT, 64, 4, C.c_void_p(256), 16, None) == -1
    assert b"workspace" in L.grrmhd_last_error()
    assert ex(C.byref(p), 10, *args, G.PERSISTENT, 64, 4, C.c_void_p(260), 1 << 20, None) == -1
    assert ex(C.byref(p), 0, *([None] * 10), G.PERSISTENT, 64, 4, None, 0, None) == 0
    t = G.Tuning()
    assert L.grrmhd_autotune_implicit_source(C.byref(p), 0, *([None] * 11), 0, None,
                                              C.byref(t), None, 0) == -1
    out = (C.c_ulonglong * 3)()
    assert L.grrmhd_implicit_stats(None, out) == -1
    assert L.grrmhd_implicit_source_stats(C.c_void_p(260), out, None) == -1
    assert L.grrmhd_implicit_source_cascade_stats(C.c_void_p(260), out, None) == -1
    assert L.grrmhd_implicit_source_cascade_stats(None, out, None) == -1


def test_batch_workspace_sizes(L):
    from paper_1312_6127_amd import grrmhd as G

    f = L.grrmhd_implicit_source_workspace_bytes_ex
    assert f(0, G.PER_CELL) == 0
    for n in (1, 63, 64, 1000, 1 << 24):
        a, b, c = f(n, G.PER_CELL), f(n, G.PERSISTENT), f(n, G.PER_ITERATION)
        assert a == b == L.grrmhd_implicit_source_workspace_bytes(n)
        # list, first-attempt record (13 doubles, 3 ints), deferred and cold lists per cell
        assert a >= 256 + 4 * n + 13 * 8 * n + 3 * 4 * n + 2 * 4 * n and a % 256 == 0
        # two queues, 47 doubles and 8 ints of lane state per cell
        assert c >= a + 8 * n + 47 * 8 * n + 8 * 4 * n
