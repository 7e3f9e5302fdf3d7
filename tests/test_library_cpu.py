"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function declared in include/grprec.h, and rejects invalid problems
before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grprec.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grprec_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def G():
    from paper_2602_21911_amd import build, grprec
    if not os.path.exists(grprec.LIB_PATH):
        build.build()
    return grprec


def test_exports_every_declared_symbol(G):
    names = _declared()
    assert len(names) >= 20
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(G.EXPORTED) == names


def _problem(G, **kw):
    cells = np.array(kw.pop("cells", [100]), dtype=np.int64)
    lengths = np.array(kw.pop("lengths", [1.0] * len(cells)), dtype=np.float64)
    base = dict(system=G.GRPREC_EULER, order=3, cfl=0.9, lam=1.0, gamma=1.4,
                bc=G.GRPREC_BC_TRANSMISSIVE, guess=0, schedule=1, block=128)
    base.update(kw)
    p = G.grprec_problem(base["system"], base["order"], base["cfl"], base["lam"], base["gamma"],
                         base["bc"], len(cells),
                         cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         lengths.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         base["guess"], 0, 0.0, 0, 0.0, None, 0.0, 0, base["schedule"], base["block"])
    return p, (cells, lengths)


def test_workspace_bytes_valid_and_invalid(G):
    p, keep = _problem(G)
    assert G.grprec_workspace_bytes(p) > 0
    for bad in (dict(cfl=1.05), dict(cfl=0.0), dict(order=6), dict(order=1), dict(gamma=1.0),
                dict(system=7), dict(bc=5), dict(cells=[100, 1]),
                dict(bc=G.GRPREC_BC_PERIODIC, cells=[10, 10]),
                dict(system=G.GRPREC_ADVECTION, lam=0.0),
                # 32-bit indexing limit: cells + segments <= INT_MAX / 3
                dict(cells=[400_000_000, 400_000_000])):
        p, keep = _problem(G, **bad)
        assert G.grprec_workspace_bytes(p) == 0, bad


def test_workspace_grows_with_autotune_snapshot(G):
    p1, k1 = _problem(G, cells=[1000] * 4, schedule=1)
    p0, k0 = _problem(G, cells=[1000] * 4, schedule=0)
    assert G.grprec_workspace_bytes(p0) > G.grprec_workspace_bytes(p1)


def test_error_strings(G):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert len(G.grprec_error_string(code)) >= 2
    assert G.grprec_error_string(-99) == "unknown error"


def test_init_rejects_null_buffers_without_gpu(G):
    p, keep = _problem(G)
    b = G.grprec_buffers(None, None, None, None, None, 0)
    h = ctypes.c_void_p()
    rc = G.lib().grprec_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(b), None)
    assert rc == G.GRPREC_E_INVALID and not h.value
