"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, agrees with the header on the parameter layout, and rejects bad input
before touching a device."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_2601_10057_amd import ccmsav as C
from workloads import circle_member

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccmsav.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccmsav_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = C.load()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(C.EXPORTED)


def test_params_layout_matches_the_header(tmp_path):
    fields = [f for f, _ in C.Params._fields_]
    src = tmp_path / "layout.c"
    body = "\n".join(f'  printf("%zu\\n", offsetof(ccmsav_params, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ccmsav.h"\nint main(void){\n'
                   f'  printf("%zu\\n", sizeof(ccmsav_params));\n{body}\n  return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(C.Params)
    for f, off in zip(fields, out[1:]):
        assert getattr(C.Params, f).offset == off, f


def _params(**kw):
    p = dict(circle_member(64).params)
    p.update(kw)
    return C.Params.from_dict(p)


def test_workspace_size_and_validation():
    lib = C.load()
    good = _params()
    n = lib.ccmsav_workspace_bytes(ctypes.byref(good))
    cells = 64 * 64
    assert n >= (6 + 8 + 2) * cells * 8
    assert lib.ccmsav_workspace_bytes(ctypes.byref(_params(nx=100))) == 0
    assert lib.ccmsav_workspace_bytes(ctypes.byref(_params(dt=-1.0))) == 0
    mixed = C.Params.from_dict(circle_member(64).params, C.MIXED)
    assert lib.ccmsav_workspace_bytes(ctypes.byref(mixed)) < n


@pytest.mark.parametrize("kw,code", [
    (dict(nx=100), -6), (dict(ny=8), -6), (dict(nx=16384), -6), (dict(dt=0.0), -1),
    (dict(eps=math.nan), -1), (dict(M0=1.0), -1), (dict(gamma_in=-1.0), -1),
    (dict(h=math.inf), -1), (dict(A=math.inf), -1), (dict(lam=-2.0), -1),
])
def test_init_rejects_bad_parameters_without_a_device(kw, code):
    lib = C.load()
    p = _params(**kw)
    h = ctypes.c_void_p()
    buf = (ctypes.c_double * 4)()
    assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(p), buf, buf, None, 0, None) == code
    assert h.value is None


def test_init_rejects_null_and_unknown_modes():
    lib = C.load()
    p = _params()
    h = ctypes.c_void_p()
    assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(p), None, None, None, 0, None) == -1
    p.precision = 7
    buf = (ctypes.c_double * 4)()
    assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(p), buf, buf, None, 0, None) == -6
    p.precision = 0
    p.flags = 32         # no such flag
    assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(p), buf, buf, None, 0, None) == -1
    # the periodic step: FP64 only, no graph, grids up to 4096, one member
    for prec, flags, n in ((C.MIXED, C.FLAG_PERIODIC, 64), (C.FP64, C.FLAG_PERIODIC | C.FLAG_GRAPH, 64),
                           (C.FP64, C.FLAG_PERIODIC, 8192)):
        q = _params(nx=n, ny=n)
        q.precision, q.flags = prec, flags
        assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(q), buf, buf, None, 0, None) == -6
        assert lib.ccmsav_workspace_bytes(ctypes.byref(q)) == 0
    q = _params()
    q.flags = C.FLAG_PERIODIC
    assert lib.ccmsav_workspace_bytes(ctypes.byref(q)) > lib.ccmsav_workspace_bytes(ctypes.byref(p))
    pair = (C.Params * 2)(q, q)
    assert lib.ccmsav_workspace_bytes_batch(2, pair) == 0
    # the classical scheme: FP64 only, Neumann, no graph, one member
    for prec, flags in ((C.MIXED, C.FLAG_CLASSICAL), (C.FP64, C.FLAG_CLASSICAL | C.FLAG_GRAPH),
                        (C.FP64, C.FLAG_CLASSICAL | C.FLAG_PERIODIC)):
        q = _params()
        q.precision, q.flags = prec, flags
        assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(q), buf, buf, None, 0, None) == -6
    q = _params()
    q.flags = C.FLAG_CLASSICAL
    assert lib.ccmsav_workspace_bytes(ctypes.byref(q)) > lib.ccmsav_workspace_bytes(ctypes.byref(p))
    assert lib.ccmsav_workspace_bytes_batch(2, (C.Params * 2)(q, q)) == 0
    assert lib.ccmsav_pcg_config(None, 1e-10, 10) == -1
    assert C.strerror(-7).startswith("an iterative solve")
    # the persistent launch: FP32 transforms, CC-MSAV with Neumann boundaries,
    # grids of 64 to 512 per direction
    for prec, flags, n in ((C.FP64, C.FLAG_PERSISTENT, 64),
                           (C.MIXED, C.FLAG_PERSISTENT | C.FLAG_PERIODIC, 64),
                           (C.MIXED_GEMM_BF16X3, C.FLAG_PERSISTENT, 64),
                           (C.MIXED, C.FLAG_PERSISTENT, 32), (C.MIXED, C.FLAG_PERSISTENT, 1024)):
        q = _params(nx=n, ny=n)
        q.precision, q.flags = prec, flags
        assert lib.ccmsav_init(ctypes.byref(h), ctypes.byref(q), buf, buf, None, 0, None) == -6
        assert lib.ccmsav_workspace_bytes(ctypes.byref(q)) == 0
    q = _params(nx=64, ny=128)
    q.precision, q.flags = C.MIXED, C.FLAG_PERSISTENT | C.FLAG_GRAPH | C.FLAG_BDF1
    assert lib.ccmsav_workspace_bytes(ctypes.byref(q)) > 0
    assert lib.ccmsav_set_spin_limit(None, 0) == -1
    assert C.strerror(-8).startswith("a grid barrier")
    assert lib.ccmsav_step(None, 1) == -1
    assert lib.ccmsav_destroy(None) == -1
    assert C.strerror(-6).startswith("unsupported")
    assert C.strerror(5) == "unknown status"
    assert C.strerror(-9) == "unknown status"


def test_batch_workspace_and_validation_without_a_device():
    lib = C.load()
    a, b = _params(), _params(nx=32, ny=128, eps=0.3)
    arr = (C.Params * 2)(a, b)
    one = lib.ccmsav_workspace_bytes(ctypes.byref(a))
    two = lib.ccmsav_workspace_bytes_batch(2, arr)
    assert two > one + (6 + 8 + 2) * 32 * 128 * 8
    assert lib.ccmsav_workspace_bytes_batch(0, arr) == 0
    bad = (C.Params * 2)(a, _params(nx=100))
    assert lib.ccmsav_workspace_bytes_batch(2, bad) == 0
    h = ctypes.c_void_p()
    buf = (ctypes.c_double * 4)()
    ptrs = (ctypes.c_void_p * 2)(ctypes.addressof(buf), ctypes.addressof(buf))
    # member count out of range, mixed precisions, mixed flags, a NULL field
    assert lib.ccmsav_init_batch(ctypes.byref(h), 0, arr, ptrs, ptrs, None, 0, None) == -1
    mixed = (C.Params * 2)(a, C.Params.from_dict(dict(circle_member(64).params), C.MIXED))
    assert lib.ccmsav_init_batch(ctypes.byref(h), 2, mixed, ptrs, ptrs, None, 0, None) == -1
    flagged = (C.Params * 2)(a, C.Params.from_dict(dict(circle_member(64).params), 0,
                                                   C.FLAG_GRAPH))
    assert lib.ccmsav_init_batch(ctypes.byref(h), 2, flagged, ptrs, ptrs, None, 0, None) == -1
    nulls = (ctypes.c_void_p * 2)(ctypes.addressof(buf), None)
    assert lib.ccmsav_init_batch(ctypes.byref(h), 2, arr, ptrs, nulls, None, 0, None) == -1
    assert h.value is None
    assert lib.ccmsav_members(None) == -1
    e = ctypes.c_double()
    assert lib.ccmsav_energy_m(None, 0, ctypes.byref(e), None) == -1
