"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function that include/tild.h declares, and rejects invalid arguments
before touching a device."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2302_02474_amd as T
from paper_2302_02474_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "tild.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tild_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtild.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_and_binding_agree():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_kernel_slot_names(lib):
    names = [lib.tild_kernel_name(i) for i in range(_lib.TILD_NUM_KERNELS)]
    assert all(n for n in names)
    assert lib.tild_kernel_name(_lib.TILD_NUM_KERNELS) is None
    assert lib.tild_kernel_name(-1) is None


def test_params_struct_layout(tmp_path):
    """The ctypes mirror of tild_params matches the header's layout, as a C compiler lays it out."""
    fields = [f for f, _ in _lib.TildParams._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"tild.h\"\nint main(void) {\n"
                   '  printf("%zu\\n", sizeof(tild_params));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(tild_params, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(_lib.TildParams)
    assert got[1:] == [getattr(_lib.TildParams, f).offset for f in fields]


def _create(lib, params, n=4, types=None, bonds=None):
    types = np.zeros(n, np.int32) if types is None else np.asarray(types, np.int32)
    bonds = np.zeros((0, 2), np.int32) if bonds is None else np.asarray(bonds, np.int32)
    ctx = ctypes.c_void_p(None)
    rc = lib.tild_create(ctypes.byref(params), int(types.shape[0]), types.ctypes.data, int(bonds.shape[0]),
                         bonds.ctypes.data if bonds.size else None, None, 0, None, ctypes.byref(ctx))
    return rc, ctx, lib.tild_last_error(None).decode()


def good():
    return T.make_params((5, 5, 5), (16, 16, 16), 4, 0.5, 0.5, 5.0)


@pytest.mark.parametrize("mutate,needle", [
    (lambda p: setattr(p, "order", 0), "order"),
    (lambda p: setattr(p, "order", 8), "order"),
    (lambda p: p.grid.__setitem__(0, 7), "grid"),
    (lambda p: p.grid.__setitem__(1, 512), "grid"),
    (lambda p: p.grid.__setitem__(2, 1), "grid"),
    (lambda p: p.box.__setitem__(1, 0.0), "box"),
    (lambda p: p.box.__setitem__(2, float("nan")), "box"),
    (lambda p: setattr(p, "dt", -1.0), "dt"),
    (lambda p: setattr(p, "gamma", 0.0), "gamma"),
    (lambda p: setattr(p, "kT", -1.0), "kT"),
    (lambda p: setattr(p, "precision", 3), "precision"),
    (lambda p: setattr(p, "flags", 32), "flag"),
    (lambda p: (setattr(p, "flags", _lib.TILD_INTEGRATOR_GJF), setattr(p, "mass", -1.0)), "mass"),
    (lambda p: (setattr(p, "flags", _lib.TILD_INTEGRATOR_GJF), setattr(p, "mass", float("nan"))), "mass"),
    (lambda p: setattr(p, "bjerrum", -1.0), "bjerrum"),
    (lambda p: setattr(p, "charge_smear", float("inf")), "charge_smear"),
    (lambda p: p.charge.__setitem__(1, float("nan")), "charge"),
    (lambda p: setattr(p, "smear_a", float("inf")), "smear_a"),
    (lambda p: (setattr(p, "smear_a", 0.0), setattr(p, "flags", _lib.TILD_POTENTIAL_SAMPLED)), "smear_a"),
    (lambda p: (setattr(p, "order", 1), setattr(p, "flags", _lib.TILD_FORCE_AD)), "order"),
])
def test_create_rejects_bad_params(lib, mutate, needle):
    p = good()
    mutate(p)
    rc, ctx, msg = _create(lib, p)
    assert rc == _lib.TILD_EINVAL
    assert ctx.value is None
    assert needle in msg


def test_create_rejects_bad_types_and_bonds(lib):
    rc, _, msg = _create(lib, good(), types=[0, 1, 2, 0])
    assert rc == _lib.TILD_EINVAL and "types" in msg
    rc, _, msg = _create(lib, good(), bonds=[[0, 4]])
    assert rc == _lib.TILD_EINVAL and "bond" in msg
    rc, _, msg = _create(lib, good(), bonds=[[2, 2]])
    assert rc == _lib.TILD_EINVAL and "bond" in msg
    rc, _, msg = _create(lib, good(), bonds=[[-1, 0]])
    assert rc == _lib.TILD_EINVAL


def test_create_rejects_plane_too_large_for_fp64(lib):
    p = T.make_params((50, 50, 50), (192, 192, 192), 5, 0.5, 0.05, 20.0, precision=T.TILD_FP64)
    rc, _, msg = _create(lib, p)
    assert rc == _lib.TILD_EINVAL and "LDS" in msg


def test_null_context_calls(lib):
    assert lib.tild_step(None, 1) == _lib.TILD_EINVAL
    assert lib.tild_synchronize(None) == _lib.TILD_EINVAL
    assert lib.tild_step_count(None) == -1
    lib.tild_destroy(None)
    out = ctypes.c_void_p(None)
    assert lib.tild_create(None, 4, None, 0, None, None, 0, None, ctypes.byref(out)) == _lib.TILD_EINVAL


def test_create_rejects_misaligned_workspace(lib):
    types = np.zeros(4, np.int32)
    ctx = ctypes.c_void_p(None)
    rc = lib.tild_create(ctypes.byref(good()), 4, types.ctypes.data, 0, None, ctypes.c_void_p(0x1000 + 16), 1 << 30,
                         None, ctypes.byref(ctx))
    assert rc == _lib.TILD_EINVAL and "aligned" in lib.tild_last_error(None).decode()
    assert ctx.value is None


def test_workspace_bytes(lib):
    # no device needed: the layout is computed on the host
    p = good()
    b0 = T.workspace_bytes(p, 1000)
    assert b0 > 0
    chain = np.stack([np.arange(999), np.arange(1, 1000)], axis=1)
    b1 = T.workspace_bytes(p, 1000, chain)
    assert b1 > b0  # partner tables
    assert T.workspace_bytes(p, 2000, chain) > b1
    p64 = T.make_params((5, 5, 5), (16, 16, 16), 4, 0.5, 0.5, 5.0, precision=T.TILD_FP64)
    assert T.workspace_bytes(p64, 1000, chain) > b1
    bad = good()
    bad.order = 0
    assert T.workspace_bytes(bad, 1000) == 0
    assert "order" in lib.tild_last_error(None).decode()
    assert T.workspace_bytes(p, 1000, np.array([[0, 1000]])) == 0


def test_batch_create_rejects_bad_arguments(lib):
    out = ctypes.c_void_p(None)
    assert lib.tild_batch_create(None, 1, None, ctypes.byref(out)) == _lib.TILD_EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.tild_batch_create(arr, 1, None, ctypes.byref(out)) == _lib.TILD_EINVAL
    assert "NULL" in lib.tild_batch_last_error(None).decode()
    assert lib.tild_batch_create(arr, 0, None, ctypes.byref(out)) == _lib.TILD_EINVAL
    assert out.value is None
    assert lib.tild_batch_step(None, 1) == _lib.TILD_EINVAL
    lib.tild_batch_destroy(None)
