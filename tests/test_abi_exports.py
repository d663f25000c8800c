"""The C-ABI library loads and exports every function include/qtx_rgf.h declares
(no GPU needed: only dlopen + symbol lookup, no compute call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtx_rgf.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qtx_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("qtx_rgf_create", "qtx_rgf_solve", "qtx_rgf_destroy"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_2606_25595_amd import qtx
    if not os.path.exists(qtx.LIB_PATH):
        pytest.fail("libqtx_rgf.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(qtx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(qtx.EXPORTED)


def test_status_strings_without_gpu():
    from paper_2606_25595_amd import qtx
    assert qtx.status_str(qtx.QTX_OK) == "QTX_OK"
    assert qtx.status_str(qtx.QTX_ERR_SINGULAR) == "QTX_ERR_SINGULAR"


def test_problem_struct_layout_matches_header(tmp_path):
    """The binding's qtx_rgf_problem has the header's size and field offsets (gcc
    compiles a probe of the header; no GPU, no library call)."""
    import shutil
    import subprocess
    from paper_2606_25595_amd import qtx
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    fields = [f[0] for f in qtx._Problem._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qtx_rgf.h"', "int main(void) {",
             '  printf("%zu\\n", sizeof(qtx_rgf_problem));']
    lines += ['  printf("%%zu\\n", offsetof(qtx_rgf_problem, %s));' % f for f in fields]
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(qtx._Problem)
    for f, off in zip(fields, vals[1:]):
        assert getattr(qtx._Problem, f).offset == off, f


def test_sigma_diag_takes_only_diagonal_blocks():
    """to_device(sigma_diag=True) sends the diagonals and refuses a block with an
    off-diagonal entry (a NaN on the diagonal is not one)."""
    import numpy as np
    from paper_2606_25595_amd import inputs, qtx
    p = inputs.random_bt_problem(3, 8, [0.1, 0.2], seed=1)
    p.SL_d = p.SL_d.copy()
    p.SL_d[1, 1, 4, 4] = np.nan
    dp = qtx.to_device(p, device="cpu", sigma_diag=True)
    assert tuple(dp.SR_d.shape) == (2, 3, 8) and tuple(dp.SL_d.shape) == (2, 3, 8)
    assert np.array_equal(dp.SR_d.numpy(), np.diagonal(p.SR_d, axis1=-2, axis2=-1))
    p.SR_d = p.SR_d.copy()
    p.SR_d[0, 1, 2, 3] = 0.1
    with pytest.raises(ValueError):
        qtx.to_device(p, device="cpu", sigma_diag=True)
    dp = qtx.to_device(p, device="cpu", out_bits=24)
    assert dp.GR_u.dtype.is_floating_point is False and tuple(dp.GR_u.shape) == (2, 2, 8 * 8 * 24 // 4)
