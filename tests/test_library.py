"""Host-side checks of the C-ABI library (no GPU calls)."""

import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_1011_5964_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "tvdeblur.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(tvdeblur_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert header_symbols() == sorted(L.EXPORTED_SYMBOLS)


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_library_loads_and_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name


STRUCTS = {"tvd_params": L.Params, "tvd_stats": L.Stats, "tvd_kernel_times": L.KernelTimes,
           "tvd_image_desc": L.ImageDesc, "tvd_batch_params": L.BatchParams, "tvd_batch_info": L.BatchInfo,
           "tvd_signal_desc": L.SignalDesc, "tvd_signal_params": L.SignalParams}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_struct_layouts_match_header(tmp_path):
    """Every binding struct has the size and field offsets that a C compiler
    gives the header's declaration."""
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tvdeblur.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_null_handle_errors_without_gpu():
    lib = L.load()
    assert lib.tvdeblur_set_bc(None, 2) == -1
    assert lib.tvdeblur_destroy(None) == 0
    assert lib.tvdeblur_last_error(None) is not None
    assert lib.tvdeblur_batch_destroy(None) == 0
    assert lib.tvdeblur_batch_get_info(None, None) == -1
    assert lib.tvdeblur_batch_last_error(None) is not None


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_batch_create_argument_errors_without_gpu():
    """Argument checks of batch creation run before any device call."""
    lib = L.load()
    out = ctypes.c_void_p()
    assert lib.tvdeblur_batch_create(None, 1, None, 1, 2, None) == -1
    assert lib.tvdeblur_batch_create(ctypes.byref(out), 0, None, 1, 2, None) == -1
    import numpy as np
    h = np.zeros((3, 3))
    h[1, 1] = 1.0
    d = (L.ImageDesc * 1)(L.ImageDesc(2, 8, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3, 3))
    assert lib.tvdeblur_batch_create(ctypes.byref(out), 1, d, 1, 2, None) == -4          # too small
    d[0].ny = 8
    assert lib.tvdeblur_batch_create(ctypes.byref(out), 1, d, 7, 2, None) == -1          # bad precision
    assert lib.tvdeblur_batch_create(ctypes.byref(out), 1, d, 1, 9, None) == -1          # bad BC
    hb = np.full((3, 3), 1.0 / 9)
    hb[0, 0] += 1e-3
    hb /= hb.sum()
    d[0].psf_host = hb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.tvdeblur_batch_create(ctypes.byref(out), 1, d, 1, 2, None) == -2          # not symmetric
    assert b"image 0" in lib.tvdeblur_batch_last_error(None)


def test_alpha_sweep_rejects_bad_alphas_without_gpu():
    """The alpha list is checked before any device call."""
    for bad in ([], [1e-3, 0.0], [1e-3, -1e-3], [float("nan")], [float("inf")]):
        with pytest.raises(ValueError):
            L.AlphaSweep((16, 16), [[1.0]], "antireflective", bad)


def test_preconditioner_maps_match_header():
    """The binding's names map onto the header's TVD_PREC_* values (the
    reblurring names reuse the same slots: I, D, P, D_P, P_D)."""
    with open(os.path.join(ROOT, "include", "tvdeblur.h")) as f:
        defs = dict(re.findall(r"#define (TVD_PREC_[A-Z_]+)\s+(\d+)", f.read()))
    c = {k: int(v) for k, v in defs.items()}
    assert L.PRECOND == {"none": c["TVD_PREC_NONE"], "diag": c["TVD_PREC_DIAG"], "x": c["TVD_PREC_X"],
                         "d_x": c["TVD_PREC_D_X"], "x_d": c["TVD_PREC_X_D"]}
    assert L.REBLUR_PRECOND == {"none": c["TVD_PREC_NONE"], "diag": c["TVD_PREC_DIAG"], "p": c["TVD_PREC_X"],
                                "d_p": c["TVD_PREC_D_X"], "p_d": c["TVD_PREC_X_D"]}


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_reblur_entry_points_reject_null_without_gpu():
    lib = L.load()
    assert lib.tvdeblur_solve_reblur(None, None, None, None, None) == -1
    assert lib.tvdeblur_op_reblur_setup(None, None, 1e-3, 0.1, 4) == -1
    assert lib.tvdeblur_op_reblur_normal(None, None, None) == -1
    assert lib.tvdeblur_op_reblur_precond(None, None, None) == -1
    assert b"NULL" in lib.tvdeblur_last_error(None)


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_signals_and_noalloc_argument_errors_without_gpu():
    """Argument checks of the 1D signal and allocation-free entry points run
    before any device call."""
    lib = L.load()
    out = ctypes.c_void_p()
    h = np.full(5, 0.2)
    hp = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def descs(*rows):
        arr = (L.SignalDesc * len(rows))()
        for k, (n, plen, bc, ptr) in enumerate(rows):
            arr[k].n, arr[k].plen, arr[k].bc, arr[k].psf_host = n, plen, bc, ptr
        return arr

    assert lib.tvdeblur_signals_create(ctypes.byref(out), 0, descs((10, 5, 2, hp)), None) == -1
    assert lib.tvdeblur_signals_create(ctypes.byref(out), 1, descs((2, 5, 2, hp)), None) == -4
    assert lib.tvdeblur_signals_create(ctypes.byref(out), 1, descs((10, 5, 7, hp)), None) == -1
    assert lib.tvdeblur_signals_create(ctypes.byref(out), 1, descs((8, 5, 4, hp)), None) == -4  # 4m+1 > n
    bad = np.array([0.1, 0.2, 0.4, 0.2, 0.1]) * 1.5
    bp = bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.tvdeblur_signals_create(ctypes.byref(out), 1, descs((10, 5, 1, bp)), None) == -3
    skew = np.array([0.1, 0.2, 0.4, 0.25, 0.05])
    sp = skew.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.tvdeblur_signals_create(ctypes.byref(out), 1, descs((10, 5, 1, sp)), None) == -2
    assert b"signal 0" in lib.tvdeblur_signals_last_error(None)
    assert lib.tvdeblur_signals_solve(None, None, None, None, None) == -1
    assert lib.tvdeblur_solve_noalloc(None, None, None, None, None) == -1


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_workspace_argument_errors_without_gpu():
    """The caller-workspace entry points reject a NULL handle before any
    device call."""
    lib = L.load()
    n = ctypes.c_size_t(0)
    assert lib.tvdeblur_workspace_bytes(None, ctypes.byref(n)) == -1
    assert lib.tvdeblur_set_workspace(None, None, 0) == -1
