"""CPU checks of the C ABI: the library loads, exports every declared entry
point, the ctypes mirrors match the C structs, and argument validation fails
cleanly without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2101_05917_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diffpd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpd_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.PROTOTYPES, n


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    fields = {"dpd_options": L.Options, "dpd_stats": L.Stats, "dpd_mesh_info": L.MeshInfo,
              "dpd_kernel_profile": L.KernelProfile, "dpd_request": L.Request,
              "dpd_result": L.Result, "dpd_batch_stats": L.BatchStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.split("\n") if l)
    for cname, cls in fields.items():
        assert int(out[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_default_options_and_status_strings():
    lib = L.load()
    o = L.Options()
    assert lib.dpd_default_options(C.byref(o)) == 0
    assert o.dx == 0.01 and o.nu == 0.45 and o.gravity[2] == -9.81 and o.fwd_max_iter == 100
    for code in L.STATUS_NAMES:
        assert lib.dpd_status_string(code)


@pytest.mark.parametrize("case", ["dup", "nu", "youngs", "fixed", "empty"])
def test_create_mesh_rejects_bad_input_without_gpu(case):
    lib = L.load()
    o = L.Options()
    lib.dpd_default_options(C.byref(o))
    cells = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    ym = np.array([1e6, 1e6])
    fixed = np.zeros((0, 3), np.int32)
    n = 2
    if case == "dup":
        cells = np.array([[0, 0, 0], [0, 0, 0]], np.int32)
    elif case == "nu":
        o.nu = 0.5
    elif case == "youngs":
        ym = np.array([1e6, -1.0])
    elif case == "fixed":
        fixed = np.array([[9, 9, 9]], np.int32)
    elif case == "empty":
        n = 0
    h = C.c_void_p()
    code = lib.dpd_create_mesh(cells.ctypes.data_as(L._I32), n, ym.ctypes.data_as(L._D),
                               fixed.ctypes.data_as(L._I32) if len(fixed) else None, len(fixed),
                               C.byref(o), C.byref(h))
    assert code == -1 and not h.value
    assert lib.dpd_last_error(None)


@pytest.mark.parametrize("case", ["range", "flat", "youngs", "fixed", "muscle", "volume", "orphan"])
def test_create_tet_mesh_rejects_bad_input_without_gpu(case):
    lib = L.load()
    o = L.Options()
    lib.dpd_default_options(C.byref(o))
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], np.float64) * 0.01
    T = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)
    ym = np.array([1e6, 1e6])
    fixed = np.zeros(0, np.int32)
    if case == "range":
        T[1, 3] = 5
    elif case == "flat":
        X[3] = [0.005, 0.005, 0.0]    # all four corners of the first in one plane
    elif case == "youngs":
        ym[1] = 0.0
    elif case == "fixed":
        fixed = np.array([7], np.int32)
    elif case == "muscle":
        o.muscle_k = 1e5
    elif case == "volume":
        o.volume_scale = 1.0
    elif case == "orphan":
        X = np.vstack([X, [[0.05, 0.05, 0.05]]])
    h = C.c_void_p()
    code = lib.dpd_create_tet_mesh(X.ctypes.data_as(L._D), len(X), T.ctypes.data_as(L._I32), len(T),
                                   ym.ctypes.data_as(L._D), fixed.ctypes.data_as(L._I32) if len(fixed) else None,
                                   len(fixed), C.byref(o), C.byref(h))
    assert code == -1 and not h.value
    assert lib.dpd_last_error(None)


def test_null_handles_are_rejected():
    lib = L.load()
    st = L.Stats()
    assert lib.dpd_forward_step(None, None, None, None, None, None, None, C.byref(st)) == -1
    assert lib.dpd_factorize(None, None) == -1
    assert lib.dpd_profile_start(None, 1) == -1
