"""Host-side checks of the C ABI: the library loads, exports every function
that include/dugks.h declares, and its GPU-free calls behave."""
import os
import re
import subprocess

import pytest

import paper_1810_07802_amd as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dugks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dugks_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = _declared()
    assert "dugks_create" in names and "dugks_step" in names and "dugks_destroy" in names
    out = subprocess.run(["nm", "-D", "--defined-only", D.build.LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (dugks_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = D.lib()
    for n in names:
        assert hasattr(L, n)


def test_footprint_matches_layout():
    # coupled: 21 values (9 f + 9 g + 2 history + phi) per cell, AC-only 12;
    # a state buffer is ny rows of nx cells, each row padded to 128 bytes;
    # two buffers
    def row(nx, nv, e):
        return -(-nx * nv * e // 128) * 128
    fp = D.footprint_bytes(1000, 700, D.FP32, D.MODEL_COUPLED)
    assert row(1000, 21, 4) == 84096
    assert 2 * 700 * row(1000, 21, 4) <= fp < 2 * 700 * row(1000, 21, 4) + 4096
    fp = D.footprint_bytes(1000, 700, D.FP64, D.MODEL_AC)
    assert 2 * 700 * row(1000, 12, 8) <= fp < 2 * 700 * row(1000, 12, 8) + 4096
    # rows of whole cache lines add nothing
    fp = D.footprint_bytes(4096, 64, D.FP32, D.MODEL_COUPLED)
    assert 2 * 21 * 4096 * 64 * 4 <= fp < 2 * 21 * 4096 * 64 * 4 + 4096


def test_null_and_bad_arguments_do_not_crash():
    L = D.lib()
    assert L.dugks_destroy(None) == 0
    assert L.dugks_step(None, 1) == D.EINVAL
    assert L.dugks_last_error(None) is not None
    with pytest.raises(D.DugksError) as e:
        D.create(2, 16)
    assert e.value.code == D.EINVAL
    with pytest.raises(D.DugksError) as e:
        D.create(16, 16, precision=7)
    assert e.value.code == D.EINVAL
    assert L.dugks_autotune(None, 10, None, None) == D.EINVAL
    # an empty batch is rejected before any device work
    with pytest.raises(D.DugksError) as e:
        D.Batch([])
    assert e.value.code == D.EINVAL
    # batch constructors and case access check their arguments first
    import ctypes as C
    b = C.c_void_p()
    assert L.dugks_batch_create(0, None, None, D.FP32, D.MODEL_COUPLED, C.byref(b)) == D.EINVAL
    nx = (C.c_int * 1)(2)
    assert L.dugks_batch_create(1, nx, nx, D.FP32, D.MODEL_COUPLED, C.byref(b)) == D.EINVAL
    assert L.dugks_batch_case(None, 0) is None
    assert L.dugks_batch_create_from(1, None, C.byref(b)) == D.EINVAL
    # pool calls on a NULL pool
    slot = C.c_int(-1)
    assert L.dugks_pool_admit_handle(None, None, 10, C.byref(slot)) == D.EINVAL
    assert L.dugks_pool_status(None, 0) == D.EINVAL
    # size limit of the C ABI: at most 2^28 cells in FP32 and 2^27 in FP64
    # (rejected before any device allocation)
    for nx, ny, prec in ((1 << 15, 1 << 14, D.FP32), (1 << 14, 1 << 14, D.FP64)):
        with pytest.raises(D.DugksError) as e:
            D.create(nx, ny, precision=prec)
        assert e.value.code == D.EINVAL and "too large" in str(e.value)


def test_params_marshalling_rejects_unknown_keys():
    with pytest.raises(KeyError):
        D.make_params(dict(bogus=1.0))
    p = D.make_params(dict(visc="reciprocal", walls_y=True, vel="deform", M=0.3))
    assert p.visc_mode == 1 and p.bc_y == 1 and p.vel_kind == 3 and p.M_phi == 0.3


def test_params_struct_matches_the_header(tmp_path):
    """The ctypes mirror of dugks_params has the C layout: size and every
    field offset, from a program compiled against include/dugks.h."""
    fields = [f for f, _ in D.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dugks.h"\n'
                   "int main(void) {\n"
                   '  printf("%zu\\n", sizeof(dugks_params));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(dugks_params, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    import ctypes
    assert got[0] == ctypes.sizeof(D.Params)
    assert got[1:] == [getattr(D.Params, f).offset for f in fields]


def test_reconstruction_and_mesh_arguments():
    assert D.make_params(dict(recon="upwind")).recon == 1
    assert D.make_params({}).recon == 0
    with pytest.raises(KeyError):
        D.make_params(dict(recon="weno"))
    L = D.lib()
    assert L.dugks_set_mesh(None, None, None) == D.EINVAL
