"""CPU checks of the C ABI: the library loads, exports every function that
include/relres.h declares, its structs match the header's layout, and
parameter validation works without touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "relres.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(relres_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2104_10231_amd import relres as b
    if not os.path.exists(b.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return b.load_library()


def test_exports_every_declared_function(lib):
    names = _declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2104_10231_amd",
                                                                      "librelres_hip.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (relres_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    from paper_2104_10231_amd.relres import SIGNATURES
    assert set(SIGNATURES) == set(names)


def test_struct_layout_matches_header(tmp_path):
    from paper_2104_10231_amd.relres import Params, Stats
    c = tmp_path / "sz.c"
    c.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "relres.h"\n'
                 'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(relres_params),'
                 ' sizeof(relres_stats), offsetof(relres_params, mix),'
                 ' offsetof(relres_stats, builds), offsetof(relres_stats, box)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    assert got == [ctypes.sizeof(Params), ctypes.sizeof(Stats), Params.mix.offset,
                   Stats.builds.offset, Stats.box.offset]


def test_version_and_error_strings(lib):
    assert lib.relres_abi_version() == 1
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        s = lib.relres_strerror(code).decode()
        assert s and s != "unknown error"
    assert lib.relres_strerror(-100).decode() == "unknown error"


def _params(**kw):
    from paper_2104_10231_amd.relres import Params
    import numpy as np
    arrs = [np.array([0.195, 0.195]), np.array([3.75, 3.75]), np.array([0.0, 1.0]),
            np.array([4.6, 4.6])]
    base = dict(rs_in=5.5, rs_out=6.0, rc_in=12.0, rc_out=14.0, skin=2.0, mix=0,
                precision=32, pair_math=0, ntypes=2)
    base.update(kw)
    ptr = ctypes.POINTER(ctypes.c_double)
    p = Params(base["rs_in"], base["rs_out"], base["rc_in"], base["rc_out"], base["skin"],
               base["ntypes"], *[a.ctypes.data_as(ptr) for a in arrs], base["mix"],
               base["precision"], base["pair_math"])
    return p, arrs


@pytest.mark.parametrize("kw,code", [
    (dict(rs_in=6.5), -2), (dict(rc_in=5.0), -2), (dict(rc_out=11.0), -2), (dict(skin=-1.0), -2),
    (dict(rs_in=0.0), -2), (dict(rs_out=float("nan")), -2),
    (dict(precision=16), -1), (dict(pair_math=16), -1), (dict(precision=64, pair_math=32), -1),
    (dict(mix=7), -1), (dict(ntypes=0), -1), (dict(ntypes=33), -1)])
def test_create_rejects_bad_parameters(lib, kw, code):
    p, _keep = _params(**kw)
    ctx = ctypes.c_void_p()
    assert lib.relres_create(ctypes.byref(p), ctypes.byref(ctx)) == code
    assert not ctx.value
    assert lib.relres_last_error().decode()


def test_null_arguments_are_rejected(lib):
    ctx = ctypes.c_void_p()
    assert lib.relres_create(None, ctypes.byref(ctx)) == -1
    assert lib.relres_set_topology(None, 0, None, None, 0, None, None) == -1
    assert lib.relres_build_lists(None, None, None, None) == -1
    assert lib.relres_forces(None, None, None, None, None, None) == -1
    assert lib.relres_set_launch(None, 4, 4) == -1
    lib.relres_destroy(None)
