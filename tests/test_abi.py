"""CPU checks of the C ABI: the library loads, exports every function that
include/relres.h declares, its structs match the header's layout, and
parameter validation works without touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
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
    from paper_2104_10231_amd.relres import Params, Stats, Tune
    c = tmp_path / "sz.c"
    c.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "relres.h"\n'
                 'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                 ' sizeof(relres_params), sizeof(relres_stats), offsetof(relres_params, mix),'
                 ' offsetof(relres_params, no_shift), offsetof(relres_params, cut_type),'
                 ' offsetof(relres_params, cut_pair),'
                 ' offsetof(relres_stats, builds), offsetof(relres_stats, box),'
                 ' offsetof(relres_stats, moved_at_last_build), sizeof(relres_tune),'
                 ' offsetof(relres_tune, trials), offsetof(relres_tune, force_us_auto));'
                 ' return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    assert got == [ctypes.sizeof(Params), ctypes.sizeof(Stats), Params.mix.offset,
                   Params.no_shift.offset, Params.cut_type.offset, Params.cut_pair.offset,
                   Stats.builds.offset, Stats.box.offset, Stats.moved_at_last_build.offset,
                   ctypes.sizeof(Tune), Tune.trials.offset, Tune.force_us_auto.offset]


def test_version_and_error_strings(lib):
    assert lib.relres_abi_version() == 7
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11, -12, 1):
        s = lib.relres_strerror(code).decode()
        assert s and s != "unknown error"
    assert lib.relres_strerror(-100).decode() == "unknown error"


def _params(**kw):
    from paper_2104_10231_amd.relres import Params
    import numpy as np
    arrs = [np.array([0.195, 0.195]), np.array([3.75, 3.75]), np.array([0.0, 1.0]),
            np.array([4.6, 4.6])]
    base = dict(rs_in=5.5, rs_out=6.0, rc_in=12.0, rc_out=14.0, skin=2.0, mix=0,
                precision=32, pair_math=0, ntypes=2, no_shift=0, cut_type=None, cut_pair=None)
    base.update(kw)
    ptr = ctypes.POINTER(ctypes.c_double)
    cuts = [None if base[k] is None else np.ascontiguousarray(base[k], dtype=np.float64)
            for k in ("cut_type", "cut_pair")]
    p = Params(base["rs_in"], base["rs_out"], base["rc_in"], base["rc_out"], base["skin"],
               base["ntypes"], *[a.ctypes.data_as(ptr) for a in arrs], base["mix"],
               base["precision"], base["pair_math"], base["no_shift"],
               *[None if a is None else a.ctypes.data_as(ptr) for a in cuts])
    return p, arrs + cuts


@pytest.mark.parametrize("kw,code", [
    (dict(rs_in=6.5), -2), (dict(rc_in=5.0), -2), (dict(rc_out=11.0), -2), (dict(skin=-1.0), -2),
    (dict(rs_in=0.0), -2), (dict(rs_out=float("nan")), -2),
    (dict(precision=16), -1), (dict(pair_math=16), -1), (dict(precision=64, pair_math=32), -1),
    (dict(mix=7), -1), (dict(ntypes=0), -1), (dict(ntypes=33), -1), (dict(no_shift=2), -1),
    # per-type distances out of order for type 1 / mixed pair
    (dict(cut_type=[[5.5, 6.0, 12.0, 14.0], [6.5, 6.0, 12.0, 14.0]]), -2),
    (dict(cut_type=[[5.5, 6.0, 12.0, 14.0], [5.5, 6.0, 12.0, float("inf")]]), -2),
    # an explicit pair table that is not symmetric
    (dict(cut_pair=[[[5.5, 6.0, 12.0, 14.0], [5.5, 6.0, 12.0, 14.0]],
                    [[5.6, 6.0, 12.0, 14.0], [5.5, 6.0, 12.0, 14.0]]]), -1)])
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
    assert lib.relres_set_list_launch(None, 8, 8, 4) == -1
    assert lib.relres_autotune(None, None, None, None, 3, None) == -1
    assert lib.relres_set_bonded(None, 0, None, None, None, 0, None, None, None, 0, None, None,
                                 None, None, 0, None, 0.5) == -1
    assert lib.relres_bonded_forces(None, None, None, None, None, None) == -1
    assert lib.relres_md_setup(None, None, 1.0, 1.0, 1.0, 1.0, 1) == -1
    assert lib.relres_md_run(None, None, None, 1, 0, None, None) == -1
    assert lib.relres_moved_atoms(None, None, None, None) == -1
    assert lib.relres_set_skins(None, None) == -1
    assert lib.relres_check_lists(None) == -1
    lib.relres_destroy(None)


# ----------------------------------------------------------------------------
# host-only parameter helpers (Eqs. 13 and 15, distance mixing): no GPU needed
# ----------------------------------------------------------------------------

def _table1():
    path = os.path.join(ROOT, "tests", "golden", "table1.txt")
    sec, fg, cg, groups = None, {}, {}, {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("["):
            sec = line.strip("[]")
            continue
        tok = line.split()
        if sec == "fg":
            fg[tok[0]] = (float(tok[1]), float(tok[2]))
        elif sec == "cg":
            cg[tok[0]] = (float(tok[1]), float(tok[2]))
        else:
            groups[tok[0]] = tok[1:]
    return fg, cg, groups


def test_eq15_helper_reproduces_table1(lib):
    from paper_2104_10231_amd.relres import cg_site_params
    fg, cg, groups = _table1()
    assert len(groups) == 8
    for name, atoms in groups.items():
        eps, sig = cg_site_params([fg[a][0] for a in atoms], [fg[a][1] for a in atoms])
        assert eps == pytest.approx(cg[name][0], rel=2e-4), name
        assert sig == pytest.approx(cg[name][1], rel=2e-4), name


def test_eq13_helper_reduces_to_eq15_under_geometric_mixing(lib):
    from paper_2104_10231_amd.relres import cg_pair_params, cg_site_params
    rng = np.random.default_rng(2)
    for n_a, n_b in ((1, 1), (3, 3), (5, 3), (4, 1)):
        ea, sa = rng.uniform(0.05, 0.3, n_a), rng.uniform(3.3, 4.0, n_a)
        eb, sb = rng.uniform(0.05, 0.3, n_b), rng.uniform(3.3, 4.0, n_b)
        e_mn = np.sqrt(np.outer(ea, eb))
        s_mn = np.sqrt(np.outer(sa, sb))
        e13, s13 = cg_pair_params(e_mn, s_mn)
        (e1, s1), (e2, s2) = cg_site_params(ea, sa), cg_site_params(eb, sb)
        # Sec. 2.3: the CG pair parameters are then the geometric means of
        # the per-site Eq. 15 values
        assert e13 == pytest.approx(np.sqrt(e1 * e2), rel=1e-12)
        assert s13 == pytest.approx(np.sqrt(s1 * s2), rel=1e-12)
    # one FG pair: Eq. 13 returns it unchanged
    e, s = cg_pair_params([0.21], [3.9])
    assert e == pytest.approx(0.21, rel=1e-15) and s == pytest.approx(3.9, rel=1e-15)


def test_eq13_keeps_the_r6_and_r12_coefficients(lib):
    # u_CG = sum of the FG pair potentials has r^-12 and r^-6 coefficients
    # sum eps sigma^12 and sum eps sigma^6 (Eq. 4); Eq. 13 must keep both
    from paper_2104_10231_amd.relres import cg_pair_params
    rng = np.random.default_rng(5)
    e_mn, s_mn = rng.uniform(0.05, 0.4, 15), rng.uniform(3.0, 4.5, 15)
    e, s = cg_pair_params(e_mn, s_mn)
    assert e * s ** 12 == pytest.approx(np.sum(e_mn * s_mn ** 12), rel=1e-12)
    assert e * s ** 6 == pytest.approx(np.sum(e_mn * s_mn ** 6), rel=1e-12)


def test_mix_distance_and_helper_validation(lib):
    from paper_2104_10231_amd.relres import RelResError, cg_pair_params, cg_site_params, mix_distance
    assert mix_distance(0, 6.0, 7.0) == pytest.approx(6.481, abs=5e-4)     # Sec. 3.4
    assert mix_distance(1, 6.0, 7.0) == 6.5
    assert mix_distance(2, 6.0, 7.0) ** 6 == pytest.approx(0.5 * (6.0 ** 6 + 7.0 ** 6), rel=1e-14)
    assert np.isnan(mix_distance(9, 6.0, 7.0))
    with pytest.raises(RelResError):
        cg_site_params([0.1, -0.2], [3.8, 3.9])
    with pytest.raises(RelResError):
        cg_pair_params([0.0, 0.0], [3.8, 3.9])
    with pytest.raises(RelResError):
        cg_site_params([], [])
