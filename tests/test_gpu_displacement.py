"""Verlet-list validity (Sec. 2.6 neighbour lists with a skin): lists built
with a skin stay exact while no atom has moved more than half the skin since
the build.  relres_moved_atoms counts the atoms that have; every build checks
the previous one and returns RELRES_WARN_DANGEROUS_BUILD when some atom had.

Expected counts come from the definition in numpy: minimum-image displacement
of each atom from its position at the build, |d| > skin / 2.  Displacements
are drawn away from that threshold (|d| <= 0.9 or >= 1.1 times half the
skin), so rounding cannot decide a case.  Integer results: compared exactly.
"""
import numpy as np
import pytest

import workloads as w
from _util import make_relres

pytestmark = pytest.mark.gpu


def _moves(rng, n, half, frac, box):
    """Displacements: a fraction `frac` of the atoms beyond half the skin
    (1.1 .. 3 times it), the rest within 0.9 times it, plus a random periodic
    image shift of whole box edges for some atoms."""
    far = rng.random(n) < frac
    mag = np.where(far, rng.uniform(1.1, 3.0, n), rng.uniform(0.0, 0.9, n)) * half
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    d = u * mag[:, None]
    d += rng.integers(-1, 2, size=(n, 3)) * np.asarray(box).reshape(-1, 3)[0] * (rng.random((n, 1)) < 0.2)
    return d, int(far.sum())


def _count_def(new, old, box, half):
    d = new - old
    d -= box * np.rint(d / box)
    return int(np.count_nonzero(np.sum(d * d, axis=1) > half * half))


def test_moved_atoms_and_dangerous_builds():
    import torch
    s = w.neopentane_liquid(0, n_side=6)
    half = 0.5 * s.skin
    rr = make_relres(s)
    p0 = torch.from_numpy(s.pos.copy()).cuda()
    print(f"[disp] N={s.n} skin={s.skin}", flush=True)
    assert rr.build_lists(p0, s.box) is False          # nothing to compare with
    assert rr.moved_atoms(p0) == 0
    rng = np.random.default_rng(3)
    d, nfar = _moves(rng, s.n, half, 0.03, s.box)
    x1 = s.pos + d
    assert _count_def(x1, s.pos, s.box, half) == nfar
    p1 = torch.from_numpy(x1).cuda()
    assert rr.moved_atoms(p1) == nfar
    # the build at x1 finds the same atoms, and says so once
    assert rr.build_lists(p1, s.box) is True
    st = rr.stats()
    assert st["dangerous_builds"] == 1 and st["moved_at_last_build"] == nfar
    assert rr.moved_atoms(p1) == 0
    assert rr.build_lists(p1, s.box) is False
    assert rr.stats()["moved_at_last_build"] == 0
    # small moves only: no warning
    d2, _ = _moves(rng, s.n, half, 0.0, s.box)
    p2 = torch.from_numpy(x1 + d2).cuda()
    assert rr.moved_atoms(p2) == 0
    assert rr.build_lists(p2, s.box) is False
    # the asynchronous build reports through relres_check_lists
    x3 = x1 + d2
    x3[7] += [0.8 * s.skin, 0.0, 0.0]
    p3 = torch.from_numpy(x3).cuda()
    assert rr.build_lists(p3, s.box, wait=False) is False
    assert rr.check_lists() is True and rr.last_check_dangerous
    assert rr.check_lists() is True and not rr.last_check_dangerous
    assert rr.stats()["dangerous_builds"] == 2
    # a NaN position counts as moved (the build itself would reject it)
    x4 = x3.copy()
    x4[11, 1] = np.nan
    assert rr.moved_atoms(torch.from_numpy(x4).cuda()) == 1
    # a new box: positions are not comparable, no check
    x5 = x3 + np.array([0.9 * s.skin, 0.0, 0.0])
    assert rr.build_lists(torch.from_numpy(x5).cuda(), s.box * 1.01) is False
    rr.close()


def test_new_topology_has_no_reference():
    import torch
    s = w.neopentane_liquid(1, n_side=6)
    rr = make_relres(s)
    p = torch.from_numpy(s.pos.copy()).cuda()
    rr.build_lists(p, s.box)
    csr = s.excl_idx is not None and len(s.excl_idx) > 0
    rr.set_topology(s.types, s.mol, s.exclude_same_mol, s.excl_offsets if csr else None,
                    s.excl_idx if csr else None)
    from paper_2104_10231_amd.relres import RelResError
    with pytest.raises(RelResError):
        rr.moved_atoms(p)
    moved = torch.from_numpy(s.pos + 3.0 * s.skin).cuda()
    assert rr.build_lists(moved, s.box) is False
    assert rr.moved_atoms(moved) == 0
    rr.close()


def test_batched_systems_use_their_own_boxes():
    import torch
    b = w.replica_batch(2, n_systems=4, min_atoms=300, max_atoms=900, total_atoms=2400)
    s = b.whole
    rr = make_relres(s)
    rr.set_systems(b.offsets)
    p0 = torch.from_numpy(s.pos.copy()).cuda()
    assert rr.build_lists(p0, b.boxes) is False
    rng = np.random.default_rng(5)
    x1 = s.pos.copy()
    want = 0
    for k, sy in enumerate(b.systems):
        lo, hi = b.offsets[k], b.offsets[k + 1]
        d, nfar = _moves(rng, hi - lo, 0.5 * s.skin, 0.05, sy.box)
        x1[lo:hi] += d
        want += nfar
        assert _count_def(x1[lo:hi], s.pos[lo:hi], sy.box, 0.5 * s.skin) == nfar
    p1 = torch.from_numpy(x1).cuda()
    assert rr.moved_atoms(p1) == want
    assert rr.build_lists(p1, b.boxes) is (want > 0)
    assert rr.stats()["moved_at_last_build"] == want
    rr.close()
