"""List grids with cells of half the list radius (relres_set_cells 2, a
125-cell stencil) against the oracle: the pair sets must be the same as with
cells of one list radius, bit-exact (the membership recipe does not depend on
the cell size), and forces, energy and virial must meet the usual bars.
Grids of five or more cells per axis take the stencil's image shifts as
known; smaller ones (here four half cells along an axis) deduplicate the
stencil and fall back to the minimum-image test."""
import numpy as np
import pytest

import oracle
import workloads as w
from _util import make_relres, pair_set, rel_rms

pytestmark = pytest.mark.gpu

TOL = {64: (1e-11, 1e-12), 32: (1e-5, 1e-7)}


def _check(s, cells, precision=None, lanes=None):
    import torch
    prec = s.precision if precision is None else precision
    print(f"[cells] {s.name} N={s.n} cells={cells} precision={prec}", flush=True)
    rr = make_relres(s, prec)
    rr.set_cells(*cells)
    if lanes:
        rr.set_launch(*lanes)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    F, E, W = rr.forces(p)
    torch.cuda.synchronize()
    st = rr.stats()
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(s, which)), which
    Fr, Er, Wr = oracle.compute(s)
    ftol, etol = TOL[prec]
    F = F.double().cpu().numpy()
    E = E.cpu().numpy()
    W = W.cpu().numpy()
    assert rel_rms(F, Fr) <= ftol, rel_rms(F, Fr)
    assert abs(E[0] - Er[0]) <= etol * abs(Er[0]), (E, Er)
    assert abs(E[1] - Er[1]) <= etol * max(abs(Er[1]), abs(Er[0]))
    assert np.abs(W - Wr).max() <= etol * np.abs(Wr).max()
    rr.close()
    return st


@pytest.mark.parametrize("cells", [(2, 2), (2, 1), (1, 2)])
def test_propane_1500_half_cells(cells):
    st = _check(w.propane_liquid(0), cells)
    # 54 A box: 13 half cells of >= 4 A (atom grid), 6 of >= 8 A (site grid)
    if cells[0] == 2:
        assert st["atom_cells"] == [13, 13, 13]
    if cells[1] == 2:
        assert st["site_cells"] == [6, 6, 6]


def test_neopentane_20480_half_cells():
    st = _check(w.neopentane_liquid(0), (2, 2))
    assert st["atom_cells"] == [33, 33, 33] and st["site_cells"] == [16, 16, 16]


@pytest.mark.parametrize("precision", [64, 32])
def test_small_box_deduplicated_stencil(precision):
    # site grid: 34 A / 8 A -> 4 half cells per axis, fewer than the stencil's 5
    s = w.random_molecules(3, 150, 34.0, kind="propane", min_dist=2.9, hybrid_fraction=0.8)
    st = _check(s, (2, 2), precision)
    assert st["site_cells"] == [4, 4, 4]


def test_non_cubic_box_without_hybrid_atoms():
    # no hybrid atoms: only the atom list (radius 8 A); 17 x 25 x 41 A box ->
    # 4, 6 and 10 half cells: one axis deduplicated, the others not
    s = w.random_molecules(6, 60, 34.0, kind="propane", min_dist=2.9, hybrid_fraction=0.0)
    box = np.array([17.0, 25.0, 41.0])
    rng = np.random.default_rng(1)
    pos = rng.uniform(0.0, 1.0, size=s.pos.shape) * box
    s = s.replace(pos=pos, box=box, exclude_same_mol=False)
    st = _check(s, (2, 2), 64)
    assert st["atom_cells"] == [4, 6, 10]


def test_batch_of_replicas_half_cells():
    import torch
    b = w.replica_batch(1, n_systems=6, min_atoms=300, max_atoms=900, total_atoms=3000)
    print(f"[cells] batch of {b.nsys}, N={b.whole.n}", flush=True)
    out = {}
    for cells in ((1, 1), (2, 2)):
        rr = make_relres(b.whole, 32)
        rr.set_systems(b.offsets)
        rr.set_cells(*cells)
        p = torch.from_numpy(b.whole.pos).cuda()
        rr.build_lists(p, b.boxes)
        F, E, W = rr.forces(p)
        torch.cuda.synchronize()
        out[cells] = ([pair_set(rr.pairs(k)) for k in (0, 1)], F.double().cpu().numpy(),
                      E.cpu().numpy(), W.cpu().numpy())
        rr.close()
    a, h = out[(1, 1)], out[(2, 2)]
    assert a[0] == h[0]
    assert rel_rms(h[1], a[1]) <= 1e-6
    assert np.abs(h[2] - a[2]).max() <= 1e-7 * np.abs(a[2]).max()
    for k, s in enumerate(b.systems):
        o0, o1 = int(b.offsets[k]), int(b.offsets[k + 1])
        Fr, Er, Wr = oracle.compute(s)
        assert rel_rms(h[1][o0:o1], Fr) <= 1e-5, k
        assert abs(h[2][k, 0] - Er[0]) <= 1e-7 * abs(Er[0]), k


def test_cells_argument_is_checked():
    from paper_2104_10231_amd.relres import RelResError
    s = w.propane_liquid(1)
    rr = make_relres(s, 32)
    for bad in ((3, 1), (1, -1)):
        with pytest.raises(RelResError):
            rr.set_cells(*bad)
    rr.close()
