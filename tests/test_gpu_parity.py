"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars:
  * neighbour pair sets: bit-exact (same FP64 membership decision on both sides);
  * FP64 path: forces within 1e-11 relative RMS, energy and virial within 1e-12;
  * FP32 path: forces within 1e-5 relative RMS, energy and virial (accumulated
    in FP64) within 1e-7 relative.
Relative RMS = ||F_gpu - F_ref||_2 / ||F_ref||_2 over all 3N components; the
virial error is max_k |W_k - W_ref,k| / max_k |W_ref,k|.
"""
import numpy as np
import pytest

import oracle
import workloads as w
from _util import gpu_run, make_relres, pair_set, rel_err, rel_rms

pytestmark = pytest.mark.gpu

TOL = {64: (1e-11, 1e-12), 32: (1e-5, 1e-7)}


def _check(s, precision, pair_math=0, pos=None, build_pos=None, lanes=None, pairs=True,
           ref=None, fscale=0.0, escale=0.0):
    """fscale/escale: magnitudes of the pair terms for results that are
    themselves near zero (an isolated pair near a zone end); the errors are
    then measured against max(|result|, scale)."""
    print(f"[parity] {s.name} N={s.n} precision={precision} pair_math={pair_math} "
          f"lanes={lanes}", flush=True)
    rr, F, E, W = gpu_run(s, precision, pair_math, pos=pos, build_pos=build_pos, lanes=lanes)
    sp = s if pos is None else s.replace(pos=pos)
    Fr, Er, Wr = oracle.compute(sp) if ref is None else ref
    ftol, etol = TOL[precision]
    if pairs:
        sb = s if build_pos is None else s.replace(pos=build_pos)
        for which in (0, 1):
            got, want = pair_set(rr.pairs(which)), pair_set(oracle.pairs(sb, which))
            assert got == want, f"list {which}: {len(got - want)} extra, {len(want - got)} missing"
    fden = max(np.sqrt(np.sum(Fr * Fr)), fscale)
    if fden > 0:
        assert np.sqrt(np.sum((F - Fr) ** 2)) <= ftol * fden, rel_rms(F, Fr)
    else:
        assert np.all(F == 0.0)
    eden = max(abs(Er[0]), escale)
    if eden > 0:
        assert abs(E[0] - Er[0]) <= etol * eden, (E, Er)
        scale = max(abs(Er[1]), abs(Er[2]), eden)
        assert abs(E[1] - Er[1]) <= etol * scale and abs(E[2] - Er[2]) <= etol * scale
    else:
        assert np.all(E == 0.0)
    wden = max(np.abs(Wr).max(), fscale * float(np.max(s.box)))
    if wden > 0:
        assert np.abs(W - Wr).max() <= etol * wden, rel_err(W, Wr)
    rr.close()
    return F, E, W


# ---------------------------------------------------------------------------
# the three workloads
# ---------------------------------------------------------------------------

def test_propane_1500_fp64():
    _check(w.propane_liquid(0), 64)


@pytest.mark.parametrize("seed", [1, 2])
def test_propane_1500_fp32(seed):
    _check(w.propane_liquid(seed).replace(precision=32), 32)


@pytest.mark.parametrize("pair_math", [32, 64])
def test_neopentane_20480_fp32(pair_math):
    _check(w.neopentane_liquid(0), 32, pair_math=pair_math)


@pytest.mark.parametrize("n_side", [8, 16, 20, 26])
def test_energy_virial_at_every_poll_width(n_side):
    """Neopentane liquids of 2560 to 87880 atoms: their force launches have
    from ~70 to ~2500 blocks, so the blocks that gather their record group
    poll 2, 4, 8 and 16 records per thread.  Energy and virial against the
    oracle at the FP32 bar, and repeated calls bitwise equal."""
    import torch
    s = w.neopentane_liquid(3, n_side=n_side)
    F, E, W = _check(s, 32)
    rr = make_relres(s, 32)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    for _ in range(3):
        F2, E2, W2 = [t.cpu().numpy() for t in rr.forces(p)]
        assert np.array_equal(E2, E) and np.array_equal(W2, W)
    rr.close()


@pytest.mark.parametrize("name,precision,pair_math", [("propane", 64, 0), ("neopentane", 32, 32),
                                                    ("neopentane", 32, 64)])
def test_forces_only_calls(name, precision, pair_math):
    """Forces without energy/virial run a kernel of their own (FP32 pair terms
    when pair_math is 32); they must meet the same force bar and leave the
    energy/virial buffers alone."""
    import torch
    s = w.propane_liquid(0) if name == "propane" else w.neopentane_liquid(0)
    print(f"[parity] forces-only {s.name} precision={precision} pair_math={pair_math}", flush=True)
    rr = make_relres(s, precision, pair_math)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    E = torch.full((3,), 123.0, dtype=torch.float64, device="cuda")
    W = torch.full((6,), 456.0, dtype=torch.float64, device="cuda")
    F0, _, _ = rr.forces(p, energy=None, virial=None, want_energy=False, want_virial=False)
    F0 = F0.double().cpu().numpy()
    F1, E1, W1 = rr.forces(p, energy=E, virial=W)
    F1 = F1.double().cpu().numpy()
    Fr, Er, Wr = oracle.compute(s)
    ftol = TOL[precision][0]
    assert rel_rms(F0, Fr) <= ftol, rel_rms(F0, Fr)
    assert rel_rms(F1, Fr) <= ftol, rel_rms(F1, Fr)
    E2 = torch.full((3,), 123.0, dtype=torch.float64, device="cuda")
    W2 = torch.full((6,), 456.0, dtype=torch.float64, device="cuda")
    rr.forces(p, energy=E2, virial=None, want_virial=False)
    torch.cuda.synchronize()
    assert abs(E2[0].item() - Er[0]) <= TOL[precision][1] * abs(Er[0])
    assert torch.all(W2 == 456.0)
    rr.close()


def test_neopentane_20480_conventional():
    s = w.neopentane_liquid(0).conventional()
    _check(s, 32)


@pytest.mark.slow
def test_copolymer_98304_sampled():
    s = w.copolymer_melt(0)
    print(f"[parity] copolymer N={s.n} (sampled rows and forces)", flush=True)
    rr, F, E, W = gpu_run(s, 32)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(s.n, size=1500, replace=False)).astype(np.int32)
    hyb = np.nonzero(np.isin(s.types, [1, 3]))[0]
    srows = np.sort(rng.choice(hyb, size=500, replace=False)).astype(np.int32)
    for which, r in ((0, rows), (1, srows)):
        ref = oracle.pairs(s, which, rows=r)
        gp = rr.pairs(which)
        got = set()
        rs = set(r.tolist())
        for i, j in gp.tolist():
            if i in rs:
                got.add((i, j))
            if j in rs:
                got.add((j, i))
        assert got == pair_set(ref), which
    Fs = oracle.compute(s, sel=rows)[0]
    assert rel_rms(F[rows], Fs) <= 1e-5, rel_rms(F[rows], Fs)
    st = rr.stats()
    assert st["n_sites"] == 24576
    rr.close()


@pytest.mark.slow
def test_copolymer_98304_energy_virial():
    s = w.copolymer_melt(0)
    print(f"[parity] copolymer N={s.n} full energy/virial", flush=True)
    rr, F, E, W = gpu_run(s, 32, pair_math=64)
    Fr, Er, Wr = oracle.compute(s)
    assert rel_rms(F, Fr) <= 1e-5
    assert abs(E[0] - Er[0]) <= 1e-7 * abs(Er[0])
    assert rel_err(W, Wr) <= 1e-7
    rr.close()


# ---------------------------------------------------------------------------
# small systems spanning several tiles, ragged tails and all regimes
# ---------------------------------------------------------------------------

SMALL = [("propane", 3, 150, 0.8), ("propane", 4, 97, 1.0), ("neopentane", 5, 61, 0.7),
         ("propane", 6, 130, 0.0), ("neopentane", 7, 40, 1.0)]


@pytest.mark.parametrize("kind,seed,n_mol,hf", SMALL)
@pytest.mark.parametrize("precision", [64, 32])
def test_small_random_systems(kind, seed, n_mol, hf, precision):
    s = w.random_molecules(seed, n_mol, 34.0, kind=kind, min_dist=2.9, hybrid_fraction=hf,
                           precision=precision)
    _check(s, precision)


@pytest.mark.parametrize("lanes", [(1, 1), (2, 4), (4, 8), (8, 16), (16, 32), (32, 64), (64, 64)])
def test_every_lane_split_gives_the_same_physics(lanes):
    s = w.random_molecules(8, 140, 36.0, kind="propane", min_dist=2.9, hybrid_fraction=0.9)
    _check(s, 64, lanes=lanes)


def test_lorentz_berthelot_and_csr_exclusions():
    s = w.random_molecules(9, 120, 35.0, kind="neopentane", min_dist=2.9, hybrid_fraction=0.8)
    # exclude only pairs of consecutive atoms inside a molecule, as explicit lists
    offs, lst = [0], []
    for i in range(s.n):
        part = [j for j in (i - 1, i + 1) if 0 <= j < s.n and s.mol[j] == s.mol[i]]
        lst += part
        offs.append(len(lst))
    s = s.replace(exclude_same_mol=False, excl_offsets=np.array(offs, np.int32),
                  excl_idx=np.array(lst, np.int32), mix=w.MIX_ARITHMETIC,
                  eps_fg=np.array([0.15, 0.07]), sig_fg=np.array([3.9, 3.6]),
                  eps_cg=np.array([0.0, 2.5]), sig_cg=np.array([3.9, 4.1]))
    _check(s, 64)
    _check(s.replace(precision=32), 32)


def test_non_cubic_box_and_unwrapped_positions():
    s = w.random_molecules(10, 130, 34.0, kind="propane", min_dist=2.9)
    box = np.array([34.0, 41.5, 37.25])
    pos = w.wrap(s.pos * (box / 34.0), box)
    s = s.replace(pos=pos, box=box)
    k = np.random.default_rng(2).integers(-1, 2, size=pos.shape)
    _check(s, 64, pos=pos + k * box, build_pos=pos + k * box)


def test_moved_positions_use_build_lists():
    """Forces at positions moved by less than skin/2 since the build are exact."""
    s = w.random_molecules(12, 130, 34.0, kind="propane", min_dist=2.9)
    moved = s.pos + np.random.default_rng(4).normal(scale=0.15, size=s.pos.shape)
    _check(s, 64, pos=moved, build_pos=s.pos, pairs=False)


def test_list_regrow_on_a_dense_cluster():
    # molecules packed into a corner of a large box: far above the mean density
    s = w.random_molecules(13, 90, 22.0, kind="propane", min_dist=2.9)
    big = s.replace(pos=s.pos + 1.0, box=np.full(3, 60.0))
    rr, F, E, W = gpu_run(big, 64)
    st = rr.stats()
    assert st["regrows"] >= 1 and st["atom_capacity"] >= st["atom_max_row"]
    Fr, Er, Wr = oracle.compute(big)
    assert rel_rms(F, Fr) <= 1e-11 and abs(E[0] - Er[0]) <= 1e-12 * abs(Er[0])
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(big, which))
    rr.close()


def test_async_build_matches_blocking_build():
    """Enqueued build + forces, checked afterwards: same lists, same bits."""
    import torch
    s = w.neopentane_liquid(0)
    print(f"[parity] async build {s.name}", flush=True)
    rr = make_relres(s, 32)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)                       # first build always waits
    F0, E0, W0 = rr.forces(p)
    F0, E0, W0 = F0.clone(), E0.clone(), W0.clone()
    moved = torch.from_numpy(s.pos + 0.3).cuda()   # a later build, enqueued
    rr.build_lists(moved, s.box, wait=False)
    F1, E1, W1 = rr.forces(moved)
    assert rr.check_lists()
    Fr, Er, Wr = oracle.compute(s.replace(pos=s.pos + 0.3))
    F1n = F1.double().cpu().numpy()
    assert rel_rms(F1n, Fr) <= TOL[32][0]
    assert abs(E1[0].item() - Er[0]) <= TOL[32][1] * abs(Er[0])
    rr.build_lists(p, s.box, wait=False)
    F2, E2, W2 = rr.forces(p)
    assert rr.check_lists()
    assert torch.equal(F2, F0) and torch.equal(E2, E0) and torch.equal(W2, W0)
    rr.close()


def test_async_build_reports_overflow_and_recovers():
    import torch
    uniform = w.random_molecules(13, 90, 60.0, kind="propane", min_dist=2.9)
    dense = w.random_molecules(13, 90, 22.0, kind="propane", min_dist=2.9)
    dense = dense.replace(pos=dense.pos + 1.0, box=np.full(3, 60.0))
    assert np.array_equal(uniform.types, dense.types) and np.array_equal(uniform.mol, dense.mol)
    print(f"[parity] async overflow N={dense.n}", flush=True)
    rr = make_relres(uniform, 64)
    rr.build_lists(torch.from_numpy(uniform.pos).cuda(), uniform.box)
    regrows = rr.stats()["regrows"]
    p = torch.from_numpy(dense.pos).cuda()
    rr.build_lists(p, dense.box, wait=False)
    rr.forces(p)                                    # enqueued on incomplete lists
    assert not rr.check_lists()                     # ... and reported as such
    with pytest.raises(Exception):
        rr.forces(p)                                # lists invalid until rebuilt
    rr.build_lists(p, dense.box, wait=False)        # grown rows: waits, complete
    assert rr.check_lists()
    F, E, W = rr.forces(p)
    st = rr.stats()
    assert st["regrows"] > regrows and st["atom_capacity"] >= st["atom_max_row"]
    Fr, Er, Wr = oracle.compute(dense)
    assert rel_rms(F.cpu().numpy(), Fr) <= TOL[64][0]
    assert abs(E[0].item() - Er[0]) <= TOL[64][1] * abs(Er[0])
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(dense, which))
    rr.close()


def test_repeated_calls_are_bitwise_identical():
    import torch
    s = w.neopentane_liquid(1)
    rr = make_relres(s)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    a = [t.clone() for t in rr.forces(p)]
    rr.build_lists(p, s.box)
    b = rr.forces(p)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    rr.close()



def test_back_to_back_launches_on_different_positions():
    """Energy/virial launches on alternating positions, enqueued back to back
    (eager and inside a captured graph) with no host wait in between: each
    launch's energy and virial are its own (the cross-block records carry a
    launch tag, so a waiting block never takes a record of the launch
    before), bitwise equal to a synchronised single call."""
    import torch
    s = w.neopentane_liquid(2)
    rng = np.random.default_rng(5)
    pa = torch.from_numpy(s.pos).cuda()
    pb = torch.from_numpy(s.pos + rng.normal(0.0, 0.05, s.pos.shape)).cuda()
    rr = make_relres(s)
    rr.build_lists(pa, s.box)
    ref = {}
    for key, p in (("a", pa), ("b", pb)):
        ref[key] = [t.clone() for t in rr.forces(p)]
        torch.cuda.synchronize()
    assert not torch.equal(ref["a"][1], ref["b"][1])
    outs = [[torch.empty_like(t) for t in ref["a"]] for _ in range(6)]
    for k, o in enumerate(outs):
        rr.forces(pa if k % 2 == 0 else pb, out=o[0], energy=o[1], virial=o[2])
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        want = ref["a" if k % 2 == 0 else "b"]
        assert all(torch.equal(x, y) for x, y in zip(o, want)), k
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for k, o in enumerate(outs):
            rr.forces(pa if k % 2 == 0 else pb, out=o[0], energy=o[1], virial=o[2])
    for rep in range(3):
        for o in outs:
            for x in o:
                x.zero_()
        g.replay()
        torch.cuda.synchronize()
        for k, o in enumerate(outs):
            want = ref["a" if k % 2 == 0 else "b"]
            assert all(torch.equal(x, y) for x, y in zip(o, want)), (rep, k)
    rr.close()


# ---------------------------------------------------------------------------
# degenerate cases and errors
# ---------------------------------------------------------------------------

def test_empty_system():
    import torch
    s = w.two_atoms(5.0)
    s = s.replace(pos=np.zeros((0, 3)), types=np.zeros(0, np.int32), mol=np.zeros(0, np.int32),
                  excl_offsets=np.zeros(1, np.int32))
    rr = make_relres(s)
    p = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    rr.build_lists(p, s.box)
    F, E, W = rr.forces(p)
    assert F.shape == (0, 3) and torch.all(E == 0) and torch.all(W == 0)
    assert len(rr.pairs(0)) == 0 and len(rr.pairs(1)) == 0
    rr.close()


@pytest.mark.parametrize("r", [3.1, 5.7, 5.9999, 6.0, 8.5, 12.0, 13.2, 14.5, 15.99])
@pytest.mark.parametrize("hyb", [(True, True), (True, False), (False, False)])
def test_two_atoms_every_regime(r, hyb):
    s = w.two_atoms(r, hybrid=hyb, direction=(1.0, 2.0, -0.5))
    rec = oracle.setup_table(s)[s.types[0], s.types[1]]
    near = np.linspace(max(0.5, r - 0.5), r + 0.5, 201)
    u, du = oracle.pair(rec, near)[:2]
    _check(s, 64, fscale=float(np.abs(du).max()), escale=float(np.abs(u).max()))


def test_single_molecule_and_all_ordinary():
    s = w.random_molecules(14, 1, 34.0, kind="neopentane")
    F, E, W = _check(s, 64)
    assert np.all(F == 0.0) and np.all(E == 0.0)
    s2 = w.random_molecules(15, 150, 34.0, kind="propane", hybrid_fraction=0.0)
    _check(s2, 32)


def test_errors_are_reported():
    import torch
    from paper_2104_10231_amd.relres import RelResError
    s = w.random_molecules(16, 10, 34.0)
    rr = make_relres(s)
    p = torch.from_numpy(s.pos).cuda()
    with pytest.raises(RelResError) as e:
        rr.forces(p)
    assert e.value.code == -6
    with pytest.raises(RelResError) as e:
        rr.build_lists(p, [31.0, 34.0, 34.0])
    assert e.value.code == -3
    bad = p.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(RelResError) as e:
        rr.build_lists(bad, s.box)
    assert e.value.code == -8
    with pytest.raises(RelResError) as e:
        rr.set_topology(np.full(s.n, 5, np.int32), s.mol)
    assert e.value.code == -4
    # more excluded partners per atom than the builder holds
    many = [j for j in range(1, 66)]
    offs = np.array([0, len(many)] + [len(many)] * (s.n - 1), np.int32)
    with pytest.raises(RelResError) as e:
        rr.set_topology(s.types, s.mol, False, offs, np.array(many, np.int32))
    assert e.value.code == -4
    rr.close()


def test_energy_virial_wait_failure_is_reported(monkeypatch):
    """The cross-block energy/virial wait is bounded; a wait that gives up
    leaves NaN energy/virial and is reported by relres_sync.  Forced from the
    host: a negative spin limit makes every waiting block give up at once, so
    no kernel ever waits."""
    import torch
    from paper_2104_10231_amd.relres import RelResError, RELRES_ERR_EW_TIMEOUT
    s = w.propane_liquid(0)
    p = torch.from_numpy(s.pos).cuda()
    monkeypatch.setenv("RELRES_EW_SPIN_LIMIT", "-1")
    rr = make_relres(s, 64)                    # the limit is read when the context is made
    monkeypatch.delenv("RELRES_EW_SPIN_LIMIT")
    rr.build_lists(p, s.box)
    F, E, W = rr.forces(p)
    with pytest.raises(RelResError) as e:
        rr.sync()
    assert e.value.code == RELRES_ERR_EW_TIMEOUT
    assert torch.isnan(E[0]) and torch.isnan(W).any()
    Fr, Er, Wr = oracle.compute(s)
    assert rel_rms(F.double().cpu().numpy(), Fr) <= 1e-11      # forces are unaffected
    rr.sync()                                  # reported once
    F2, E2, W2 = rr.forces(p, want_energy=False, want_virial=False)
    rr.sync()                                  # no energy asked: nothing waits
    rr.close()
    ok = make_relres(s, 64)
    ok.build_lists(p, s.box)
    F3, E3, W3 = ok.forces(p)
    ok.sync()
    assert abs(E3[0].item() - Er[0]) <= 1e-12 * abs(Er[0])
    ok.close()


@pytest.mark.parametrize("cand", [2, 4])
@pytest.mark.parametrize("cells", [(1, 1), (2, 2)])
def test_candidate_rounds_carry_the_slot_across_rounds(cand, cells):
    """Stencils of several hundred candidates (crowded cells): each round of
    64 x cand candidates finds every candidate's slot from the slots that
    start inside the round and the slot carried over from the previous round.
    Pair sets equal the oracle's for both candidate counts and both cell
    sizes, and the lists give identical forces."""
    import torch
    s = w.random_molecules(17, 80, 15.0, kind="propane", min_dist=2.0)
    big = s.replace(pos=s.pos + 20.0, box=np.full(3, 60.0), skin=8.0)
    print(f"[parity] crowded rounds cand={cand} cells={cells}", flush=True)
    rr = make_relres(big, 64)
    rr.set_cells(*cells)
    rr.set_list_launch(8, 8, cand)
    p = torch.from_numpy(big.pos).cuda()
    rr.build_lists(p, big.box)
    assert rr.stats()["atom_max_row"] > 64
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(big, which))
    F, E, W = rr.forces(p)
    torch.cuda.synchronize()
    Fr, Er, Wr = oracle.compute(big)
    assert rel_rms(F.double().cpu().numpy(), Fr) <= 1e-11
    assert abs(E.cpu().numpy()[0] - Er[0]) <= 1e-12 * abs(Er[0])
    rr.close()


def test_crowded_cells_need_several_passes():
    """Cells holding more than 64 atoms while the mean occupancy is low: the
    one-wave-per-cell builder loops over home atoms in passes of 64."""
    s = w.random_molecules(17, 80, 15.0, kind="propane", min_dist=2.0)
    big = s.replace(pos=s.pos + 20.0, box=np.full(3, 60.0), skin=8.0)
    rr, F, E, W = gpu_run(big, 64)
    st = rr.stats()
    assert st["atom_max_row"] > 64
    Fr, Er, Wr = oracle.compute(big)
    assert rel_rms(F, Fr) <= 1e-11 and abs(E[0] - Er[0]) <= 1e-12 * abs(Er[0])
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(big, which))
    rr.close()


def _one_launch_case(name):
    if name == "propane":
        return w.propane_liquid(1)
    if name == "dense":        # 8 cells of ~19 atoms, no sites: one cell per wave
        return w.random_molecules(21, 50, 23.0, kind="propane", hybrid_fraction=0.0)
    if name == "hexane":       # ~38 sites per site cell: too crowded for buckets
        return w.hexane_liquid(1, n_mol=150, density=0.012)
    if name == "batch":
        return w.replica_batch(4, n_systems=4, min_atoms=300, max_atoms=700, total_atoms=2000)
    s = w.random_molecules(17, 80, 15.0, kind="propane", min_dist=2.0)
    return s.replace(pos=s.pos + 20.0, box=np.full(3, 60.0), skin=8.0)


def _run_placement(s):
    import torch
    if isinstance(s, w.Batch):
        rr = make_relres(s.whole, 64)
        rr.set_systems(s.offsets)
        p = torch.from_numpy(s.whole.pos).cuda()
        rr.build_lists(p, s.boxes)
    else:
        rr = make_relres(s, 64)
        p = torch.from_numpy(s.pos).cuda()
        rr.build_lists(p, s.box)
    out = [t.cpu().numpy() for t in rr.forces(p)]
    torch.cuda.synchronize()
    return rr, out


# path of the default build for each case: 1 = one launch, 3 = classic
_ONE_LAUNCH = {"propane": 1, "dense": 1, "crowded": 1, "batch": 1, "hexane": 3}


@pytest.mark.parametrize("name", list(_ONE_LAUNCH))
def test_one_launch_placement_matches_the_classic_path(monkeypatch, name):
    """Grids of few cells put their members into cell order in one launch
    from per-cell buckets filled while binning (a crowded cell that outgrows
    its bucket collects its members from the key array; cells of more than
    28 members on average keep the classic launches); RELRES_PLACE=classic
    always takes the scan / scatter / cell-sort launches.  Both give the
    oracle's pair sets and bitwise identical lists, forces, energies and
    virials."""
    s = _one_launch_case(name)
    print(f"[parity] placement {name}", flush=True)
    out = {}
    for mode in ("default", "classic"):
        if mode == "classic":
            monkeypatch.setenv("RELRES_PLACE", "classic")
        else:
            monkeypatch.delenv("RELRES_PLACE", raising=False)
        rr, res = _run_placement(s)
        assert rr.stats()["place_launches"] == (_ONE_LAUNCH[name] if mode == "default" else 3)
        if not isinstance(s, w.Batch):
            for which in (0, 1):
                assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(s, which))
        out[mode] = res + [rr.pairs(0), rr.pairs(1)]
        rr.close()
    for a, b in zip(out["default"], out["classic"]):
        assert np.array_equal(a, b)
    if not isinstance(s, w.Batch):
        Fr, Er, Wr = oracle.compute(s)
        assert rel_rms(out["default"][0], Fr) <= 1e-11
        assert abs(out["default"][1][0] - Er[0]) <= 1e-12 * max(abs(Er[0]), 1e-300)


def test_cell_per_block_list_kernel(monkeypatch):
    """The one-block-per-cell list builder (chosen by RELRES_LIST_KERNEL=block)
    gives the same pair sets and forces."""
    monkeypatch.setenv("RELRES_LIST_KERNEL", "block")
    s = w.propane_liquid(3)
    _check(s, 64)
    _check(s.conventional(), 64)


@pytest.mark.parametrize("rows", ["1,1", "2,5", "4,3", "16,12"])
def test_rows_per_wave_of_the_list_kernel(monkeypatch, rows):
    """Any number of home rows per list-kernel wave (RELRES_LIST_ROWS =
    "atom,site") builds the same lists: pair sets equal to the oracle's and
    forces, energies and virials bitwise equal to the default's, for a liquid
    with bonded exclusions and for a batch of systems."""
    import torch
    s = w.hexane_liquid(2, n_mol=150, density=0.012)
    b = w.replica_batch(4, n_systems=4, min_atoms=300, max_atoms=700, total_atoms=2000)

    def batch_run():
        rr = make_relres(b.whole, 32)
        rr.set_systems(b.offsets)
        p = torch.from_numpy(b.whole.pos).cuda()
        rr.build_lists(p, b.boxes)
        out = [t.double().cpu().numpy() for t in rr.forces(p)]
        rr.close()
        return out

    base = gpu_run(s, 32)[1:]
    base_b = batch_run()
    monkeypatch.setenv("RELRES_LIST_ROWS", rows)
    _check(s, 32)
    got = gpu_run(s, 32)[1:]
    for x, y in zip(got, base):
        assert np.array_equal(x, y)
    for x, y in zip(batch_run(), base_b):
        assert np.array_equal(x, y)


def test_grid_of_many_cells():
    """A dilute box of 25^3 atom cells (more than one scan segment: the cell
    offsets come from the two-launch scan) still gives the oracle's pair sets
    and forces."""
    s = w.random_molecules(12, 300, 200.0, kind="propane", min_dist=2.9, hybrid_fraction=0.7)
    _check(s, 64)


def test_graph_replay_matches_eager():
    """relres_forces captured in a HIP graph: every replay, with eager library
    work and synchronisation in between, reproduces the eager results bitwise."""
    import torch
    s = w.neopentane_liquid(2)
    rr = make_relres(s)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    F, E, W = rr.forces(p)                     # warm-up: sizes internal buffers
    F0, E0, W0 = [t.clone() for t in rr.forces(p)]
    gen = rr.generation()
    assert gen == rr.stats()["generation"]
    Fg = torch.empty_like(F0)
    Eg = torch.empty_like(E0)
    Wg = torch.empty_like(W0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            rr.forces(p, out=Fg, energy=Eg, virial=Wg)
    for rep in range(4):
        Fg.zero_(); Eg.zero_(); Wg.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Fg, F0) and torch.equal(Eg, E0) and torch.equal(Wg, W0), rep
        # eager work in between replays
        F1, E1, W1 = rr.forces(p)
        torch.cuda.synchronize()
        assert torch.equal(F1, F0)
        rr.build_lists(p, s.box)
        assert rr.generation() == gen
    rr.close()
