"""GPU parity of the pair_style options of Sec. 2.5 against the oracle:
pair_modify shift no, the sixth-power mixing rule, distances per type (mixed
for unlike types, as the switching distance of Sec. 3.4) and per type pair.
Same bars as the other parity tests (pair sets bit-exact; FP64: forces 1e-11,
energy/virial 1e-12; FP32: forces 1e-5, energy/virial 1e-7), and the adjoint
at the bars of the gradient tests."""
import numpy as np
import pytest

import oracle
import workloads as w
from _util import make_relres, pair_set, rel_rms
from test_gpu_grad import _compare as grad_compare
from test_gpu_parity import TOL, _check

pytestmark = pytest.mark.gpu

# propane-like groups switch at 6 A, neopentane-like ones at 7 A (Sec. 3.4),
# zones of 0.5 A; all share r_c = 12/14 A
GROUP_DIST = {3: [5.75, 6.25, 12.0, 14.0], 5: [6.75, 7.25, 12.0, 14.0]}


def _propane_per_type():
    s = w.propane_liquid(0)
    return s.replace(cut_type=np.array([[5.3, 5.8, 11.5, 13.5], [6.4, 6.9, 12.0, 14.0]]))


def _mixed_groups(precision=32, n_atoms=6000, seed=4):
    """Propane- and neopentane-like molecules together, each group with its
    own switching distance; types 0/1 propane CH3/CH2, 2/3 neopentane CH3/C."""
    s = w.mixed_liquid(seed, n_atoms, 0.0090, precision=precision, skin=2.0)
    ct = np.array([GROUP_DIST[3], GROUP_DIST[3], GROUP_DIST[5], GROUP_DIST[5]])
    return s.replace(cut_type=ct)


@pytest.mark.parametrize("precision", [64, 32])
def test_shift_no(precision):
    s = w.propane_liquid(1).replace(shift=False, precision=precision)
    F, E, W = _check(s, precision)
    # forces and virial as under shift yes; the energy is not
    Fy, Ey, Wy = oracle.compute(s.replace(shift=True))
    assert rel_rms(F, Fy) <= TOL[precision][0]
    assert abs(E[0] - Ey[0]) > 1e-3 * abs(Ey[0])


def test_sixthpower_mixing_three_types():
    s = w.random_molecules(7, 200, 40.0, kind="neopentane", min_dist=2.9)
    rng = np.random.default_rng(3)
    types = rng.integers(0, 3, size=s.n).astype(np.int32)
    s = s.replace(types=types, mix=w.MIX_SIXTHPOWER, precision=64,
                  eps_fg=np.array([0.195, 0.091, 0.28]), sig_fg=np.array([3.75, 3.95, 3.4]),
                  eps_cg=np.array([0.0, 1.3, 2.4]), sig_cg=np.array([0.0, 4.6, 5.3]))
    _check(s, 64)


@pytest.mark.parametrize("precision,pair_math", [(64, 0), (32, 32), (32, 64)])
def test_per_type_distances(precision, pair_math):
    _check(_propane_per_type().replace(precision=precision), precision, pair_math=pair_math)


@pytest.mark.parametrize("precision,pair_math", [(64, 0), (32, 32)])
def test_two_groups_with_their_own_switching_distances(precision, pair_math):
    s = _mixed_groups(precision)
    tab = oracle.setup_table(s)
    assert tab[1, 3, oracle.CUT + 1] == pytest.approx(np.sqrt(6.25 * 7.25))
    _check(s, precision, pair_math=pair_math)


def test_explicit_pair_table():
    """pair_coeff a b ... with its own distances for every pair of three
    types, here not a mix of per-type values."""
    s = w.random_molecules(5, 300, 38.0, kind="propane", min_dist=2.9)
    rng = np.random.default_rng(8)
    types = rng.integers(0, 3, size=s.n).astype(np.int32)
    cp = np.zeros((3, 3, 4))
    base = {(0, 0): [5.0, 5.6, 11.0, 12.5], (1, 1): [6.0, 6.5, 12.0, 14.0],
            (2, 2): [6.5, 7.0, 12.0, 13.0], (0, 1): [5.5, 6.5, 12.0, 13.5],
            (0, 2): [5.0, 5.0, 11.5, 11.5], (1, 2): [6.2, 6.8, 12.5, 13.8]}
    for (a, b), v in base.items():
        cp[a, b] = cp[b, a] = v
    s = s.replace(types=types, precision=64, cut_pair=cp,
                  eps_fg=np.array([0.195, 0.091, 0.15]), sig_fg=np.array([3.75, 3.95, 3.6]),
                  eps_cg=np.array([0.0, 1.0, 1.6]), sig_cg=np.array([0.0, 4.6, 4.9]))
    _check(s, 64)


@pytest.mark.parametrize("precision", [64, 32])
def test_per_type_distances_with_ten_types(precision):
    """More types than the kernel stages in LDS: tables read from HBM."""
    s = w.random_molecules(9, 200, 40.0, kind="neopentane", min_dist=2.9)
    rng = np.random.default_rng(5)
    nt = 10
    types = rng.integers(0, nt, size=s.n).astype(np.int32)
    rs = rng.uniform(5.0, 7.0, nt)
    rc = rng.uniform(12.0, 13.5, nt)
    ct = np.stack([rs, rs + 0.5, rc, rc + 1.5], axis=1)
    eps_cg = np.where(np.arange(nt) % 3 == 0, 0.0, rng.uniform(0.8, 2.5, nt))
    s = s.replace(types=types, precision=precision, cut_type=ct, shift=False,
                  eps_fg=rng.uniform(0.05, 0.3, nt), sig_fg=rng.uniform(3.4, 4.0, nt),
                  eps_cg=eps_cg, sig_cg=np.where(eps_cg > 0, rng.uniform(4.2, 5.0, nt), 0.0))
    _check(s, precision)


def test_neopentane_20480_per_type_distances():
    """The benchmark liquid with the C hybrid switching later than CH3."""
    s = w.neopentane_liquid(0)
    ct = np.array([[5.5, 6.0, 12.0, 14.0], [6.0, 6.5, 12.0, 14.0]])
    _check(s.replace(cut_type=ct), 32, pair_math=32)


def test_uniform_per_type_distances_equal_global_ones():
    """Equal per-type distances take the global-cutoff kernels and give the
    bitwise result of the global parameters."""
    import torch
    s = w.propane_liquid(2).replace(precision=32)
    ct = np.array([[s.rs_in, s.rs_out, s.rc_in, s.rc_out]] * 2)
    out = []
    for sys in (s, s.replace(cut_type=ct)):
        rr = make_relres(sys, 32)
        p = torch.from_numpy(sys.pos).cuda()
        rr.build_lists(p, sys.box)
        F, E, W = rr.forces(p)
        out.append((F.cpu(), E.cpu(), W.cpu()))
        rr.close()
    assert all(torch.equal(a, b) for a, b in zip(*out))


def test_batched_replicas_with_group_distances():
    import torch
    b = w.replica_batch(2, n_systems=5, min_atoms=300, max_atoms=900, total_atoms=2500,
                        precision=64)
    ct = np.array([GROUP_DIST[3], GROUP_DIST[3], GROUP_DIST[5], GROUP_DIST[5]])
    systems = [s.replace(cut_type=ct) for s in b.systems]
    b = w.batch_of(systems)
    print(f"[interface] batch of {b.nsys} with group distances, N={b.whole.n}", flush=True)
    rr = make_relres(b.whole, 64)
    rr.set_systems(b.offsets)
    p = torch.from_numpy(b.whole.pos).cuda()
    rr.build_lists(p, b.boxes)
    F, E, W = rr.forces(p)
    F, E, W = F.cpu().numpy(), E.cpu().numpy(), W.cpu().numpy()
    ftol, etol = TOL[64]
    want = {0: set(), 1: set()}
    for k, s in enumerate(b.systems):
        o0, o1 = int(b.offsets[k]), int(b.offsets[k + 1])
        Fr, Er, Wr = oracle.compute(s)
        assert rel_rms(F[o0:o1], Fr) <= ftol, k
        assert abs(E[k, 0] - Er[0]) <= etol * abs(Er[0]), k
        assert np.abs(W[k] - Wr).max() <= etol * np.abs(Wr).max(), k
        for which in (0, 1):
            want[which] |= {(i + o0, j + o0) for i, j in pair_set(oracle.pairs(s, which))}
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == want[which]
    rr.close()


@pytest.mark.parametrize("variant", ["sixthpower", "shift_no", "per_type"])
def test_adjoint_with_options(variant):
    s = w.random_molecules(3, 150, 34.0, kind="propane", min_dist=2.9, hybrid_fraction=0.8)
    if variant == "sixthpower":
        s = s.replace(mix=w.MIX_SIXTHPOWER, sig_cg=np.array([4.0, 4.6]))
    elif variant == "shift_no":
        s = s.replace(shift=False)
    else:
        s = s.replace(cut_type=np.array([[5.3, 5.8, 11.5, 13.5], [6.4, 6.9, 12.0, 14.0]]))
    grad_compare(s, seed=4, e_bar=0.8)
