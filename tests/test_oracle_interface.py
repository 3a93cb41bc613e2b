"""Pins of the oracle's pair_style options (Sec. 2.5): pair_modify shift no,
the sixth-power mixing rule, and distances given per type (mixed for unlike
types, Sec. 3.4) or per type pair.

Independent references:
  * shift no: cases 3 and 4 of Eq. 20 become the textbook LJ and the Eq. 17
    closed-form polynomial with no constant; cases 1 and 2 and every force
    stay as under shift yes; the energy changes by Gamma_c- (from Eq. 17 in
    closed form) per hybrid pair in [r_s+, r_c+), counted with numpy;
  * sixth-power mixing: its defining properties (sigma_ab^6 is the mean of
    the sixth powers; the dispersion coefficient eps sigma^6 is the geometric
    mean of the two types' ones);
  * per-type distances: the mixed switching distance of Sec. 3.4
    (sqrt(6 * 7) A ~ 6.481 A), like-type records equal to those of a system
    with that type's distances as the global ones, a two-atom system whose
    pairs sit between two types' cutoffs, continuity at every pair's own
    boundaries, forces against finite differences.
"""
import numpy as np
import pytest

import oracle
import workloads as w
from test_oracle_pins import eq17, lj_sym, polyval


def _propane(seed=3, n_mol=150, L=34.0, hf=0.8):
    return w.random_molecules(seed, n_mol, L, kind="propane", min_dist=2.9, hybrid_fraction=hf)


def _gamma_c(eps, sig, rci, rco):
    """Gamma_c- of Eq. 19 from the closed form of Eq. 17."""
    return polyval(eq17(lj_sym(eps, sig, rci), rco - rci), rco - rci)


# ----------------------------------------------------------------------------
# pair_modify shift no
# ----------------------------------------------------------------------------

def test_shift_no_drops_gamma_c_in_cases_3_and_4_only():
    s = w.propane_liquid(0)
    yes = oracle.setup_table(s)[1, 1]
    no = oracle.setup_table(s.replace(shift=False))[1, 1]
    eps, sig = 1.0, 4.6                      # CG parameters of the hybrid type
    gc = _gamma_c(eps, sig, s.rc_in, s.rc_out)
    assert abs(gc) > 1e-4
    r = np.linspace(2.8, 15.0, 3001)
    uy, dy, cy = oracle.pair(yes, r)[:3]
    un, dn, cn = oracle.pair(no, r)[:3]
    assert np.array_equal(cy, cn)
    assert np.array_equal(dy, dn)            # forces do not change
    inner = cy <= 2
    assert np.array_equal(uy[inner], un[inner])
    outer = (cy == 3) | (cy == 4)
    np.testing.assert_allclose(un[outer] - uy[outer], gc, rtol=1e-9)
    # case 3 is the plain CG LJ; case 4 at r_c- starts from u_CG(r_c-)
    for x in (s.rs_out, 7.3, 10.0, s.rc_in - 1e-9):
        assert oracle.pair(no, x)[0][0] == pytest.approx(lj_sym(eps, sig, x)[0], rel=1e-12)
    assert oracle.pair(no, s.rc_in)[0][0] == pytest.approx(lj_sym(eps, sig, s.rc_in)[0], rel=1e-12)
    # the potential jumps by Gamma_c- at r_s+ and at r_c+
    h = 1e-9
    jump_s = oracle.pair(no, s.rs_out)[0][0] - oracle.pair(no, s.rs_out - h)[0][0]
    assert jump_s == pytest.approx(gc, rel=1e-6)
    assert oracle.pair(no, s.rc_out - h)[0][0] == pytest.approx(gc, rel=1e-6)
    assert oracle.pair(no, s.rc_out)[0][0] == 0.0


def test_shift_no_changes_energy_by_gamma_c_per_outer_hybrid_pair():
    s = _propane()
    sn = s.replace(shift=False)
    Fy, Ey, Wy = oracle.compute(s)
    Fn, En, Wn = oracle.compute(sn)
    assert np.array_equal(Fy, Fn) and np.array_equal(Wy, Wn)
    d = s.pos[:, None, :] - s.pos[None, :, :]
    d -= s.box * np.round(d / s.box)
    r = np.sqrt((d ** 2).sum(-1))
    i, j = np.triu_indices(s.n, 1)
    hyb = s.eps_cg[s.types] > 0
    keep = (s.mol[i] != s.mol[j]) & hyb[i] & hyb[j]
    rij = r[i, j][keep]
    count = int(np.sum((rij >= s.rs_out) & (rij < s.rc_out)))
    assert count > 100
    gc = _gamma_c(s.eps_cg[1], s.sig_cg[1], s.rc_in, s.rc_out)
    assert En[0] - Ey[0] == pytest.approx(count * gc, rel=1e-9)
    assert En[1] == Ey[1]                    # the FG part is untouched


# ----------------------------------------------------------------------------
# sixth-power mixing
# ----------------------------------------------------------------------------

def test_sixthpower_mixing_rule():
    s = w.propane_liquid(0).replace(mix=w.MIX_SIXTHPOWER, eps_cg=np.array([0.0, 1.3]),
                                    sig_cg=np.array([4.1, 4.6]))
    s3 = s.replace(types=s.types, eps_fg=np.array([0.195, 0.091, 0.3]),
                   sig_fg=np.array([3.75, 3.95, 3.3]), eps_cg=np.array([0.0, 1.3, 2.2]),
                   sig_cg=np.array([4.1, 4.6, 5.2]))
    tab = oracle.setup_table(s3)
    for a in range(3):
        for b in range(3):
            R = tab[a, b]
            for E, S, ie, is_ in ((s3.eps_fg, s3.sig_fg, oracle.EPS_FG, oracle.SIG_FG),
                                  (s3.eps_cg, s3.sig_cg, oracle.EPS_CG, oracle.SIG_CG)):
                if ie == oracle.EPS_CG and not (E[a] > 0 and E[b] > 0):
                    assert R[ie] == 0.0          # Eq. 14
                    continue
                assert R[is_] ** 6 == pytest.approx(0.5 * (S[a] ** 6 + S[b] ** 6), rel=1e-14)
                c6 = R[ie] * R[is_] ** 6
                assert c6 == pytest.approx(np.sqrt(E[a] * S[a] ** 6 * E[b] * S[b] ** 6), rel=1e-14)
                if a == b:
                    assert R[ie] == pytest.approx(E[a], rel=1e-15)
                    assert R[is_] == pytest.approx(S[a], rel=1e-15)
    # equal sigmas: the rule reduces to geometric mixing
    g = oracle.setup_table(s3.replace(sig_fg=np.full(3, 3.8), mix=w.MIX_GEOMETRIC))
    t6 = oracle.setup_table(s3.replace(sig_fg=np.full(3, 3.8)))
    np.testing.assert_allclose(t6[:, :, oracle.EPS_FG], g[:, :, oracle.EPS_FG], rtol=1e-15)


# ----------------------------------------------------------------------------
# distances per type and per type pair
# ----------------------------------------------------------------------------

def _two_group_system(seed=3):
    """Propane-like liquid whose two types carry different distances: r_s
    6 A for the ordinary type and 7 A for the hybrid one (Sec. 3.4's pair of
    switching distances), r_c 12/14 A for both."""
    s = _propane(seed)
    ct = np.array([[5.8, 6.2, 12.0, 14.0], [6.8, 7.2, 12.0, 14.0]])
    return s.replace(cut_type=ct)


def test_mixed_switching_distance_of_section_3_4():
    s = w.propane_liquid(0).replace(cut_type=np.array([[6.0, 6.0, 12.0, 14.0],
                                                       [7.0, 7.0, 12.0, 14.0]]))
    tab = oracle.setup_table(s)
    mixed = tab[0, 1, oracle.CUT:oracle.CUT + 4]
    assert mixed[0] == pytest.approx(6.481, abs=5e-4) and mixed[1] == mixed[0]
    assert np.array_equal(tab[1, 0, oracle.CUT:oracle.CUT + 4], mixed)
    assert list(tab[0, 0, oracle.CUT:oracle.CUT + 4]) == [6.0, 6.0, 12.0, 14.0]
    assert list(tab[1, 1, oracle.CUT:oracle.CUT + 4]) == [7.0, 7.0, 12.0, 14.0]
    # the other rules mix the distances as they mix sigma
    lb = oracle.setup_table(s.replace(mix=w.MIX_ARITHMETIC))
    assert lb[0, 1, oracle.CUT] == 6.5
    s6 = oracle.setup_table(s.replace(mix=w.MIX_SIXTHPOWER))
    assert s6[0, 1, oracle.CUT] ** 6 == pytest.approx(0.5 * (6.0 ** 6 + 7.0 ** 6), rel=1e-14)


def test_like_pairs_equal_a_system_with_their_distances_as_global():
    s = _two_group_system()
    tab = oracle.setup_table(s)
    for t in range(2):
        c = s.cut_type[t]
        g = oracle.setup_table(s.replace(cut_type=None, rs_in=c[0], rs_out=c[1], rc_in=c[2],
                                         rc_out=c[3]))
        assert np.array_equal(tab[t, t], g[t, t])


def test_explicit_pair_table_equals_mixed_per_type_distances():
    s = _two_group_system()
    tab = oracle.setup_table(s)
    cp = tab[:, :, oracle.CUT:oracle.CUT + 4].copy()
    sp = s.replace(cut_type=None, cut_pair=cp)
    assert np.array_equal(oracle.setup_table(sp), tab)
    F1, E1, W1 = oracle.compute(s)
    F2, E2, W2 = oracle.compute(sp)
    assert np.array_equal(F1, F2) and np.array_equal(E1, E2) and np.array_equal(W1, W2)


def test_pair_cutoffs_act_per_type_pair():
    """Two atoms 13 A apart: beyond r_c+ = 12.5 A of one type, inside r_c+ =
    14 A of the other."""
    base = w.two_atoms(13.0)
    ct = np.array([[5.0, 5.5, 11.0, 12.5], [6.0, 6.5, 12.0, 14.0]])
    for t, inside in ((0, False), (1, True)):
        s = base.replace(types=np.full(2, t, np.int32), eps_cg=np.array([1.1, 1.0]),
                         sig_cg=np.array([4.4, 4.6]), cut_type=ct)
        F, E, _ = oracle.compute(s)
        if inside:
            # case 4 of Eq. 20 with the type's own r_c-, r_c+ (Eq. 17 closed form)
            c = ct[t]
            g = eq17(lj_sym(s.eps_cg[t], s.sig_cg[t], c[2]), c[3] - c[2])
            du = polyval(g, 13.0 - c[2], 1)
            assert E[0] == pytest.approx(polyval(g, 13.0 - c[2]) - polyval(g, c[3] - c[2]), rel=1e-10)
            assert abs(F[0]).max() == pytest.approx(abs(du), rel=1e-10)
        else:
            assert E[0] == 0.0 and np.all(F == 0.0)


@pytest.mark.parametrize("pair_ab", [(0, 0), (0, 1), (1, 1)])
def test_continuity_at_each_pairs_own_boundaries(pair_ab):
    s = _two_group_system()
    rec = oracle.setup_table(s)[pair_ab]
    cut = rec[oracle.CUT:oracle.CUT + 4]
    u, du = oracle.pair(rec, np.linspace(3.0, 15.0, 2001))[:2]
    umax, dmax = max(1.0, np.abs(u).max()), max(1.0, np.abs(du).max())
    h = 1e-9
    for b in cut:
        u_lo, du_lo = oracle.pair(rec, b - h)[:2]
        u_hi, du_hi = oracle.pair(rec, b + h)[:2]
        assert abs(u_hi[0] - u_lo[0]) <= 4 * h * dmax + 1e-13 * umax, b
        assert abs(du_hi[0] - du_lo[0]) <= 1e-6 * dmax, b
    far = oracle.pair(rec, np.array([cut[3], cut[3] + 1e-9]))
    assert np.all(far[0] == 0.0) and np.all(far[1] == 0.0)


def test_list_radii_are_the_largest_pair_distances():
    s = _two_group_system()
    rso, rco = oracle.list_radii(s)
    assert rso == 7.2 and rco == 14.0
    # the atom list holds every pair up to the largest r_s+ plus the skin
    got = oracle.pairs(s, 0)
    d = s.pos[got[:, 0]] - s.pos[got[:, 1]]
    d -= s.box * np.round(d / s.box)
    assert np.sqrt((d ** 2).sum(-1)).max() > 6.2 + s.skin


@pytest.mark.parametrize("variant", ["shift_no", "sixthpower", "per_type"])
def test_forces_are_minus_energy_gradient(variant):
    s = _two_group_system(seed=4)
    if variant == "shift_no":
        s = s.replace(cut_type=None, shift=False)
    elif variant == "sixthpower":
        s = s.replace(cut_type=None, mix=w.MIX_SIXTHPOWER, sig_cg=np.array([4.0, 4.6]))
    F, E, _ = oracle.compute(s)
    rng = np.random.default_rng(1)
    h = 1e-5
    for flat in rng.choice(3 * s.n, size=24, replace=False):
        i, k = divmod(int(flat), 3)
        p = s.pos.copy(); p[i, k] += h
        Ep = oracle.compute(s, pos=p)[1][0]
        p[i, k] -= 2 * h
        Em = oracle.compute(s, pos=p)[1][0]
        fd = -(Ep - Em) / (2 * h)
        assert abs(fd - F[i, k]) <= 1e-6 * max(1.0, abs(F[i, k])), (i, k, fd, F[i, k])


def test_per_type_distances_are_validated():
    s = w.propane_liquid(0).replace(cut_type=np.array([[6.0, 5.0, 12.0, 14.0],
                                                       [6.0, 6.5, 12.0, 14.0]]))
    with pytest.raises(ValueError):
        oracle.setup_table(s)
