"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these re-types the oracle's formulas to compare them with themselves:
  * LJ derivatives against sympy differentiation of Eq. 11;
  * the numerically solved boundary systems (Eqs. 7/8) against the paper's
    closed forms (Eq. 17, and Eq. 18 with the corrected gamma_4+);
  * energy/force/curvature continuity at the four zone boundaries (Sec. 2.2)
    and u~(r_c+) = 0 (Eq. 9);
  * textbook special cases: plain LJ in the FG core and the CG window,
    truncated-and-shifted LJ for empty zones, the pure-CG limit r_s -> 0 and
    the reference (all-FG) limit (Sec. 2.1);
  * forces against central finite differences of the energy, the virial
    against finite strain derivatives, net force zero, invariances;
  * Table 1 against the Eq. 15 helper;
  * the pair sets against an independent numpy enumeration.
"""
import numpy as np
import pytest
import sympy

import oracle
import workloads as w

# ----------------------------------------------------------------------------
# independent textbook LJ (Eq. 11) and its derivatives via sympy
# ----------------------------------------------------------------------------
_r, _e, _s = sympy.symbols("r e s", positive=True)
_u = 4 * _e * ((_s / _r) ** 12 - (_s / _r) ** 6)
_LJ = sympy.lambdify((_e, _s, _r), [_u, sympy.diff(_u, _r), sympy.diff(_u, _r, 2),
                                    sympy.diff(_u, _r, 3)], "math")


def lj_sym(eps, sig, r):
    return np.array(_LJ(float(eps), float(sig), float(r)), dtype=float)


def eq17(u3, D):
    u, du, d2u = u3[:3]
    return np.array([u, du, 0.5 * d2u, -du / D ** 2 - 2 * d2u / (3 * D),
                     du / (2 * D ** 3) + d2u / (4 * D ** 2)])


def eq18(u3, D, printed=False):
    u, du, d2u = u3[:3]
    g4 = (-du / (2 * D ** 3) - d2u / (4 * D ** 2)) if printed else \
         (-du / (2 * D ** 3) + d2u / (4 * D ** 2))
    return np.array([u - 0.5 * du * D + d2u * D ** 2 / 12.0, 0.0, 0.0,
                     du / D ** 2 - d2u / (3 * D), g4])


def polyval(g, d, k=0):
    """k-th derivative of sum g_m d^m (numpy, independent of the oracle)."""
    p = np.polynomial.polynomial.Polynomial(g)
    for _ in range(k):
        p = p.deriv()
    return p(d)


CASES = [(0.195, 3.75, 5.5, 0.5), (1.0, 4.6, 6.0, 0.5), (3.04, 3.94, 12.0, 2.0),
         (0.091, 3.95, 5.0, 0.05), (21.133 * w.ZJ, 3.942, 7.0, 0.3)]


def test_lj_derivatives_match_sympy():
    for eps, sig, r0, _ in CASES:
        for r in (2.9, r0, 9.7, 13.3):
            np.testing.assert_allclose(oracle.lj(eps, sig, r), lj_sym(eps, sig, r)[:3],
                                       rtol=1e-13, atol=0)


@pytest.mark.parametrize("eps,sig,rm,D", CASES)
def test_switch_off_solve_matches_eq17(eps, sig, rm, D):
    u3 = lj_sym(eps, sig, rm)
    g = oracle.solve_poly(0, D, u3)
    ref = eq17(u3, D)
    scale = np.max(np.abs(ref * D ** np.arange(5)))
    np.testing.assert_allclose(g * D ** np.arange(5), ref * D ** np.arange(5),
                               rtol=0, atol=1e-12 * scale)
    # Eq. 7 boundary conditions
    assert abs(polyval(g, 0.0) - u3[0]) <= 1e-12 * scale
    assert abs(polyval(g, 0.0, 1) - u3[1]) <= 1e-12 * scale / D
    assert abs(polyval(g, 0.0, 2) - u3[2]) <= 1e-12 * scale / D ** 2
    assert abs(polyval(g, D, 1)) <= 1e-11 * scale / D
    assert abs(polyval(g, D, 2)) <= 1e-11 * scale / D ** 2


@pytest.mark.parametrize("eps,sig,rp,D", CASES)
def test_switch_on_solve_matches_corrected_eq18(eps, sig, rp, D):
    u3 = lj_sym(eps, sig, rp)
    g = oracle.solve_poly(1, D, u3)
    ref = eq18(u3, D)
    scale = np.max(np.abs(ref * D ** np.arange(5)))
    np.testing.assert_allclose(g * D ** np.arange(5), ref * D ** np.arange(5),
                               rtol=0, atol=1e-12 * scale)
    # Eq. 8 boundary conditions hold for the solved polynomial
    assert abs(polyval(g, D) - u3[0]) <= 1e-12 * scale
    assert abs(polyval(g, D, 1) - u3[1]) <= 1e-11 * scale / D
    assert abs(polyval(g, D, 2) - u3[2]) <= 1e-11 * scale / D ** 2
    # ... but Eq. 18 as printed (sign of the u'' term in gamma_4+) violates
    # f''_+(D) = u''(r_+): it yields -5 u'' instead.
    bad = eq18(u3, D, printed=True)
    np.testing.assert_allclose(polyval(bad, D, 2), -5.0 * u3[2], rtol=1e-9)
    assert abs(polyval(bad, D, 2) - u3[2]) > 1.0 * abs(u3[2])


def _records():
    out = []
    for sysf in (w.propane_liquid, w.neopentane_liquid):
        s = sysf(0)
        tab = oracle.setup_table(s)
        for a in range(s.ntypes):
            for b in range(s.ntypes):
                out.append((s, tab[a, b], (a, b)))
    # Lorentz-Berthelot, four types: parameters only (no need to grow chains)
    s = w.propane_liquid(0).replace(
        eps_fg=np.array([0.195, 0.195, 0.091, 0.091]), sig_fg=np.array([3.75, 3.75, 3.95, 3.95]),
        eps_cg=np.array([0.0, 3.12, 0.0, 1.456]), sig_cg=np.array([3.75, 3.75, 3.95, 3.95]),
        mix=w.MIX_ARITHMETIC)
    tab = oracle.setup_table(s)
    for a in range(4):
        for b in range(4):
            out.append((s, tab[a, b], (a, b)))
    return out


RECORDS = _records()


@pytest.mark.parametrize("k", range(len(RECORDS)))
def test_continuity_at_all_boundaries(k):
    s, rec, _ = RECORDS[k]
    cut = oracle.cutoffs(s)
    rr = np.linspace(3.0, 15.0, 4001)
    u, du, _, _, _ = oracle.pair(rec, rr)
    umax = max(1.0, np.abs(u).max())
    dmax = max(1.0, np.abs(du).max())
    h = 1e-9
    for b in cut:
        u_lo, du_lo = oracle.pair(rec, b - h)[:2]
        u_hi, du_hi = oracle.pair(rec, b + h)[:2]
        assert abs(u_hi[0] - u_lo[0]) <= 4 * h * dmax + 1e-13 * umax, b
        assert abs(du_hi[0] - du_lo[0]) <= 1e-6 * dmax, b
        # second derivative: one-sided difference quotients of u~'
        h2 = 1e-5
        left = (oracle.pair(rec, b - h2)[1] - oracle.pair(rec, b - 3 * h2)[1]) / (2 * h2)
        right = (oracle.pair(rec, b + 3 * h2)[1] - oracle.pair(rec, b + h2)[1]) / (2 * h2)
        assert abs(left[0] - right[0]) <= 1e-3 * dmax, b
    # u~ vanishes from r_c+ on (Eq. 9 with Gamma_c+ = Gamma_c-)
    far = oracle.pair(rec, np.array([cut[3], cut[3] + 1e-12, 20.0]))
    assert np.all(far[0] == 0.0) and np.all(far[1] == 0.0)
    # the FG/CG split adds up to Eq. 20
    uu, _, _, efg, ecg = oracle.pair(rec, rr)
    np.testing.assert_allclose(efg + ecg, uu, rtol=0, atol=1e-12 * umax)


def test_ordinary_pairs_vanish_beyond_rs():
    s = w.propane_liquid(0)
    rec = oracle.setup_table(s)[0, 1]      # ordinary-hybrid: eps_CG = 0 (Eq. 14)
    cut = oracle.cutoffs(s)
    r = np.linspace(s.rs_out, 20.0, 500)
    u, du = oracle.pair(rec, r)[:2]
    assert np.all(u == 0.0) and np.all(du == 0.0)


def test_textbook_lj_in_fg_core_and_cg_window():
    s = w.propane_liquid(0)
    tab = oracle.setup_table(s)
    cut = oracle.cutoffs(s)
    for a, b in [(0, 0), (0, 1), (1, 1)]:
        eps, sig = np.sqrt(s.eps_fg[a] * s.eps_fg[b]), np.sqrt(s.sig_fg[a] * s.sig_fg[b])
        r = np.linspace(2.5, s.rs_in - 1e-6, 50)
        u, du, which = oracle.pair(tab[a, b], r)[:3]
        assert np.all(which == 1)
        ref = np.array([lj_sym(eps, sig, x) for x in r])
        np.testing.assert_allclose(du, ref[:, 1], rtol=1e-13)
        np.testing.assert_allclose(u - u[0], ref[:, 0] - ref[0, 0], rtol=0,
                                   atol=1e-12 * np.abs(ref[:, 0]).max())
    eps, sig = 1.0, 4.6
    r = np.linspace(s.rs_out, s.rc_in - 1e-6, 50)
    u, du, which = oracle.pair(tab[1, 1], r)[:3]
    assert np.all(which == 3)
    ref = np.array([lj_sym(eps, sig, x) for x in r])
    np.testing.assert_allclose(du, ref[:, 1], rtol=1e-13)


def test_empty_zones_give_truncated_shifted_lj():
    s = w.two_atoms(5.0).replace(rs_in=10.0, rs_out=10.0, rc_in=10.0, rc_out=10.0,
                                 eps_cg=np.array([0.0, 0.0]))
    rec = oracle.setup_table(s)[1, 1]
    cut = oracle.cutoffs(s)
    r = np.array([3.0, 4.2, 6.0, 9.999, 10.0, 11.0])
    u, du = oracle.pair(rec, r)[:2]
    uc = lj_sym(0.195, 3.75, 10.0)[0]
    for k, x in enumerate(r):
        if x < 10.0:
            ref = lj_sym(0.195, 3.75, x)
            assert u[k] == pytest.approx(ref[0] - uc, rel=1e-13, abs=1e-15)
            assert du[k] == pytest.approx(ref[1], rel=1e-13)
        else:
            assert u[k] == 0.0 and du[k] == 0.0


def test_reference_limit_is_smoothed_fg_lj():
    """r_s -> r_c with no CG sites: plain FG LJ up to r_c- minus a constant,
    then the Eq. 17 switch-off polynomial (closed form) to zero at r_c+."""
    s = w.propane_liquid(0).conventional()
    rec = oracle.setup_table(s)[0, 1]
    cut = oracle.cutoffs(s)
    eps, sig = 0.195, 3.75
    g = eq17(lj_sym(eps, sig, 12.0), 2.0)
    shift = polyval(g, 2.0)
    for x in (3.3, 7.7, 11.9, 12.0, 12.5, 13.99, 14.0):
        u, du = (q[0] for q in oracle.pair(rec, x)[:2])
        if x < 12.0:
            ref = lj_sym(eps, sig, x)
            assert u == pytest.approx(ref[0] - shift, rel=1e-12, abs=1e-14)
            assert du == pytest.approx(ref[1], rel=1e-13)
        elif x < 14.0:
            assert u == pytest.approx(polyval(g, x - 12.0) - shift, rel=1e-10, abs=1e-14)
            assert du == pytest.approx(polyval(g, x - 12.0, 1), rel=1e-10, abs=1e-14)
        else:
            assert u == 0.0


def _dense_system(seed=3, n_mol=150, L=34.0, kind="propane", hf=0.8):
    return w.random_molecules(seed, n_mol, L, kind=kind, min_dist=2.9, hybrid_fraction=hf)


def test_pure_cg_limit_equals_cg_sites_alone():
    """r_s -> 0 (Sec. 2.1): only the CG potential between hybrid sites remains."""
    s = _dense_system(hf=1.0)
    relres = s.replace(rs_in=1.0, rs_out=1.0)
    F, E, W = oracle.compute(relres)
    h = np.nonzero(s.types == 1)[0]
    sub = s.replace(pos=s.pos[h], types=np.zeros(len(h), np.int32), mol=s.mol[h],
                    excl_offsets=np.zeros(len(h) + 1, np.int32),
                    eps_fg=np.array([1.0]), sig_fg=np.array([4.6]),
                    eps_cg=np.array([0.0]), sig_cg=np.array([4.6]),
                    rs_in=s.rc_in, rs_out=s.rc_out, rc_in=s.rc_out, rc_out=s.rc_out)
    Fs, Es, Ws = oracle.compute(sub)
    assert E[0] == pytest.approx(Es[0], rel=1e-12)
    np.testing.assert_allclose(F[h], Fs, rtol=0, atol=1e-12 * np.abs(Fs).max())
    others = np.setdiff1d(np.arange(s.n), h)
    assert np.abs(F[others]).max() == 0.0
    np.testing.assert_allclose(W, Ws, rtol=0, atol=1e-12 * np.abs(Ws).max())


def _regimes_hit(s):
    tab = oracle.setup_table(s)
    cut = oracle.cutoffs(s)
    d = s.pos[:, None, :] - s.pos[None, :, :]
    d -= s.box * np.round(d / s.box)
    r = np.sqrt((d ** 2).sum(-1))
    iu = np.triu_indices(s.n, 1)
    keep = s.mol[iu[0]] != s.mol[iu[1]]
    hit = set()
    for i, j in zip(iu[0][keep], iu[1][keep]):
        if r[i, j] < cut[3]:
            hit.add(int(oracle.pair(tab[s.types[i], s.types[j]], r[i, j])[2][0]))
    return hit


def test_forces_are_minus_energy_gradient():
    s = _dense_system()
    assert _regimes_hit(s) >= {1, 2, 3, 4}
    F, E, _ = oracle.compute(s)
    rng = np.random.default_rng(0)
    h = 1e-5
    for flat in rng.choice(3 * s.n, size=40, replace=False):
        i, k = divmod(int(flat), 3)
        p = s.pos.copy(); p[i, k] += h
        Ep = oracle.compute(s, pos=p)[1][0]
        p[i, k] -= 2 * h
        Em = oracle.compute(s, pos=p)[1][0]
        fd = -(Ep - Em) / (2 * h)
        assert abs(fd - F[i, k]) <= 1e-6 * max(1.0, abs(F[i, k])), (i, k, fd, F[i, k])


def test_virial_diagonal_is_minus_strain_derivative():
    s = _dense_system(seed=5)
    _, E, W = oracle.compute(s)
    h = 1e-7
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        Ep = oracle.compute(s.replace(pos=s.pos * sc, box=s.box * sc))[1][0]
        sc[a] = 1 - h
        Em = oracle.compute(s.replace(pos=s.pos * sc, box=s.box * sc))[1][0]
        fd = -(Ep - Em) / (2 * h)
        assert fd == pytest.approx(W[a], rel=1e-6, abs=1e-6)


def test_virial_rotates_as_a_tensor():
    s = _dense_system(seed=6)
    _, _, W = oracle.compute(s)
    L = s.box[0]
    rot = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    p2 = w.wrap(s.pos @ rot.T, s.box)
    _, _, W2 = oracle.compute(s.replace(pos=p2))

    def mat(v):
        return np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])
    np.testing.assert_allclose(mat(W2), rot @ mat(W) @ rot.T, rtol=0,
                               atol=1e-10 * np.abs(W).max())
    assert L == s.box[1]


def test_net_force_translation_and_permutation():
    s = _dense_system(seed=7, kind="neopentane", n_mol=80)
    F, E, W = oracle.compute(s)
    assert np.abs(F.sum(0)).max() <= 1e-12 * np.abs(F).sum()
    shift = np.array([13.1, -7.7, 101.3])
    F2, E2, W2 = oracle.compute(s.replace(pos=w.wrap(s.pos + shift, s.box)))
    assert E2[0] == pytest.approx(E[0], rel=1e-11)
    np.testing.assert_allclose(F2, F, rtol=0, atol=1e-10 * np.abs(F).max())
    perm = np.random.default_rng(1).permutation(s.n)
    sp = s.replace(pos=s.pos[perm], types=s.types[perm], mol=s.mol[perm],
                   excl_offsets=np.zeros(s.n + 1, np.int32))
    F3, E3, W3 = oracle.compute(sp)
    assert E3[0] == pytest.approx(E[0], rel=1e-12)
    np.testing.assert_allclose(F3, F[perm], rtol=0, atol=1e-12 * np.abs(F).max())


def test_exclusions_remove_exactly_the_intramolecular_pairs():
    s = _dense_system(seed=8, n_mol=60)
    _, E_ex, _ = oracle.compute(s)
    s_all = s.replace(exclude_same_mol=False)
    _, E_all, _ = oracle.compute(s_all)
    tab = oracle.setup_table(s)
    cut = oracle.cutoffs(s)
    intra = 0.0
    for m in np.unique(s.mol):
        idx = np.nonzero(s.mol == m)[0]
        for a in range(len(idx)):
            for b in range(a + 1, len(idx)):
                i, j = idx[a], idx[b]
                d = s.pos[i] - s.pos[j]
                d -= s.box * np.round(d / s.box)
                intra += oracle.pair(tab[s.types[i], s.types[j]], np.linalg.norm(d))[0][0]
    # the bonded intramolecular terms are ~1e4 each: compare on their scale
    assert E_ex[0] == pytest.approx(E_all[0] - intra, rel=0, abs=1e-13 * abs(E_all[0]))
    # the same exclusions given as explicit CSR lists
    offs, lst = [0], []
    for i in range(s.n):
        part = [j for j in np.nonzero(s.mol == s.mol[i])[0] if j != i]
        lst += part
        offs.append(len(lst))
    s_csr = s.replace(exclude_same_mol=False, excl_offsets=np.array(offs, np.int32),
                      excl_idx=np.array(lst, np.int32))
    F1, E1, W1 = oracle.compute(s)
    F2, E2, W2 = oracle.compute(s_csr)
    assert np.array_equal(F1, F2) and np.array_equal(E1, E2) and np.array_equal(W1, W2)


def _table1():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")
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


def test_table1_cg_parameters_follow_eq15():
    fg, cg, groups = _table1()
    assert len(cg) == 8
    for name, atoms in groups.items():
        e = [fg[a][0] for a in atoms]
        sg = [fg[a][1] for a in atoms]
        sig, eps = oracle.cg_params_eq15(e, sg)
        assert eps == pytest.approx(cg[name][0], rel=2e-4), name
        assert sig == pytest.approx(cg[name][1], rel=2e-4), name
        # Eq. 13 over all mu-nu pairs of two identical groups with geometric
        # mixing reduces to Eq. 15 (Sec. 2.3)
        E = np.sqrt(np.outer(e, e)); S = np.sqrt(np.outer(sg, sg))
        sig13, eps13 = oracle.cg_params_eq13(E, S)
        assert sig13 == pytest.approx(sig, rel=1e-12)
        assert eps13 == pytest.approx(eps, rel=1e-12)


def _np_pairs(s, which, margin=1e-7):
    """Independent enumeration: rint minimum image, r compared with r_l."""
    rl = (s.rs_out if which == 0 else s.rc_out) + s.skin
    hyb = s.eps_cg[s.types] > 0
    d = s.pos[:, None, :] - s.pos[None, :, :]
    d -= s.box * np.round(d / s.box)
    r = np.sqrt((d ** 2).sum(-1))
    i, j = np.triu_indices(s.n, 1)
    keep = np.ones(len(i), bool)
    if s.exclude_same_mol:
        keep &= s.mol[i] != s.mol[j]
    if len(s.excl_idx):
        ex = set()
        for a in range(s.n):
            for b in s.excl_idx[s.excl_offsets[a]:s.excl_offsets[a + 1]]:
                ex.add((min(a, b), max(a, b)))
        keep &= np.array([(a, b) not in ex for a, b in zip(i, j)])
    if which == 1:
        keep &= hyb[i] & hyb[j]
    rij = r[i, j]
    sure_in = keep & (rij < rl - margin)
    sure_out = ~keep | (rij > rl + margin)
    return set(zip(i[sure_in], j[sure_in])), set(zip(i[~sure_out], j[~sure_out]))


@pytest.mark.parametrize("which", [0, 1])
def test_pair_sets_match_independent_enumeration(which):
    for s in (w.propane_liquid(0), _dense_system(seed=9, kind="neopentane", n_mol=90)):
        got = set(map(tuple, oracle.pairs(s, which).tolist()))
        sure, maybe = _np_pairs(s, which)
        assert sure <= got <= maybe
        assert len(got) > 0


def test_pair_sets_with_csr_exclusions():
    # a short chain system: exclusions |i-j| <= 3 inside each "molecule"
    s = _dense_system(seed=10, n_mol=100)
    offs, lst = [0], []
    for i in range(s.n):
        part = [j for j in range(max(0, i - 3), min(s.n, i + 4)) if j != i and s.mol[j] == s.mol[i]]
        lst += part
        offs.append(len(lst))
    s = s.replace(exclude_same_mol=False, excl_offsets=np.array(offs, np.int32),
                  excl_idx=np.array(lst, np.int32))
    for which in (0, 1):
        got = set(map(tuple, oracle.pairs(s, which).tolist()))
        sure, maybe = _np_pairs(s, which)
        assert sure <= got <= maybe


def test_sampled_rows_agree_with_full_enumeration():
    s = w.propane_liquid(1)
    full = oracle.pairs(s, 0)
    rows = np.array([0, 7, 500, 1499], np.int32)
    part = oracle.pairs(s, 0, rows=rows)
    for i in rows:
        mine = set(part[part[:, 0] == i][:, 1].tolist())
        ref = set(full[full[:, 0] == i][:, 1].tolist()) | set(full[full[:, 1] == i][:, 0].tolist())
        assert mine == ref
    F, E, W = oracle.compute(s)
    Fs = oracle.compute(s, sel=rows)[0]
    np.testing.assert_array_equal(Fs, F[rows])


def test_empty_switching_zone_keeps_energy_continuous():
    s = w.two_atoms(5.0).replace(rs_in=6.0, rs_out=6.0)
    rec = oracle.setup_table(s)[1, 1]
    cut = oracle.cutoffs(s)
    lo, hi = oracle.pair(rec, np.array([6.0 - 1e-10, 6.0]))[0]
    assert hi == pytest.approx(lo, abs=1e-8)


def test_energy_split_and_unwrapped_positions():
    s = w.propane_liquid(2)
    F, E, W = oracle.compute(s)
    assert E[1] + E[2] == pytest.approx(E[0], rel=1e-13)
    k = np.random.default_rng(3).integers(-1, 2, size=s.pos.shape)
    F2, E2, W2 = oracle.compute(s, pos=s.pos + k * s.box)
    assert E2[0] == pytest.approx(E[0], rel=1e-11)
    np.testing.assert_allclose(F2, F, rtol=0, atol=1e-9 * np.abs(F).max())


def test_cutoff_order_is_validated():
    s = w.two_atoms(5.0).replace(rs_in=6.5, rs_out=6.0)
    with pytest.raises(ValueError):
        oracle.setup_table(s)


# ----------------------------------------------------------------------------
# the FG/CG energy split (reported as energy[1], energy[2]) against closed
# forms: Eq. 17 for f_s-^FG and f_c-^CG, the corrected Eq. 18 for f_s+^CG and
# Eq. 19 for Gamma_c-; none of these goes through the oracle's solver
# ----------------------------------------------------------------------------

def _split_reference(eps_fg, sig_fg, eps_cg, sig_cg, cut, r, shift=True):
    """Closed-form FG and CG parts of Eq. 20 at distance r (one pair).

    FG part: u_FG(r) - f_s-(Dr_s) below r_s-, f_s-(d) - f_s-(Dr_s) on
    [r_s-, r_s+), 0 beyond.  CG part (zero for pairs with an ordinary site,
    Eq. 14): gamma_0+ - Gamma_c- below r_s-, f_s+(d) - Gamma_c- on
    [r_s-, r_s+), u_CG(r) - Gamma_c- on [r_s+, r_c-), f_c-(d) - Gamma_c- on
    [r_c-, r_c+), 0 beyond; under shift no the last two subtract nothing.
    """
    rsi, rso, rci, rco = cut
    Ds, Dc = rso - rsi, rco - rci
    fs = eq17(lj_sym(eps_fg, sig_fg, rsi), Ds)
    fs_end = polyval(fs, Ds)
    if r < rsi:
        efg = lj_sym(eps_fg, sig_fg, r)[0] - fs_end
    elif r < rso:
        efg = polyval(fs, r - rsi) - fs_end
    else:
        efg = 0.0
    if eps_cg == 0.0:
        return efg, 0.0
    sp = eq18(lj_sym(eps_cg, sig_cg, rso), Ds)
    cm = eq17(lj_sym(eps_cg, sig_cg, rci), Dc)
    gam_c = polyval(cm, Dc)
    g_out = gam_c if shift else 0.0
    if r < rsi:
        ecg = sp[0] - gam_c
    elif r < rso:
        ecg = polyval(sp, r - rsi) - gam_c
    elif r < rci:
        ecg = lj_sym(eps_cg, sig_cg, r)[0] - g_out
    elif r < rco:
        ecg = polyval(cm, r - rci) - g_out
    else:
        ecg = 0.0
    return efg, ecg


# distances inside every zone of Eq. 20, plus points next to each boundary
_SPLIT_R = (3.1, 4.4, 5.49, 5.5, 5.62, 5.8, 5.99, 6.0, 6.7, 9.5, 11.99, 12.0, 12.6, 13.4, 13.99,
            14.0, 15.5)


@pytest.mark.parametrize("shift", [True, False])
def test_energy_split_matches_closed_forms_per_zone(shift):
    s = w.propane_liquid(0).replace(shift=shift)
    tab = oracle.setup_table(s)
    cut = (s.rs_in, s.rs_out, s.rc_in, s.rc_out)
    r = np.array(_SPLIT_R)
    for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        e_fg = np.sqrt(s.eps_fg[a] * s.eps_fg[b])
        s_fg = np.sqrt(s.sig_fg[a] * s.sig_fg[b])
        hyb = s.eps_cg[a] > 0 and s.eps_cg[b] > 0
        e_cg = np.sqrt(s.eps_cg[a] * s.eps_cg[b]) if hyb else 0.0
        s_cg = np.sqrt(s.sig_cg[a] * s.sig_cg[b]) if hyb else 0.0
        u, _, which, efg, ecg = oracle.pair(tab[a, b], r)
        for k, x in enumerate(r):
            rf, rc = _split_reference(e_fg, s_fg, e_cg, s_cg, cut, x, shift)
            scale = max(1.0, abs(rf), abs(rc))
            assert abs(efg[k] - rf) <= 1e-12 * scale, (a, b, x, efg[k], rf)
            assert abs(ecg[k] - rc) <= 1e-12 * scale, (a, b, x, ecg[k], rc)
        # a pair with an ordinary site carries no CG energy anywhere (Eq. 14)
        if not hyb:
            assert np.all(ecg == 0.0)
        # from r_s+ on the FG part is gone and the CG part is all of Eq. 20
        beyond = r >= s.rs_out
        assert np.all(efg[beyond] == 0.0)
        np.testing.assert_array_equal(ecg[beyond], u[beyond])


def test_energy_split_constant_below_rs_minus():
    """Below r_s- the CG part is the constant gamma_0+ - Gamma_c- (no force):
    the same value at every distance, and the FG part alone carries the
    textbook LJ shape there."""
    s = w.propane_liquid(0)
    rec = oracle.setup_table(s)[1, 1]
    r = np.linspace(2.8, s.rs_in - 1e-9, 40)
    u, du, which, efg, ecg = oracle.pair(rec, r)
    assert np.all(which == 1)
    assert np.ptp(ecg) == 0.0
    sp0 = eq18(lj_sym(1.0, 4.6, s.rs_out), s.rs_out - s.rs_in)[0]
    gam_c = polyval(eq17(lj_sym(1.0, 4.6, s.rc_in), s.rc_out - s.rc_in), s.rc_out - s.rc_in)
    assert ecg[0] == pytest.approx(sp0 - gam_c, rel=1e-12)
    ref = np.array([lj_sym(0.195, 3.75, x)[0] for x in r])
    np.testing.assert_allclose(efg - efg[0], ref - ref[0], rtol=0, atol=1e-12 * np.abs(ref).max())


def test_energy_split_reference_limit_has_no_cg_part():
    """The reference system (Sec. 2.1; r_s -> r_c, no CG interaction) puts the
    whole energy into the FG part, in every pair and in the system total."""
    s = w.propane_liquid(0).conventional()
    tab = oracle.setup_table(s)
    r = np.array([3.3, 6.0, 11.0, 12.5, 13.9, 14.2])
    for a in range(s.ntypes):
        for b in range(s.ntypes):
            u, _, _, efg, ecg = oracle.pair(tab[a, b], r)
            assert np.all(ecg == 0.0)
            np.testing.assert_array_equal(efg, u)
    sub = w.random_molecules(4, 60, 30.0, kind="propane", min_dist=2.9).conventional()
    F, E, W = oracle.compute(sub)
    assert E[2] == 0.0 and E[1] == E[0]
