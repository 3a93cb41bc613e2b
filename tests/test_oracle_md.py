"""Pins of the oracle's molecular-dynamics pieces (Sec. 3.2): bonded terms,
scaled 1-4 pairs and the Nose-Hoover velocity-Verlet integrator.

Independent references:
  * textbook energies at constructed geometries: K (r - r0)^2 for a stretched
    bond, K (theta - theta0)^2 for a bent angle, K (1 + cos 3 phi) for chains
    built with a chosen dihedral (the builder and the oracle's measured
    dihedral agree);
  * forces against central finite differences of each energy, Newton's third
    law, the bonded virial against strain derivatives;
  * the 1-4 pairs at scale 1 equal the change of the non-bonded energy and
    forces when the 1-4 pairs are removed from the exclusions (a different
    path through the oracle), and scale linearly;
  * the integrator: with no thermostat coupling (tau -> infinity) K + U is
    conserved to O(dt^2); with the thermostat the extended energy is
    conserved; running forward, reversing v and xi, and running again
    returns to the start (time reversibility of the symmetric splitting);
    halving dt quarters the energy error.
"""
import numpy as np
import pytest

import oracle
import workloads as w


def _hexane(n_mol=60, seed=1, jiggle=0.08):
    s = w.hexane_liquid(seed, n_mol=n_mol, density=0.012)
    rng = np.random.default_rng(seed + 100)
    return s.replace(pos=s.pos + rng.normal(scale=jiggle, size=s.pos.shape))


def _single_chain(dihedrals, box=60.0):
    """One hexane chain in a large box (no pair within r_c+ of another chain)."""
    s = w.hexane_liquid(0, n_mol=1, density=6 / box ** 3)
    x = w.chain_positions(6, dihedrals) + box / 2
    return s.replace(pos=x, box=np.full(3, box))


# ----------------------------------------------------------------------------
# bonded terms
# ----------------------------------------------------------------------------

def test_textbook_energies_at_constructed_geometries():
    b = w.hexane_liquid(0, n_mol=1).bonded
    K_d = b["dih_k"][0]
    for phi, want in ((np.pi, 0.0), (np.pi / 3, 0.0), (-np.pi / 3, 0.0), (np.pi / 2, K_d),
                      (2.0, K_d * (1 + np.cos(6.0)))):
        s = _single_chain([np.pi, phi, np.pi])
        x = s.pos
        assert abs(abs(oracle.dihedral_angle(x[1], x[2], x[3], x[4], s.box)) - abs(phi)) < 1e-12
        _, E, _ = oracle.bonded(s)
        assert E[0] == pytest.approx(0.0, abs=1e-20) and E[1] == pytest.approx(0.0, abs=1e-20)
        assert E[2] == pytest.approx(want, rel=1e-12, abs=1e-12)
    # a stretched bond and a bent angle
    s = _single_chain([np.pi] * 3)
    x = s.pos.copy()
    u = (x[0] - x[1]) / np.linalg.norm(x[0] - x[1])
    x[0] = x[1] + u * (b["bond_r0"][0] + 0.05)
    # moving atom 0 along its bond keeps every angle and dihedral
    _, E, _ = oracle.bonded(s.replace(pos=x))
    assert E[0] == pytest.approx(b["bond_k"][0] * 0.05 ** 2, rel=1e-12)
    assert E[1] == pytest.approx(0.0, abs=1e-18)
    th = b["angle_t0"][0] + 0.1
    y = w.chain_positions(3, [], angle=th) + 30.0
    s3 = s.replace(pos=np.vstack([y, x[3:]]))     # atoms 0-2 form the bent angle
    b3 = dict(b, bonds=b["bonds"][:2], bond_k=b["bond_k"][:2], bond_r0=b["bond_r0"][:2],
              angles=b["angles"][:1], angle_k=b["angle_k"][:1], angle_t0=b["angle_t0"][:1],
              dihedrals=b["dihedrals"][:0], dih_k=b["dih_k"][:0], dih_n=b["dih_n"][:0],
              dih_d=b["dih_d"][:0])
    _, E, _ = oracle.bonded(s3.replace(bonded=b3))
    assert E[1] == pytest.approx(b["angle_k"][0] * 0.1 ** 2, rel=1e-10)


@pytest.mark.parametrize("term", ["bonds", "angles", "dihedrals"])
def test_bonded_forces_are_minus_energy_gradient(term):
    s = _hexane()
    b = dict(s.bonded)
    for other in {"bonds", "angles", "dihedrals"} - {term}:
        b[other] = b[other][:0]
    s = s.replace(bonded=b)
    k = ["bonds", "angles", "dihedrals"].index(term)
    F, E, _ = oracle.bonded(s)
    assert E[k] > 0.0
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).max()
    rng = np.random.default_rng(k)
    h = 1e-6
    for flat in rng.choice(3 * s.n, size=30, replace=False):
        i, c = divmod(int(flat), 3)
        p = s.pos.copy(); p[i, c] += h
        Ep = oracle.bonded(s, pos=p)[1][k]
        p[i, c] -= 2 * h
        Em = oracle.bonded(s, pos=p)[1][k]
        fd = -(Ep - Em) / (2 * h)
        assert abs(fd - F[i, c]) <= 1e-6 * max(1.0, abs(F[i, c])), (term, i, c, fd, F[i, c])


def test_bonded_virial_is_minus_strain_derivative():
    s = _hexane(seed=3)
    _, E, W = oracle.bonded(s)
    h = 1e-7
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        Ep = oracle.bonded(s.replace(pos=s.pos * sc, box=s.box * sc))[1].sum()
        sc[a] = 1 - h
        Em = oracle.bonded(s.replace(pos=s.pos * sc, box=s.box * sc))[1].sum()
        assert -(Ep - Em) / (2 * h) == pytest.approx(W[a], rel=1e-5, abs=1e-6)


# ----------------------------------------------------------------------------
# 1-4 pairs
# ----------------------------------------------------------------------------

def test_pairs14_equal_the_pairs_the_exclusions_remove():
    s = _hexane(seed=2)
    b = s.bonded
    # exclusions without the 1-4 pairs
    n = s.n
    partners = [[] for _ in range(n)]
    for a, c in np.vstack([b["bonds"], b["angles"][:, [0, 2]]]):
        partners[a].append(c)
        partners[c].append(a)
    offs = np.zeros(n + 1, np.int32)
    offs[1:] = np.cumsum([len(q) for q in partners])
    idx = np.array([j for q in partners for j in sorted(q)], np.int32)
    s13 = s.replace(excl_offsets=offs, excl_idx=idx)
    F13, E13, W13 = oracle.compute(s13)
    F14x, E14x, W14x = oracle.compute(s)
    one = s.replace(bonded=dict(b, scale14=1.0))
    F1, E1, W1 = oracle.pairs14(one)
    np.testing.assert_allclose(F1, F13 - F14x, rtol=0, atol=1e-10 * np.abs(F13).max())
    np.testing.assert_allclose(E1, E13 - E14x, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(W1, W13 - W14x, rtol=0, atol=1e-9 * np.abs(W13).max())
    Fh, Eh, Wh = oracle.pairs14(s)
    np.testing.assert_allclose(Fh, 0.5 * F1, rtol=1e-15, atol=0)
    np.testing.assert_allclose(Eh, 0.5 * E1, rtol=1e-15, atol=0)


# ----------------------------------------------------------------------------
# integrator
# ----------------------------------------------------------------------------

def _md_start(n_mol=40, seed=5):
    s = _hexane(n_mol=n_mol, seed=seed, jiggle=0.03)
    return s, s.pos.copy(), s.bonded["velocities"].copy()


def test_nve_limit_conserves_energy_to_second_order():
    s, x, v = _md_start()
    drift = []
    for dt in (1.0, 0.5):
        steps = int(round(40 / dt))
        _, _, xi, _, tr = oracle.nvt_run(s, x, v, steps, dt, 290.0, tau=1e12)
        assert abs(xi) < 1e-12
        e = tr[:, 5] + tr[:, :5].sum(axis=1)          # K + U
        drift.append(np.abs(e - e[0]).max())
    # this start is far from equilibrium (K doubles within 40 fs)
    assert drift[0] < 3e-3 * abs(e[0])
    # halving dt reduces the energy fluctuation about four times
    assert 2.5 < drift[0] / drift[1] < 6.0, drift


def test_thermostat_conserves_the_extended_energy():
    s, x, v = _md_start(seed=6)
    err = []
    for dt in (1.0, 0.5):
        steps = int(round(60 / dt))
        _, _, xi, eta, tr = oracle.nvt_run(s, x, v, steps, dt, 400.0, tau=50.0)
        nve = oracle.nvt_run(s, x, v, steps, dt, 400.0, tau=1e12)[4]
        H = tr[:, 6]
        # the thermostat did act: the start is colder than 400 K, so xi turns
        # negative and the velocities are scaled up by exp(-eta), here about
        # 3.7 % (|eta| ~ 0.037); a run without coupling ends about 5 % colder.
        # The final xi alone is no measure (about -6e-4 here): K overshoots
        # towards 400 K and xi is on its way back through zero.
        assert eta < -0.01
        assert tr[-1, 5] > 1.02 * nve[-1, 5]
        err.append(np.abs(H - H[0]).max())
        assert err[-1] < 2e-3 * abs(H[0])
    assert 2.5 < err[0] / err[1] < 6.0, err


def test_integrator_is_time_reversible():
    s, x, v = _md_start(n_mol=30, seed=7)
    x1, v1, xi1, eta1, _ = oracle.nvt_run(s, x, v, 25, 1.0, 350.0, tau=80.0, xi=0.002)
    x2, v2, xi2, _, _ = oracle.nvt_run(s, x1, -v1, 25, 1.0, 350.0, tau=80.0, xi=-xi1)
    assert np.abs(x2 - x).max() < 1e-8
    assert np.abs(-v2 - v).max() < 1e-9
    assert abs(-xi2 - 0.002) < 1e-10
