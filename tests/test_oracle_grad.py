"""Pins of the oracle's analytic gradient (CPU).

The oracle differentiates Eqs. 7-9 and 20 analytically (the boundary systems
of Eqs. 7/8 are linear, so the coefficient derivatives solve the same systems
with differentiated right-hand sides).  These tests check it against what the
mathematics fixes independently of that derivation:
  * central finite differences of the oracle's own energy and forces, with
    respect to every per-type parameter and to positions;
  * linearity in epsilon: dE/d eps_FG = E / eps_FG for a single-type FG system;
  * a pair that is not hybrid-hybrid does not depend on CG parameters (Eq. 14).
"""
import numpy as np
import pytest

import oracle
import workloads as w

PARAMS = ("eps_fg", "sig_fg", "eps_cg", "sig_cg")


def _objective(s, g, e_bar, pos=None):
    F, E, _ = oracle.compute(s, pos=pos)
    return e_bar * E[0] + float(np.sum(g * F))


def _system(seed=3, mix=0):
    # propane-like molecules in a 26 A box: pairs in every regime of Eq. 20,
    # two types (ordinary CH3, hybrid CH2) with distinct FG parameters
    s = w.random_molecules(seed, 40, 36.0, kind="propane", min_dist=2.9)
    s = s.replace(eps_fg=np.array([0.195, 0.091]), sig_fg=np.array([3.75, 3.95]),
                  eps_cg=np.array([0.0, 1.0]), sig_cg=np.array([0.0, 4.6]), mix=mix)
    return s


def _variant(name):
    """Pair-style options of Sec. 2.5: mixing rules, shift no, distances per
    type (mixed for the unlike pair)."""
    if name == "geometric":
        return _system(mix=0)
    if name == "lorentz_berthelot":
        return _system(mix=1)
    if name == "sixthpower":
        return _system(mix=2)
    if name == "shift_no":
        return _system().replace(shift=False)
    if name == "per_type_distances":
        return _system().replace(cut_type=np.array([[5.3, 5.8, 11.5, 13.5],
                                                    [6.4, 6.9, 12.0, 14.0]]))
    raise ValueError(name)


VARIANTS = ["geometric", "lorentz_berthelot", "sixthpower", "shift_no", "per_type_distances"]


@pytest.mark.parametrize("variant", VARIANTS)
def test_parameter_gradient_matches_central_differences(variant):
    s = _variant(variant)
    rng = np.random.default_rng(7)
    g = rng.normal(size=(s.n, 3))
    e_bar = 0.7
    dtheta, _ = oracle.grad(s, g, e_bar)
    for P, name in enumerate(PARAMS):
        vals = np.asarray(getattr(s, name), float)
        for t in range(s.ntypes):
            if P >= 2 and vals[t] == 0.0:
                assert dtheta[P, t] == 0.0          # ordinary type: no CG pair
                continue
            h = 1e-6 * vals[t]
            hi, lo = vals.copy(), vals.copy()
            hi[t] += h
            lo[t] -= h
            fd = (_objective(s.replace(**{name: hi}), g, e_bar) -
                  _objective(s.replace(**{name: lo}), g, e_bar)) / (2 * h)
            assert abs(dtheta[P, t] - fd) <= 1e-6 * max(abs(fd), 1e-3), (name, t, dtheta[P, t], fd)


@pytest.mark.parametrize("variant", ["geometric", "sixthpower", "per_type_distances"])
def test_position_gradient_matches_central_differences(variant):
    s = _variant(variant)
    rng = np.random.default_rng(11)
    g = rng.normal(size=(s.n, 3))
    e_bar = -1.3
    _, dpos = oracle.grad(s, g, e_bar)
    h = 1e-6
    for i in rng.choice(s.n, 6, replace=False):
        for c in range(3):
            p1, p0 = s.pos.copy(), s.pos.copy()
            p1[i, c] += h
            p0[i, c] -= h
            fd = (_objective(s, g, e_bar, pos=p1) - _objective(s, g, e_bar, pos=p0)) / (2 * h)
            assert abs(dpos[i, c] - fd) <= 1e-6 * max(abs(fd), 1e-2), (i, c, dpos[i, c], fd)


def test_energy_is_linear_in_epsilon():
    # one type, no hybrid atoms: E is exactly eps_FG times a function of sigma
    s = _system().replace(types=np.zeros(120, np.int32)[: _system().n],
                          eps_fg=np.array([0.3]), sig_fg=np.array([3.8]),
                          eps_cg=np.array([0.0]), sig_cg=np.array([0.0]))
    _, E, _ = oracle.compute(s)
    dtheta, dpos = oracle.grad(s, np.zeros((s.n, 3)), 1.0)
    assert abs(dtheta[0, 0] - E[0] / 0.3) <= 1e-12 * abs(E[0] / 0.3)
    F, _, _ = oracle.compute(s)
    assert np.allclose(dpos, -F, rtol=0, atol=1e-12 * np.abs(F).max())


def test_energy_gradient_with_respect_to_positions_is_minus_the_force():
    s = _system()
    F, _, _ = oracle.compute(s)
    _, dpos = oracle.grad(s, np.zeros((s.n, 3)), 1.0)
    assert np.allclose(dpos, -F, rtol=0, atol=1e-12 * np.abs(F).max())
