"""Property tests of the oracle over random small systems (hypothesis; fixed
derandomised examples so every run checks the same cases):

  * Newton's third law: the forces sum to zero;
  * translation invariance: shifting every atom by one vector (and by whole
    box edges) changes no force and no energy;
  * permutation invariance: renumbering the atoms permutes the forces and
    keeps the energy and virial;
  * forces are -dE/dx by central differences, where Eq. 20 is C2 (finite
    zones, pair_modify shift yes).

Tolerances are relative to the magnitude of the summed terms (sum of |u'|
per atom, sum of |u|), since a random configuration may cancel its net force.
"""
import numpy as np
from hypothesis import HealthCheck, given, settings

import oracle
from _strategies import term_scales, tiny_systems

SETTINGS = dict(max_examples=40, deadline=None, derandomize=True, database=None,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@settings(**SETTINGS)
@given(tiny_systems())
def test_forces_sum_to_zero(s):
    F, E, W = oracle.compute(s)
    fs, es, ws = term_scales(s)
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * max(fs, 1e-300)


@settings(**SETTINGS)
@given(tiny_systems())
def test_translation_invariance(s):
    F, E, W = oracle.compute(s)
    fs, es, ws = term_scales(s)
    rng = np.random.default_rng(s.n)
    shift = rng.uniform(-50.0, 50.0, 3)
    images = rng.integers(-2, 3, size=(s.n, 3)) * s.box
    F2, E2, W2 = oracle.compute(s, pos=s.pos + shift + images)
    assert np.abs(F2 - F).max() <= 1e-10 * max(fs, 1e-300)
    assert abs(E2[0] - E[0]) <= 1e-12 * max(es, 1e-300)
    assert np.abs(W2 - W).max() <= 1e-10 * max(ws, 1e-300)


@settings(**SETTINGS)
@given(tiny_systems())
def test_permutation_invariance(s):
    F, E, W = oracle.compute(s)
    fs, es, ws = term_scales(s)
    perm = np.random.default_rng(s.n + 1).permutation(s.n)
    sp = s.replace(pos=s.pos[perm], types=s.types[perm], mol=s.mol[perm])
    F2, E2, W2 = oracle.compute(sp)
    assert np.abs(F2 - F[perm]).max() <= 1e-12 * max(fs, 1e-300)
    assert abs(E2[0] - E[0]) <= 1e-13 * max(es, 1e-300)
    assert np.abs(W2 - W).max() <= 1e-12 * max(ws, 1e-300)
    # and the pair sets are the same pairs under the renumbering
    for which in (0, 1):
        a = {tuple(sorted((perm[i], perm[j]))) for i, j in oracle.pairs(sp, which).tolist()}
        b = set(map(tuple, oracle.pairs(s, which).tolist()))
        assert a == b


@settings(**SETTINGS)
@given(tiny_systems(max_atoms=24))
def test_forces_are_minus_energy_gradient(s):
    if not (s.rs_out > s.rs_in and s.rc_out > s.rc_in and s.shift):
        return                                  # Eq. 20 is only C0 with an empty zone
    F, E, W = oracle.compute(s)
    fs, es, ws = term_scales(s)
    h = 1e-6
    rng = np.random.default_rng(s.n + 2)
    for flat in rng.choice(3 * s.n, size=min(6, 3 * s.n), replace=False):
        i, c = divmod(int(flat), 3)
        p = s.pos.copy()
        p[i, c] += h
        ep = oracle.compute(s, pos=p)[1][0]
        p[i, c] -= 2 * h
        em = oracle.compute(s, pos=p)[1][0]
        fd = -(ep - em) / (2 * h)
        assert abs(fd - F[i, c]) <= 1e-6 * max(fs, 1.0) + 1e-9 * es, (i, c, fd, F[i, c])
