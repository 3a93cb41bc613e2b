"""GPU parity over random small systems (hypothesis; fixed derandomised
examples): 2-64 atoms, 1-3 types with random hybrid flags and LJ parameters,
every mixing rule, empty or finite switching zones, pair_modify shift yes/no,
skins of 0-2 A, boxes just above twice the list radius, random molecules.

Bars: pair sets bit-exact; FP64 forces within 1e-11 and FP32 within 1e-5,
energies and virials within 1e-12 (FP64) and 1e-7 (FP32), each relative to
the larger of the result and the magnitude of the terms summed into it (a
random configuration can cancel its net force or energy almost exactly).
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings

import oracle
from _strategies import term_scales, tiny_systems
from _util import make_relres, pair_set

pytestmark = pytest.mark.gpu

TOL = {64: (1e-11, 1e-12), 32: (1e-5, 1e-7)}
SETTINGS = dict(max_examples=40, deadline=None, derandomize=True, database=None,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


def _check(s, precision):
    import torch
    rr = make_relres(s, precision)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    F, E, W = [t.double().cpu().numpy() for t in rr.forces(p)]
    Fr, Er, Wr = oracle.compute(s)
    for which in (0, 1):
        assert pair_set(rr.pairs(which)) == pair_set(oracle.pairs(s, which)), which
    rr.close()
    fs, es, ws = term_scales(s)
    ftol, etol = TOL[precision]
    assert np.sqrt(np.sum((F - Fr) ** 2)) <= ftol * max(np.sqrt(np.sum(Fr * Fr)), fs, 1e-300)
    for k in range(3):
        assert abs(E[k] - Er[k]) <= etol * max(abs(Er[k]), es, 1e-300), (k, E, Er)
    assert np.abs(W - Wr).max() <= etol * max(np.abs(Wr).max(), ws, 1e-300)


@settings(**SETTINGS)
@given(tiny_systems(precision=64))
def test_random_small_systems_fp64(s):
    print(f"[property] N={s.n} types={s.ntypes} box={s.box.round(2).tolist()}", flush=True)
    _check(s, 64)


@settings(**SETTINGS)
@given(tiny_systems(precision=32))
def test_random_small_systems_fp32(s):
    print(f"[property] N={s.n} types={s.ntypes} box={s.box.round(2).tolist()}", flush=True)
    _check(s, 32)
