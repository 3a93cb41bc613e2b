"""GPU parity of the molecular model (Sec. 3.2) against the oracle: bonded
terms and scaled 1-4 pairs (relres_bonded_forces), and Nose-Hoover
velocity-Verlet trajectories (relres_md_run).

Bars: bonded forces, energies and virial are FP64 on both sides (1e-11
relative RMS for forces, 1e-12 for energies and virial); FP32 contexts add
the FP64 bonded forces to FP32 forces (1e-5).  Trajectories: 20 steps of
1 fs with FP64 forces, positions and velocities within 1e-9 relative (the
per-step rounding differences, ~1e-15, grow by the system's instability;
measured growth over 20 steps stays below 1e3), thermostat variables and
per-step energies likewise.
"""
import numpy as np
import pytest

import oracle
import workloads as w
from _util import make_relres, rel_rms

pytestmark = pytest.mark.gpu


def _hexane(n_mol=120, seed=1, jiggle=0.05, precision=64):
    s = w.hexane_liquid(seed, n_mol=n_mol, density=0.012, precision=precision)
    rng = np.random.default_rng(seed + 100)
    return s.replace(pos=s.pos + rng.normal(scale=jiggle, size=s.pos.shape))


def _ctx(s, precision=64):
    import torch
    rr = make_relres(s, precision)
    rr.set_bonded(s.bonded)
    p = torch.from_numpy(np.ascontiguousarray(s.pos)).cuda()
    rr.build_lists(p, s.box)
    return rr, p


@pytest.mark.parametrize("precision", [64, 32])
def test_bonded_and_14_forces(precision):
    import torch
    s = _hexane(precision=precision)
    print(f"[md] bonded forces N={s.n} precision={precision}", flush=True)
    rr, p = _ctx(s, precision)
    dt = torch.float64 if precision == 64 else torch.float32
    F = torch.zeros((s.n, 3), dtype=dt, device="cuda")
    E, W = rr.bonded_forces(p, F)
    torch.cuda.synchronize()
    Fb, Eb, Wb = oracle.bonded(s)
    F14, E14, W14 = oracle.pairs14(s)
    Fr = Fb + F14
    ftol = 1e-11 if precision == 64 else 1e-5
    assert rel_rms(F.double().cpu().numpy(), Fr) <= ftol
    E = E.cpu().numpy()
    want = np.array([Eb[0], Eb[1], Eb[2], E14[0]])
    np.testing.assert_allclose(E, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    Wr = Wb + W14
    assert np.abs(W.cpu().numpy() - Wr).max() <= 1e-12 * np.abs(Wr).max()
    rr.close()


def test_all_forces_of_the_model():
    import torch
    s = _hexane(seed=2)
    rr, p = _ctx(s)
    F, E, W = rr.forces(p)
    Eb, Wb = rr.bonded_forces(p, F)
    torch.cuda.synchronize()
    Fr, Ur, Wr = oracle.md_forces(s, s.pos)
    assert rel_rms(F.cpu().numpy(), Fr) <= 1e-11
    assert abs(E[0].item() - Ur[0]) <= 1e-12 * abs(Ur[0])
    Wt = W.cpu().numpy() + Wb.cpu().numpy()
    assert np.abs(Wt - Wr).max() <= 1e-12 * np.abs(Wr).max()
    rr.close()


def _gpu_run(s, steps, dt, T, tau, rebuild_every=10, thermo_every=1, xi=0.0, eta=0.0):
    import torch
    rr, p = _ctx(s)
    v = torch.from_numpy(np.ascontiguousarray(s.bonded["velocities"])).cuda()
    rr.md_setup(s.bonded["masses"], dt, T, tau, rebuild_every=rebuild_every)
    if xi or eta:
        rr.md_state(xi, eta)
    th = rr.md_run(p, v, steps, thermo_every)
    torch.cuda.synchronize()
    xi1, eta1 = rr.md_state()
    out = (p.cpu().numpy(), v.cpu().numpy(), xi1, eta1, None if th is None else th.cpu().numpy())
    rr.close()
    return out


@pytest.mark.parametrize("tau", [100.0, 1e12])
def test_trajectory_matches_the_oracle(tau):
    s = _hexane(n_mol=100, seed=3, jiggle=0.03)
    steps, dt, T = 20, 1.0, 300.0
    print(f"[md] trajectory N={s.n} steps={steps} tau={tau}", flush=True)
    x, v, xi, eta, th = _gpu_run(s, steps, dt, T, tau)
    xr, vr, xir, etar, tr = oracle.nvt_run(s, s.pos, s.bonded["velocities"], steps, dt, T, tau)
    assert np.abs(x - xr).max() <= 1e-9 * np.abs(xr).max()
    assert rel_rms(v, vr) <= 1e-9
    assert abs(xi - xir) <= 1e-9 * max(abs(xir), 1e-6)
    assert abs(eta - etar) <= 1e-9 * max(abs(etar), 1e-6)
    # per-step energies: non-bonded, 1-4, bonds, angles, dihedrals, K, extended
    assert th.shape == (steps, 8)
    for k in range(7):
        scale = max(np.abs(tr[:, k]).max(), 1e-9)
        assert np.abs(th[:, k] - tr[:, k]).max() <= 1e-9 * scale, k


def test_runs_are_bitwise_repeatable_and_resumable():
    s = _hexane(n_mol=80, seed=4, jiggle=0.03)
    a = _gpu_run(s, 12, 1.0, 300.0, 100.0)
    b = _gpu_run(s, 12, 1.0, 300.0, 100.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    # 12 steps = 5 + 7 steps when the second run starts from the first's state
    h = _gpu_run(s, 5, 1.0, 300.0, 100.0)
    t = _gpu_run(s.replace(pos=h[0], bonded=dict(s.bonded, velocities=h[1])), 7, 1.0, 300.0,
                 100.0, xi=h[2], eta=h[3])
    assert np.abs(t[0] - a[0]).max() <= 1e-12 * np.abs(a[0]).max()
    assert rel_rms(t[1], a[1]) <= 1e-11


def test_stale_lists_are_reported():
    """A skin of 0.05 A with builds every 40 steps: atoms outrun half the
    skin and the run reports it instead of using stale lists silently."""
    import torch
    from paper_2104_10231_amd.relres import RelResError, RELRES_ERR_STALE_LISTS
    s = _hexane(n_mol=60, seed=5).replace(skin=0.05)
    rr, p = _ctx(s)
    v = torch.from_numpy(np.ascontiguousarray(s.bonded["velocities"])).cuda()
    rr.md_setup(s.bonded["masses"], 1.0, 300.0, 100.0, rebuild_every=40)
    with pytest.raises(RelResError) as e:
        rr.md_run(p, v, 40)
    assert e.value.code == RELRES_ERR_STALE_LISTS
    rr.close()


def test_new_topology_drops_bonded_terms():
    """Bonded terms refer to atoms of one topology: a new topology drops them
    (and the integrator setup) instead of reading tables of the old size."""
    import torch
    from paper_2104_10231_amd.relres import RelResError
    s = _hexane(n_mol=80, seed=6)
    rr, p = _ctx(s)
    small = w.hexane_liquid(7, n_mol=40, density=0.012)
    rr.set_topology(small.types, small.mol, False, small.excl_offsets, small.excl_idx)
    ps = torch.from_numpy(small.pos).cuda()
    rr.build_lists(ps, s.box)
    F = torch.zeros((small.n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(RelResError):
        rr.bonded_forces(ps, F)
    with pytest.raises(RelResError):
        rr.md_run(ps, torch.zeros_like(ps), 1)
    rr.close()
