"""GPU parity of the adjoint kernel (relres_backward) and the autograd layer
against the oracle's analytic gradient (itself pinned by central differences
in test_oracle_grad.py).

J = e_bar * E + sum_i g_i . F_i with random g and e_bar; gradients with
respect to positions and to the per-type eps/sigma (FG and CG), the latter
carried through the mixing rule by torch.  Bar: FP64 arithmetic on both
sides, sums of O(10^4-10^5) terms with cancellation -> norm-relative error
<= 1e-9 (per-parameter relative error <= 1e-8 or 1e-10 of the gradient scale).
"""
import numpy as np
import pytest

import oracle
import workloads as w
from _util import make_relres

pytestmark = pytest.mark.gpu

PARAMS = ("eps_fg", "sig_fg", "eps_cg", "sig_cg")


def _gpu_grad(s, g, e_bar, precision=64):
    import torch
    from paper_2104_10231_amd.autograd import energy_forces
    rr = make_relres(s, precision)
    pos = torch.from_numpy(s.pos).cuda().requires_grad_(True)
    rr.build_lists(pos.detach(), s.box)
    theta = [torch.tensor(np.asarray(getattr(s, k), np.float64), requires_grad=True) for k in PARAMS]
    F, E = energy_forces(rr, pos, *theta)
    J = e_bar * E + (torch.from_numpy(g).cuda().to(F.dtype) * F).sum()
    J.backward()
    dtheta = np.stack([t.grad.numpy() for t in theta])
    dpos = pos.grad.cpu().numpy()
    rr.close()
    return dtheta, dpos


def _compare(s, seed=0, e_bar=0.9, precision=64):
    print(f"[grad] {s.name} N={s.n} ntypes={s.ntypes} precision={precision}", flush=True)
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(s.n, 3))
    if precision == 32:
        # J multiplies g by FP32 forces, so dJ/dF reaches the kernel rounded
        g = g.astype(np.float32).astype(np.float64)
    dt_ref, dp_ref = oracle.grad(s, g, e_bar)
    dt, dp = _gpu_grad(s, g, e_bar, precision)
    assert np.linalg.norm(dp - dp_ref) <= 1e-9 * np.linalg.norm(dp_ref), \
        np.linalg.norm(dp - dp_ref) / np.linalg.norm(dp_ref)
    scale = np.abs(dt_ref).max()
    for P, name in enumerate(PARAMS):
        for t in range(s.ntypes):
            ref = dt_ref[P, t]
            assert abs(dt[P, t] - ref) <= 1e-8 * abs(ref) + 1e-10 * scale, (name, t, dt[P, t], ref)


def test_propane_1500_gradient():
    _compare(w.propane_liquid(0))


@pytest.mark.parametrize("kind,seed,n_mol,hf", [("propane", 3, 150, 0.8),
                                                 ("neopentane", 5, 61, 0.7),
                                                 ("propane", 6, 130, 0.0)])
def test_small_systems_gradient(kind, seed, n_mol, hf):
    _compare(w.random_molecules(seed, n_mol, 34.0, kind=kind, min_dist=2.9, hybrid_fraction=hf),
             seed=seed)


def test_fp32_context_backward_is_fp64():
    # the backward pass recomputes in FP64 whatever the force precision
    _compare(w.random_molecules(4, 97, 34.0, kind="propane", min_dist=2.9), precision=32)


def test_copolymer_lorentz_berthelot_four_types():
    s = w.copolymer_melt(1, n_chains=16, n_beads=48)
    _compare(s, seed=2, e_bar=-0.4)


def test_six_types_with_csr_exclusions():
    s = w.random_molecules(9, 120, 35.0, kind="neopentane", min_dist=2.9)
    rng = np.random.default_rng(5)
    types = rng.integers(0, 6, size=s.n).astype(np.int32)
    offs, lst = [0], []
    for i in range(s.n):
        lst += [j for j in (i - 1, i + 1) if 0 <= j < s.n and s.mol[j] == s.mol[i]]
        offs.append(len(lst))
    s = s.replace(types=types, exclude_same_mol=False, excl_offsets=np.array(offs, np.int32),
                  excl_idx=np.array(lst, np.int32),
                  eps_fg=rng.uniform(0.05, 0.3, 6), sig_fg=rng.uniform(3.4, 4.0, 6),
                  eps_cg=np.array([0.0, 0.0, 0.0, 1.2, 2.0, 3.1]),
                  sig_cg=np.array([0.0, 0.0, 0.0, 4.2, 4.5, 4.8]))
    _compare(s, seed=3, e_bar=1.7)


def test_energy_only_and_forces_only_objectives():
    s = w.random_molecules(4, 97, 34.0, kind="propane", min_dist=2.9)
    _compare(s, seed=1, e_bar=0.0)                      # forces only
    rng = np.random.default_rng(0)
    dt_ref, dp_ref = oracle.grad(s, np.zeros((s.n, 3)), 1.0)
    dt, dp = _gpu_grad(s, np.zeros((s.n, 3)), 1.0)      # energy only: dp = -F
    assert np.linalg.norm(dp - dp_ref) <= 1e-10 * np.linalg.norm(dp_ref)
    assert np.allclose(dt, dt_ref, rtol=1e-9, atol=1e-12 * np.abs(dt_ref).max())


def test_set_pair_params_equals_a_fresh_context():
    import torch
    s = w.random_molecules(4, 97, 34.0, kind="propane", min_dist=2.9)
    s2 = s.replace(eps_fg=np.array([0.21, 0.08]), sig_fg=np.array([3.7, 4.0]),
                   eps_cg=np.array([0.0, 1.4]), sig_cg=np.array([0.0, 4.4]))
    rr = make_relres(s, 64)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    ef = np.sqrt(np.outer(s2.eps_fg, s2.eps_fg))
    sf = np.sqrt(np.outer(s2.sig_fg, s2.sig_fg))
    ec = np.sqrt(np.outer(s2.eps_cg, s2.eps_cg))
    sc = np.sqrt(np.outer(s2.sig_cg, s2.sig_cg))
    rr.set_pair_params(ef, sf, ec, sc)
    F1, E1, W1 = rr.forces(p)
    r2 = make_relres(s2, 64)
    r2.build_lists(p, s2.box)
    F2, E2, W2 = r2.forces(p)
    assert torch.equal(F1, F2) and torch.equal(E1, E2) and torch.equal(W1, W2)
    rr.close()
    r2.close()


def test_backward_is_bitwise_repeatable():
    import torch
    s = w.propane_liquid(0)
    rr = make_relres(s, 64)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    g = torch.from_numpy(np.random.default_rng(0).normal(size=(s.n, 3))).cuda()
    e = torch.tensor([0.3], dtype=torch.float64, device="cuda")
    a1, b1 = rr.backward(p, g, e)
    a2, b2 = rr.backward(p, g, e)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)
    rr.close()


def test_backward_rejects_more_than_eight_types():
    import torch
    from paper_2104_10231_amd.relres import RelResError
    s = w.random_molecules(4, 30, 34.0, kind="propane", min_dist=2.9)
    s = s.replace(types=(np.arange(s.n) % 9).astype(np.int32), eps_fg=np.full(9, 0.1),
                  sig_fg=np.full(9, 3.8), eps_cg=np.zeros(9), sig_cg=np.zeros(9))
    rr = make_relres(s, 64)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    with pytest.raises(RelResError):
        rr.backward(p, torch.zeros_like(p))
    rr.close()


def test_force_matching_over_perturbed_frames():
    """Loss sum_frames sum_i |F_i(theta) - F_ref,i|^2 with reference forces
    from the oracle at other parameters: its gradient summed over frames."""
    import torch
    from paper_2104_10231_amd.autograd import energy_forces
    base = w.random_molecules(3, 150, 34.0, kind="propane", min_dist=2.9, hybrid_fraction=0.8)
    frames = w.perturbed_frames(base, n_frames=4, sigma=0.05, seed=11)
    ref_params = dict(eps_fg=np.array([0.21, 0.10]), sig_fg=np.array([3.70, 3.90]),
                      eps_cg=np.array([0.0, 1.2]), sig_cg=np.array([0.0, 4.5]))
    print(f"[grad] force matching, {len(frames)} frames of N={base.n}", flush=True)
    rr = make_relres(base, 64)
    theta = [torch.tensor(np.asarray(getattr(base, k), np.float64), requires_grad=True)
             for k in PARAMS]
    dt_ref = np.zeros((4, base.ntypes))
    loss_total = 0.0
    for f in frames:
        Fref, _, _ = oracle.compute(f.replace(**ref_params))
        pos = torch.from_numpy(f.pos).cuda()
        rr.build_lists(pos, f.box)
        F, _ = energy_forces(rr, pos, *theta)
        loss = ((F - torch.from_numpy(Fref).cuda()) ** 2).sum()
        loss.backward()
        loss_total += loss.item()
        Fo, _, _ = oracle.compute(f)
        d, _ = oracle.grad(f, 2.0 * (Fo - Fref), 0.0)
        dt_ref += d
    dt = np.stack([t.grad.numpy() for t in theta])
    scale = np.abs(dt_ref).max()
    assert loss_total > 0.0
    for P in range(4):
        for t in range(base.ntypes):
            assert abs(dt[P, t] - dt_ref[P, t]) <= 1e-8 * abs(dt_ref[P, t]) + 1e-10 * scale, \
                (PARAMS[P], t, dt[P, t], dt_ref[P, t])
    rr.close()


def test_set_type_params_equals_a_fresh_context():
    """relres_set_type_params mixes per-type values inside the library: the
    same forces, energy and virial, bit for bit, as a context created with
    them (both mixing rules that differ in sigma)."""
    import torch
    for mix in (w.MIX_GEOMETRIC, w.MIX_ARITHMETIC, w.MIX_SIXTHPOWER):
        s = w.random_molecules(4, 97, 34.0, kind="propane", min_dist=2.9).replace(mix=mix)
        new = dict(eps_fg=np.array([0.21, 0.08]), sig_fg=np.array([3.7, 4.0]),
                   eps_cg=np.array([0.0, 1.4]), sig_cg=np.array([0.0, 4.4]))
        rr = make_relres(s, 64)
        p = torch.from_numpy(s.pos).cuda()
        rr.build_lists(p, s.box)
        rr.set_type_params(new["eps_fg"], new["sig_fg"], new["eps_cg"], new["sig_cg"])
        F1, E1, W1 = rr.forces(p)
        r2 = make_relres(s.replace(**new), 64)
        r2.build_lists(p, s.box)
        F2, E2, W2 = r2.forces(p)
        assert torch.equal(F1, F2) and torch.equal(E1, E2) and torch.equal(W1, W2), mix
        rr.close()
        r2.close()


def test_type_params_validation_and_pair_table_state():
    import torch
    from paper_2104_10231_amd.relres import RelResError
    s = w.random_molecules(4, 40, 34.0, kind="propane", min_dist=2.9)
    rr = make_relres(s, 64)
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    # the hybrid types define the site list: an ordinary type stays ordinary
    with pytest.raises(RelResError):
        rr.set_type_params(s.eps_fg, s.sig_fg, np.array([0.5, 1.0]), np.array([4.0, 4.6]))
    with pytest.raises(RelResError):
        rr.set_type_params(s.eps_fg, s.sig_fg, np.array([0.0, 0.0]), s.sig_cg)
    gpos, gt = rr.backward_types(p, torch.zeros_like(p), torch.ones(1, dtype=torch.float64))
    assert gt.shape == (4, s.ntypes)
    assert torch.all(gt[2:, 0] == 0.0)          # ordinary type: no CG gradient (Eq. 14)
    # pair tables set directly have no per-type values to differentiate
    ef = np.sqrt(np.outer(s.eps_fg, s.eps_fg))
    sf = np.sqrt(np.outer(s.sig_fg, s.sig_fg))
    ec = np.sqrt(np.outer(s.eps_cg, s.eps_cg))
    sc = np.sqrt(np.outer(s.sig_cg, s.sig_cg))
    rr.set_pair_params(ef, sf, ec, sc)
    with pytest.raises(RelResError):
        rr.backward_types(p, torch.zeros_like(p))
    rr.close()
