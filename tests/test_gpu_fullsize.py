"""Oracle parity at the full sizes of the batching and differentiation
workloads, in the launch configuration the benchmark times.

  * 256 replicas of 300-18000 atoms (1.2 M atoms, per-replica skins of 2.0 A,
    1.5 A in the smallest boxes) in one context with the automatic kernel
    shapes: eight replicas spanning the range (smallest and largest, the
    smallest boxes, and sizes in between) against the oracle one by one --
    forces, energy and virial of the replica, and both pair sets bit-exact;
  * the 20480-atom neopentane liquid, two of its 64 frames perturbed by
    0.05 A Gaussian noise: the gradients of the energy and of the force-
    matching loss sum |F - F_ref|^2 (F_ref from the oracle at perturbed
    parameters) with respect to positions and per-type eps/sigma, from an
    FP32 forward context, against the oracle's analytic gradient (itself
    pinned by central differences in test_oracle_grad.py).
Bars as elsewhere: FP32 forces 1e-5 relative RMS, energy/virial 1e-7; FP64
adjoint 1e-9 (positions, norm-relative) and 1e-8 per parameter.
"""
import numpy as np
import pytest

import oracle
import workloads as w
from _util import make_relres, rel_rms

pytestmark = pytest.mark.gpu

PARAMS = ("eps_fg", "sig_fg", "eps_cg", "sig_cg")


def _pairs_of(all_pairs, o0, o1):
    """Pairs of one replica (its atoms are [o0, o1)), in replica indices,
    canonical (i < j) and sorted as the library returns them."""
    sel = (all_pairs[:, 0] >= o0) & (all_pairs[:, 0] < o1)
    p = all_pairs[sel] - o0
    assert np.all((p[:, 1] >= 0) & (p[:, 1] < o1 - o0)), "a pair crosses replicas"
    return p


def test_replica_batch_256_full_size():
    import torch
    b = w.replica_batch(0, skin_max=2.0)
    n = b.whole.n
    print(f"[fullsize] batch of {b.nsys} replicas, N={n}", flush=True)
    rr = make_relres(b.whole, 32)
    rr.set_systems(b.offsets)
    rr.set_skins(b.skins)
    p = torch.from_numpy(b.whole.pos).cuda()
    rr.build_lists(p, b.boxes)
    F, E, W = rr.forces(p)
    torch.cuda.synchronize()
    F = F.double().cpu().numpy()
    E = E.cpu().numpy()
    W = W.cpu().numpy()
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(E)) and np.all(np.isfinite(W))
    # forces only: rows of at least 8 list entries per lane (this batch's
    # automatic lane split) take the force kernel's 4-entry batches
    st = rr.stats()
    assert st["atom_entries"] / n >= 16, st                 # 8 per lane at 2 lanes per row
    F0, _, _ = rr.forces(p, energy=None, virial=None, want_energy=False, want_virial=False)
    F0 = F0.double().cpu().numpy()
    sizes = np.diff(b.offsets)
    order = np.argsort(sizes, kind="stable")
    small_box = int(np.argmin([s.box[0] for s in b.systems]))
    pick = []
    for k in [int(order[0]), int(order[-1]), small_box, int(np.argmin(b.skins))] + \
             [int(order[int(q * (b.nsys - 1))]) for q in (0.15, 0.3, 0.45, 0.6, 0.75, 0.9)]:
        if k not in pick and len(pick) < 8:
            pick.append(k)
    assert b.skins.min() < b.skins.max()              # both skins are present
    pa, ps = rr.pairs(0), rr.pairs(1)
    for k in pick:
        s = b.systems[k]
        o0, o1 = int(b.offsets[k]), int(b.offsets[k + 1])
        print(f"[fullsize] replica {k}: N={s.n}, box {s.box[0]:.2f} A, skin {s.skin}", flush=True)
        Fr, Er, Wr = oracle.compute(s)
        assert rel_rms(F[o0:o1], Fr) <= 1e-5, (k, rel_rms(F[o0:o1], Fr))
        assert rel_rms(F0[o0:o1], Fr) <= 1e-5, (k, rel_rms(F0[o0:o1], Fr))
        assert abs(E[k, 0] - Er[0]) <= 1e-7 * abs(Er[0]), (k, E[k], Er)
        assert np.abs(W[k] - Wr).max() <= 1e-7 * np.abs(Wr).max(), (k, W[k], Wr)
        for which, got in ((0, pa), (1, ps)):
            ref = oracle.pairs(s, which)
            mine = _pairs_of(got, o0, o1)
            assert mine.shape == ref.shape and np.array_equal(mine, ref), (k, which)
    rr.close()


@pytest.mark.parametrize("frame", [0, 37])
def test_gradients_20480_atom_frames(frame):
    import torch
    from paper_2104_10231_amd.autograd import energy_forces
    s = w.neopentane_liquid(0)
    f = w.perturbed_frames(s, n_frames=64, sigma=0.05, seed=1)[frame]
    ref = dict(eps_fg=s.eps_fg * 1.03, sig_fg=s.sig_fg * 0.99, eps_cg=s.eps_cg * 1.05,
               sig_cg=s.sig_cg * 1.01)
    print(f"[fullsize] gradient frame {frame}, N={f.n}", flush=True)
    Fref = oracle.compute(f.replace(**ref))[0]
    rr = make_relres(s, 32)
    pos = torch.from_numpy(f.pos).cuda().requires_grad_(True)
    rr.build_lists(pos.detach(), f.box)
    theta = [torch.tensor(np.asarray(getattr(s, k), np.float64), requires_grad=True)
             for k in PARAMS]
    F, E = energy_forces(rr, pos, *theta)
    L = ((F.double() - torch.from_numpy(Fref).cuda()) ** 2).sum()
    gL = torch.autograd.grad(L, theta + [pos], retain_graph=True)
    gE = torch.autograd.grad(E, theta + [pos])
    Fg = F.detach().double().cpu().numpy()
    rr.close()
    # the kernel receives dL/dF rounded to the FP32 forces' type
    g = (2.0 * (Fg - Fref)).astype(np.float32).astype(np.float64)
    for got, (gg, eb) in ((gL, (g, 0.0)), (gE, (np.zeros_like(g), 1.0))):
        dt_ref, dp_ref = oracle.grad(f, gg, eb)
        dt = np.stack([t.numpy() for t in got[:4]])
        dp = got[4].cpu().numpy()
        assert np.linalg.norm(dp - dp_ref) <= 1e-9 * np.linalg.norm(dp_ref), \
            np.linalg.norm(dp - dp_ref) / np.linalg.norm(dp_ref)
        scale = np.abs(dt_ref).max()
        for P in range(4):
            for t in range(s.ntypes):
                assert abs(dt[P, t] - dt_ref[P, t]) <= 1e-8 * abs(dt_ref[P, t]) + 1e-10 * scale, \
                    (PARAMS[P], t, dt[P, t], dt_ref[P, t])
