"""relres_forces_noalloc, the entry point for callers that cannot allocate:
the same forces, energy and virial as relres_forces (bit for bit: the same
kernels in the same order), on two calls in a row with the second on a
smaller system, through the C ABI, with its static scratch shared by every
context on the GPU; and its refusals (scratch too small, energy/virial of
several systems)."""
import numpy as np
import pytest

import workloads as w
from _util import make_relres

pytestmark = pytest.mark.gpu


def _check_equal(rr, p, ew=True):
    import torch
    F1, E1, W1 = rr.forces(p, want_energy=ew, want_virial=ew)
    F2 = torch.full_like(F1, 7.0)
    E2 = torch.full_like(E1, 7.0) if ew else None
    W2 = torch.full_like(W1, 7.0) if ew else None
    rr.forces_noalloc(p, F2, E2, W2)
    torch.cuda.synchronize()
    assert torch.equal(F1, F2)
    if ew:
        assert torch.equal(E1, E2) and torch.equal(W1, W2)
        assert torch.all(torch.isfinite(E2)) and torch.all(torch.isfinite(W2))
    return F2, E2, W2


def test_noalloc_equals_relres_forces_on_two_calls():
    import torch
    big = w.neopentane_liquid(0)               # 20480 atoms, FP32 forces
    small = w.propane_liquid(0)                # 1500 atoms, FP64 forces
    print(f"[noalloc] N={big.n} then N={small.n}", flush=True)
    rb = make_relres(big)
    pb = torch.from_numpy(big.pos).cuda()
    rb.build_lists(pb, big.box)
    rs = make_relres(small)
    ps = torch.from_numpy(small.pos).cuda()
    rs.build_lists(ps, small.box)
    _check_equal(rb, pb)
    _check_equal(rs, ps)                       # second call, smaller input
    # the scratch keeps the last call's records: calls alternate safely
    for _ in range(3):
        _check_equal(rb, pb)
        _check_equal(rs, ps)
    _check_equal(rs, ps, ew=False)
    rb.close()
    rs.close()


def test_noalloc_refusals():
    import torch
    from paper_2104_10231_amd.relres import RelResError
    s = w.propane_liquid(0, n_mol=23000)       # 69000 atoms
    rr = make_relres(s, 32)
    rr.set_launch(64, 64)                      # ~23000 blocks of records: beyond the array
    p = torch.from_numpy(s.pos).cuda()
    rr.build_lists(p, s.box)
    F = torch.empty((s.n, 3), dtype=torch.float32, device="cuda")
    E = torch.empty(3, dtype=torch.float64, device="cuda")
    with pytest.raises(RelResError):
        rr.forces_noalloc(p, F, E, None)
    F1 = rr.forces(p, want_energy=False, want_virial=False)[0]
    rr.forces_noalloc(p, F)                    # forces only need no scratch
    torch.cuda.synchronize()
    assert torch.equal(F, F1)
    rr.close()
    # several systems: energy/virial need per-row context buffers
    b = w.replica_batch(1, n_systems=3, min_atoms=300, max_atoms=600, total_atoms=1500)
    rb = make_relres(b.whole, 32)
    rb.set_systems(b.offsets)
    pb = torch.from_numpy(b.whole.pos).cuda()
    rb.build_lists(pb, b.boxes)
    Fb = torch.empty((b.whole.n, 3), dtype=torch.float32, device="cuda")
    Eb = torch.empty((b.nsys, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(RelResError):
        rb.forces_noalloc(pb, Fb, Eb, None)
    rb.forces_noalloc(pb, Fb)
    torch.cuda.synchronize()
    assert torch.equal(Fb, rb.forces(pb, want_energy=False, want_virial=False)[0])
    rb.close()
