"""Helpers shared by the tests: adapt a workloads.System to the HIP binding
and compare results with the oracle."""
import numpy as np

import oracle


def make_relres(sys, precision=None, pair_math=0):
    from paper_2104_10231_amd.relres import RelRes
    rr = RelRes(rs_in=sys.rs_in, rs_out=sys.rs_out, rc_in=sys.rc_in, rc_out=sys.rc_out,
                skin=sys.skin, eps_fg=sys.eps_fg, sig_fg=sys.sig_fg, eps_cg=sys.eps_cg,
                sig_cg=sys.sig_cg, mix=sys.mix,
                precision=sys.precision if precision is None else precision,
                pair_math=pair_math, shift=sys.shift, cut_type=sys.cut_type,
                cut_pair=sys.cut_pair)
    has_csr = sys.excl_idx is not None and len(sys.excl_idx) > 0
    rr.set_topology(sys.types, sys.mol, sys.exclude_same_mol,
                    sys.excl_offsets if has_csr else None, sys.excl_idx if has_csr else None)
    return rr


def gpu_run(sys, precision=None, pair_math=0, pos=None, build_pos=None, lanes=None):
    import torch
    rr = make_relres(sys, precision, pair_math)
    if lanes is not None:
        rr.set_launch(*lanes)
    p = torch.from_numpy(np.ascontiguousarray(sys.pos if pos is None else pos)).cuda()
    pb = p if build_pos is None else torch.from_numpy(np.ascontiguousarray(build_pos)).cuda()
    rr.build_lists(pb, sys.box)
    F, E, W = rr.forces(p)
    torch.cuda.synchronize()
    return rr, F.double().cpu().numpy(), E.cpu().numpy(), W.cpu().numpy()


def rel_rms(a, b):
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(a * a)))


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def pair_set(arr):
    return set(map(tuple, np.asarray(arr).tolist()))
