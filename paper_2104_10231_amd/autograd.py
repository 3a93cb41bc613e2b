"""Differentiable RelRes energy and forces (torch.autograd over the C ABI).

``energy_forces(rr, pos, eps_fg, sig_fg, eps_cg, sig_cg)`` returns the forces
(N, 3) and the total energy of Eq. 3 as tensors that carry gradients to the
positions and to the per-type FG/CG Lennard-Jones parameters.  The forward
pass is ``relres_forces`` on the pair parameters mixed here with torch
operations (Sec. 2.3: geometric means, Lorentz-Berthelot or the sixth-power
rule of pair_modify mix; CG parameters only for hybrid-hybrid pairs, Eq. 14),
so torch carries the
gradient through the mixing rule; the backward pass is ``relres_backward``,
a HIP kernel that recomputes every pair term in FP64 and returns dJ/dx and
dJ/d(pair parameter) for J = e_bar E + sum_i g_i . F_i.  Any loss of the
energy and forces works, e.g. force matching sum_i |F_i - F_ref,i|^2.

The context's pair parameters are the ones of the most recent forward call;
the backward pass re-installs the parameters of its own forward call if they
changed since.
"""
from __future__ import annotations

import torch

from .relres import RelRes

__all__ = ["mix_pair_tables", "energy_forces"]


def _mix(eps, sig, mix: int, mask=None):
    """Mixed (eps_ab, sigma_ab) tables of one family (FG or CG) under the
    pair_modify mix rule: geometric (0), Lorentz-Berthelot (1) or sixth-power
    (2).  Entries outside ``mask`` are zero and never enter a square root or
    a division, so ordinary types (eps_CG = 0) get no infinite gradients."""
    one = torch.ones((), dtype=eps.dtype, device=eps.device)
    zero = torch.zeros((), dtype=eps.dtype, device=eps.device)
    m = torch.ones((eps.shape[0], eps.shape[0]), dtype=torch.bool, device=eps.device) \
        if mask is None else mask
    ee = torch.where(m, eps[:, None] * eps[None, :], one)
    if mix == 2:
        s3 = sig ** 3
        s6 = torch.where(m, s3[:, None] ** 2 + s3[None, :] ** 2, one)
        e = torch.where(m, 2.0 * torch.sqrt(ee) * s3[:, None] * s3[None, :] / s6, zero)
        s = torch.where(m, (0.5 * s6) ** (1.0 / 6.0), zero)
        return e, s
    e = torch.where(m, torch.sqrt(ee), zero)
    if mix == 1:
        s = torch.where(m, 0.5 * (sig[:, None] + sig[None, :]), zero)
    else:
        s = torch.where(m, torch.sqrt(torch.where(m, sig[:, None] * sig[None, :], one)), zero)
    return e, s


def mix_pair_tables(eps_fg, sig_fg, eps_cg, sig_cg, mix: int, hybrid):
    """Per-type parameters -> (ntypes, ntypes) pair tables (FG and CG); the
    CG tables only for hybrid-hybrid pairs (Eq. 14)."""
    ef, sf = _mix(eps_fg, sig_fg, mix)
    h = torch.as_tensor(hybrid, dtype=torch.bool, device=eps_cg.device)
    ec, sc = _mix(eps_cg, sig_cg, mix, h[:, None] & h[None, :])
    return ef, sf, ec, sc


class _RelResFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rr: RelRes, pos, ef, sf, ec, sc):
        tables = tuple(t.detach().to("cpu", torch.float64).clone() for t in (ef, sf, ec, sc))
        cur = getattr(rr, "_installed_tables", None)
        if cur is None or not all(torch.equal(a, b) for a, b in zip(cur, tables)):
            rr.set_pair_params(*tables)     # waits for the device: only when changed
            rr._installed_tables = tables
        else:
            tables = cur
        F, E, _ = rr.forces(pos, want_virial=False)
        ctx.rr = rr
        ctx.tables = tables
        ctx.devices = tuple(t.device for t in (ef, sf, ec, sc))
        ctx.save_for_backward(pos)
        return F, (E[0] if rr.nsys == 1 else E[:, 0])

    @staticmethod
    def backward(ctx, grad_forces, grad_energy):
        rr = ctx.rr
        if getattr(rr, "_installed_tables", None) is not ctx.tables:
            rr.set_pair_params(*ctx.tables)
            rr._installed_tables = ctx.tables
        (pos,) = ctx.saved_tensors
        gpos, gpair = rr.backward(pos, grad_forces, grad_energy)
        grads = tuple(gpair[k].to(ctx.devices[k]) for k in range(4))
        return (None, gpos) + grads


def energy_forces(rr: RelRes, pos: torch.Tensor, eps_fg, sig_fg, eps_cg, sig_cg):
    """Forces (N, 3) and total energy (one per system when the context holds
    several), differentiable with respect to ``pos`` and the per-type
    parameters (1-D tensors of length ntypes).  Lists must
    have been built for ``pos`` (``rr.build_lists``)."""
    tables = mix_pair_tables(eps_fg, sig_fg, eps_cg, sig_cg, rr.mix, rr.hybrid)
    return _RelResFunction.apply(rr, pos, *tables)
