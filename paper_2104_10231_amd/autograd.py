"""Differentiable RelRes energy and forces (torch.autograd over the C ABI).

``energy_forces(rr, pos, eps_fg, sig_fg, eps_cg, sig_cg)`` returns the forces
(N, 3) and the total energy of Eq. 3 as tensors that carry gradients to the
positions and to the per-type FG/CG Lennard-Jones parameters.  The forward
pass is ``relres_forces`` on the pair parameters mixed here with torch
operations (Sec. 2.3: geometric means, or Lorentz-Berthelot for sigma; CG
parameters only for hybrid-hybrid pairs, Eq. 14), so torch carries the
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


def _outer_mean(a: torch.Tensor, arithmetic: bool) -> torch.Tensor:
    if arithmetic:
        return 0.5 * (a[:, None] + a[None, :])
    return torch.sqrt(a[:, None] * a[None, :])


def mix_pair_tables(eps_fg, sig_fg, eps_cg, sig_cg, mix: int, hybrid):
    """Per-type parameters -> (ntypes, ntypes) pair tables (FG and CG)."""
    ef = _outer_mean(eps_fg, False)
    sf = _outer_mean(sig_fg, mix == 1)
    h = torch.as_tensor(hybrid, dtype=torch.bool, device=eps_cg.device)
    hm = h[:, None] & h[None, :]
    one = torch.ones((), dtype=eps_cg.dtype, device=eps_cg.device)
    zero = torch.zeros((), dtype=eps_cg.dtype, device=eps_cg.device)
    # only hybrid-hybrid entries enter the square roots, so ordinary types
    # (eps_CG = 0) never produce infinite gradients
    eo = torch.where(hm, eps_cg[:, None] * eps_cg[None, :], one)
    ec = torch.where(hm, torch.sqrt(eo), zero)
    if mix == 1:
        sc = torch.where(hm, 0.5 * (sig_cg[:, None] + sig_cg[None, :]), zero)
    else:
        so = torch.where(hm, sig_cg[:, None] * sig_cg[None, :], one)
        sc = torch.where(hm, torch.sqrt(so), zero)
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
