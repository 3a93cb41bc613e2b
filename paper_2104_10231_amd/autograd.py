"""Differentiable RelRes energy and forces (torch.autograd over the C ABI).

``energy_forces(rr, pos, eps_fg, sig_fg, eps_cg, sig_cg)`` returns the forces
(N, 3) and the total energy of Eq. 3 as tensors that carry gradients to the
positions and to the per-type FG/CG Lennard-Jones parameters.  Argument
marshalling only: the forward pass installs the per-type parameters with
``relres_set_type_params`` (the library mixes them, Sec. 2.3 and Eq. 14) and
calls ``relres_forces``; the backward pass is ``relres_backward_types``, a
HIP kernel that recomputes every pair term in FP64 and returns dJ/dx and
dJ/d(per-type parameter), carried through the mixing rule by the library,
for J = e_bar E + sum_i g_i . F_i.  Any loss of the energy and forces works,
e.g. force matching sum_i |F_i - F_ref,i|^2.

The context's parameters are the ones of the most recent forward call; the
backward pass re-installs the parameters of its own forward call if they
changed since.
"""
from __future__ import annotations

import torch

from .relres import RelRes

__all__ = ["energy_forces"]


def _install(rr: RelRes, params):
    cur = getattr(rr, "_installed_params", None)
    if cur is not None and (cur is params or all(torch.equal(a, b) for a, b in zip(cur, params))):
        return cur
    rr.set_type_params(*params)         # waits for the device: only when changed
    rr._installed_params = params
    return params


class _RelResFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rr: RelRes, pos, eps_fg, sig_fg, eps_cg, sig_cg):
        params = tuple(t.detach().to("cpu", torch.float64).clone()
                       for t in (eps_fg, sig_fg, eps_cg, sig_cg))
        params = _install(rr, params)
        F, E, _ = rr.forces(pos, want_virial=False)
        ctx.rr = rr
        ctx.params = params
        ctx.devices = tuple(t.device for t in (eps_fg, sig_fg, eps_cg, sig_cg))
        ctx.save_for_backward(pos)
        return F, (E[0] if rr.nsys == 1 else E[:, 0])

    @staticmethod
    def backward(ctx, grad_forces, grad_energy):
        rr = ctx.rr
        _install(rr, ctx.params)
        (pos,) = ctx.saved_tensors
        gpos, gtype = rr.backward_types(pos, grad_forces, grad_energy)
        grads = tuple(gtype[k].to(ctx.devices[k]) for k in range(4))
        return (None, gpos) + grads


def energy_forces(rr: RelRes, pos: torch.Tensor, eps_fg, sig_fg, eps_cg, sig_cg):
    """Forces (N, 3) and total energy (one per system when the context holds
    several), differentiable with respect to ``pos`` and the per-type
    parameters (1-D tensors of length ntypes).  Lists must have been built
    for ``pos`` (``rr.build_lists``)."""
    return _RelResFunction.apply(rr, pos, eps_fg, sig_fg, eps_cg, sig_cg)
