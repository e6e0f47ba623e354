"""Differentiable EAM force matching on the GPU.

A batch of fixed snapshots is binned and listed once; the forces of a trainable
EAM (three uniform cubic B-splines) come from md_eam_forces, and the gradient of
any loss of those forces with respect to the spline coefficients comes from the
hand-written adjoint kernel md_eam_backward, wrapped in a torch.autograd.Function
(EAMForces).  The force-matching loss itself and its cotangent come from the library
too (md_force_loss, in ForceMatchingLoss); torch then only holds memory and applies
the chain rule's upstream scalar.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from . import md


class SnapshotBatch:
    """All snapshots as one md_batch (one box per snapshot), binned and listed once."""

    def __init__(self, snapshots, r_ns, precision=N.MD_FP64, lanes=4, max_neigh=128,
                 device="cuda", density_jacobian=True):
        boxes = [s.box for s in snapshots]
        counts = [s.pos.shape[0] for s in snapshots]
        pos = np.concatenate([s.pos for s in snapshots], axis=0)
        self.plan = md.Plan(boxes, counts, r_ns, device)
        self.state = md.State(self.plan, pos, None, precision)
        self.nl = md.NeighborList(self.plan.n_atoms, max_neigh, lanes, device)
        md.md_bin_cells(self.state, N.MD_ALWAYS)
        md.md_build_neighbors(self.state, self.nl, N.MD_ALWAYS)
        self.n = self.plan.n_atoms
        self.n_snap = len(snapshots)
        self.precision = precision
        self.saved = torch.zeros((3, self.n), dtype=torch.float64, device=device)
        self.bws = None
        self.lws = None  # md_force_loss workspace
        # the positions never change, so d rhobar / d c_rho (n x n_rho FP64) is computed once
        # per rho grid; the density pass (rhobar = jac c_rho) and the adjoint read it instead
        # of visiting every list
        self.use_jac = bool(density_jacobian)
        self._jac = {}  # (rho x_lo, h, ncoef, r_cut) -> Jacobian, or None where not available
        ids = self.state.id.long()
        # current (cell) order -> original order permutation, for the caller's references
        self.order_ids = ids

    def to_current_order(self, a):
        """[n, 3] array in the original atom order -> [3, n] tensor in the current order."""
        t = torch.as_tensor(np.asarray(a, np.float64), device=self.state.pos.device)
        return t[self.order_ids].t().contiguous()

    def _forces(self, pot: md.EAMPotential, saved):
        jac = self.jacobian(pot)
        if jac is None:
            md.md_eam_forces(self.state, pot, self.nl, saved=saved)
        else:
            md.md_eam_forces_jac(self.state, pot, self.nl, jac, saved=saved)

    def forces(self, pot: md.EAMPotential, saved=True):
        self._forces(pot, self.saved if saved else None)
        return self.state.force.double()

    def loss(self, pot: md.EAMPotential, f_ref, saved, grad_force):
        """Forces at pot's coefficients ({rhobar, F', F''} into saved), then the loss against
        f_ref ([3, n] FP64) as a 0-dim device tensor and its cotangent into grad_force."""
        self._forces(pot, saved)
        if self.lws is None:
            nb = int(N.lib().md_force_loss_workspace_bytes(self.n))
            self.lws = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.state.pos.device)
        return md.md_force_loss(self.state.force, f_ref, self.precision, grad_force=grad_force,
                                ws=self.lws)

    def backward(self, pot: md.EAMPotential, grad_force, saved=None):
        """Gradient with respect to pot's current coefficients; `saved` ({rhobar, F', F''} of
        the forward pass at those coefficients) defaults to the last forces(saved=True)."""
        g = grad_force.to(torch.float64).contiguous()
        nb = int(N.lib().md_backward_workspace_bytes(C.byref(self.plan.c), C.byref(pot.c)))
        if self.bws is None or self.bws.numel() < nb:
            self.bws = torch.zeros(max(nb, 1), dtype=torch.uint8, device=self.state.pos.device)
        return md.md_eam_backward(self.state, pot, self.nl, self.saved if saved is None else saved,
                                  g, ws=self.bws, jac=self.jacobian(pot))

    def jacobian(self, pot: md.EAMPotential):
        """The density Jacobian for pot's rho grid and cutoff (kept), or None if not used or
        not available (more than 128 rho coefficients)."""
        if not self.use_jac:
            return None
        r = pot.c.rho
        key = (r.x_lo, r.h, r.ncoef, pot.c.r_cut)
        if key not in self._jac:
            nb = int(N.lib().md_density_jacobian_bytes(C.byref(self.plan.c), C.byref(pot.c)))
            self._jac[key] = md.md_eam_density_jacobian(self.state, pot, self.nl) if nb else None
        return self._jac[key]


class EAMForces(torch.autograd.Function):
    """forces = EAMForces.apply(coef, batch, potential): coef is the concatenated
    (phi | rho | F) coefficient vector; the result is [3, n] in the batch's current order.

    The state the gradient needs -- the coefficients and the forward pass's {rhobar, F',
    F''} -- is kept per call in ctx, so forward passes at other coefficients between this
    call and its backward (a second loss, a closure, numerical gradient checks) do not
    change its gradient."""

    @staticmethod
    def forward(ctx, coef, batch: SnapshotBatch, pot: md.EAMPotential):
        c = coef.detach().to(torch.float64).contiguous()
        pot.set_coefficients_flat(c)
        f = batch.forces(pot, saved=True).clone()
        ctx.batch, ctx.pot = batch, pot
        ctx.coef = c.clone()
        ctx.saved = batch.saved.clone()
        ctx.version = pot.version
        ctx.coef_dtype = coef.dtype
        return f

    @staticmethod
    def backward(ctx, grad_f):
        pot = ctx.pot
        if pot.version == ctx.version:
            g = ctx.batch.backward(pot, grad_f, saved=ctx.saved)
        else:
            # a later forward changed the coefficients: differentiate at this call's, then
            # put the later ones back (with their version, so their own backward stays direct)
            later, later_version = pot.coefficients_flat(), pot.version
            pot.set_coefficients_flat(ctx.coef)
            try:
                g = ctx.batch.backward(pot, grad_f, saved=ctx.saved)
            finally:
                pot.set_coefficients_flat(later)
                pot.version = later_version
        return g.to(ctx.coef_dtype), None, None


class ForceMatchingLoss(torch.autograd.Function):
    """loss = ForceMatchingLoss.apply(coef, batch, potential, f_ref): forces of the
    concatenated (phi | rho | F) coefficients (md_eam_forces), their mean squared error
    against f_ref ([3, n] FP64, current order) and its cotangent G = dL/dF (md_force_loss);
    backward is md_eam_backward of G.  Like EAMForces, each call keeps its own
    coefficients, {rhobar, F', F''} and G for its backward."""

    @staticmethod
    def forward(ctx, coef, batch: SnapshotBatch, pot: md.EAMPotential, f_ref):
        c = coef.detach().to(torch.float64).contiguous()
        pot.set_coefficients_flat(c)
        saved = torch.empty((3, batch.n), dtype=torch.float64, device=f_ref.device)
        G = torch.empty((3, batch.n), dtype=torch.float64, device=f_ref.device)
        loss = batch.loss(pot, f_ref, saved, G)
        ctx.batch, ctx.pot = batch, pot
        ctx.coef = c.clone()
        ctx.saved, ctx.G = saved, G
        ctx.version = pot.version
        ctx.coef_dtype = coef.dtype
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        pot = ctx.pot
        if pot.version == ctx.version:
            g = ctx.batch.backward(pot, ctx.G, saved=ctx.saved)
        else:
            later, later_version = pot.coefficients_flat(), pot.version
            pot.set_coefficients_flat(ctx.coef)
            try:
                g = ctx.batch.backward(pot, ctx.G, saved=ctx.saved)
            finally:
                pot.set_coefficients_flat(later)
                pot.version = later_version
        return (g * grad_loss).to(ctx.coef_dtype), None, None, None


def force_matching_loss(coef, batch, pot, f_ref):
    """L = 1/(S N) sum |F - F_ref|^2 over all atoms of all snapshots (f_ref: [3, n], current
    order), differentiable with respect to coef."""
    return ForceMatchingLoss.apply(coef, batch, pot, f_ref.to(torch.float64).contiguous())
