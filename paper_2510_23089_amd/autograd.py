"""torch.autograd wrappers of the differentiable calls of libqtt.

Each Function's forward runs the library's forward kernels and keeps what
the library's adjoint needs (the `saved` buffer of mpo_apply, the input
cores); its backward runs the library's adjoint kernels.  Cores are
capacity-layout tensors (m, cap, 2, cap) -- or (count, m, cap, 2, cap) for a
batch -- with their device bond arrays passed alongside (not differentiable).

The use case is gradient-based phase retrieval: a complex transmission mask
given as an MPS is propagated by the Fresnel MPOs (x then y axis, each a
zip-up plus truncation sweep) and decompressed, and the squared intensity
error against a target drives the mask (the paper's outlook names phase
retrieval among the inverse problems the method could serve).
"""
import torch

from . import api


def _wrap(cores, bonds):
    if cores.dim() == 5:
        return api.MPSBatch.wrap(cores, bonds)
    return api.MPS.wrap(cores, bonds)


class _Apply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cores, bonds, mpo, chi, chi_zip, tau):
        psi = _wrap(cores, bonds)
        batched = cores.dim() == 5
        saved = api.saved_buffer(psi, mpo, chi, chi_zip)
        if batched:
            out = api.mpo_apply_batched(psi, mpo, chi, chi_zip, tau=tau, saved=saved)
        else:
            out = api.mpo_apply(psi, mpo, chi, chi_zip, tau=tau, saved=saved)
        ctx.save_for_backward(cores, bonds, out.cores, out.bonds, saved)
        ctx.mpo, ctx.chi, ctx.chi_zip, ctx.batched, ctx.tau = mpo, chi, chi_zip, batched, tau
        ctx.mark_non_differentiable(out.bonds)
        return out.cores, out.bonds

    @staticmethod
    def backward(ctx, g_cores, g_bonds):
        cores, bonds, ocores, obonds, saved = ctx.saved_tensors
        psi, out = _wrap(cores, bonds), _wrap(ocores, obonds)
        gout = _wrap(g_cores.contiguous(), obonds)
        if ctx.batched:
            g = api.mpo_apply_backward_batched(psi, ctx.mpo, ctx.chi, saved, out, gout, ctx.chi_zip, tau=ctx.tau)
        else:
            g = api.mpo_apply_backward(psi, ctx.mpo, ctx.chi, saved, out, gout, ctx.chi_zip, tau=ctx.tau)
        return g.cores, None, None, None, None, None


class _Dense(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cores, bonds):
        psi = _wrap(cores, bonds)
        dense = api.tt_to_dense_batched(psi) if cores.dim() == 5 else api.tt_to_dense(psi)
        ctx.save_for_backward(cores, bonds)
        return dense

    @staticmethod
    def backward(ctx, g_dense):
        cores, bonds = ctx.saved_tensors
        psi = _wrap(cores, bonds)
        if cores.dim() == 5:
            g = api.tt_to_dense_backward_batched(psi, g_dense.contiguous())
        else:
            g = api.tt_to_dense_backward(psi, g_dense.contiguous())
        return g.cores, None


class _Loss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, field, target):
        loss, grad = api.intensity_loss(field, target, with_grad=True)
        ctx.save_for_backward(grad)
        return loss.sum()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.real.dtype), None


def mpo_apply(cores, bonds, mpo, chi, chi_zip=0, tau=0.0):
    """Differentiable MPO x MPS (zip-up + sweep to chi); returns (cores, bonds).
    tau: the keep rule's numerical-zero threshold on lam_i / lam_1 (0: the
    library default)."""
    return _Apply.apply(cores, bonds, mpo, int(chi), int(chi_zip or 0), float(tau or 0.0))


def to_dense(cores, bonds):
    """Differentiable decompression to the N x N field(s)."""
    return _Dense.apply(cores, bonds)


def intensity_loss(field, target):
    """Differentiable sum over fields and pixels of (|E|^2 - I_target)^2."""
    return _Loss.apply(field, target)


class PhaseRetrieval:
    """Loss and gradient of a mask MPS (or a batch of them) under Fresnel
    propagation: L = sum (|dense(W^y W^x mask)|^2 - I_target)^2, with both
    applications truncated to chi.  wx, wy: MPO (single) or MPOBatch.
    tau: keep threshold of both applications (0: the library default)."""

    def __init__(self, wx, wy, chi, chi_zip=0, tau=0.0):
        self.wx, self.wy, self.chi, self.chi_zip = wx, wy, int(chi), int(chi_zip or 0)
        self.tau = float(tau or 0.0)

    def field(self, cores, bonds):
        c1, b1 = mpo_apply(cores, bonds, self.wx, self.chi, self.chi_zip, self.tau)
        c2, b2 = mpo_apply(c1, b1, self.wy, self.chi, self.chi_zip, self.tau)
        return to_dense(c2, b2)

    def loss(self, cores, bonds, target):
        return intensity_loss(self.field(cores, bonds), target)

    def loss_and_grad(self, cores, bonds, target):
        x = cores.detach().requires_grad_(True)
        val = self.loss(x, bonds, target)
        (g,) = torch.autograd.grad(val, x)
        return val.detach(), g
