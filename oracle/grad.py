"""Differentiable twin of the oracle: zip-up, sweep, decompression and the
intensity loss in torch (CPU, complex128), so that autograd gives the float64
reference gradient.

Test infrastructure, like the rest of ``oracle``.

The forward computation is the same algorithm as ``oracle.zipup`` (Sec. 5
MPO x MPS application read as zip-up then TT-rounding; the keep rule of
``oracle.ttsvd``), restated with torch tensors: the SVDs are
factorisations M -> (V_k, M V_k) with V_k the top right singular vectors
(``_KeepRight``: forward by ``torch.linalg.svd``, backward written out from
the eigenvector perturbation formula of G = M^H M), truncated by the same
keep rule, whose integer decisions are taken on detached singular values.
Everything else (contractions, decompression, loss) is differentiated by
torch autograd.

The learning problem the adjoint serves (phase retrieval, named in the
paper's outlook as future work) is read as follows: a complex transmission
mask given as an MPS multiplies a unit plane wave, the field is propagated by
the Fresnel MPO (x axis, then y axis, Sec. 6.1) with truncation to chi, and
the loss is the summed squared intensity error
    L = sum_px (|E_z|^2 - I_target)^2 .
Gradients follow torch's convention for a real loss of complex variables:
grad = dL/dRe + i dL/dIm.
"""
import numpy as np
import torch

from .ttsvd import keep_count, TAU_F64

CT = torch.complex128

# Pairs (kept i, discarded j) with lam_i - lam_j <= GAP_AD * lam_1 contribute
# nothing to the derivative.  Reading: the paper's truncation is an SVD, but a
# solver that reaches it through the Gram matrix (Sec. 4: each cut is a
# Schmidt decomposition, its weights the eigenvalues of the reduced density
# matrix) resolves eigenvectors only to about eps lam_1 / gap, and a pair's
# term divides by that gap once more; below about 1e-10 lam_1 the product
# is no longer small where the discarded weights are near the float64 floor,
# so such a pair's derivative is taken as zero.  The exact derivative differs
# from this one only through the dropped pairs (about 5e-4 relative for
# phase masks of 1024^2 at chi 64 with tau = 1e-13); the library's adjoint
# follows the same reading.
GAP_AD = 1e-10


def as_tensors(cores, requires_grad=False):
    return [torch.tensor(np.asarray(c), dtype=CT, requires_grad=requires_grad) for c in cores]


class _KeepRight(torch.autograd.Function):
    """Truncated factorisation M -> (V_k, M V_k), V_k the top-k eigenvectors
    of M^H M (right singular vectors of M).

    Backward: with G = M^H M = V diag(lam) V^H (all n eigenpairs), incoming
    gradients gV (n x k) and gC (rows x k),
        Vbar = gV + M^H gC,           Mbar = gC V_k^H,
        Z_ij = (V_perp^H Vbar)_ij / (lam_j - lam_i)   (i discarded, j kept;
               0 where lam_j - lam_i <= GAP_AD lam_1),
        Gbar = V_perp Z V_k^H,        Mbar += M (Gbar + Gbar^H).
    The kept-kept block of the eigenvector derivative is left out: every use
    of the pair (V_k, M V_k) in the zip-up and the sweep is invariant under
    V_k -> V_k Q for unitary Q (the next factorisation absorbs Q), so its
    contribution to the gradient of such a function vanishes identically,
    and evaluating it would only amplify rounding by 1/(lam_i - lam_j)."""

    @staticmethod
    def forward(ctx, mat, k):
        _, s, vh = torch.linalg.svd(mat, full_matrices=True)
        n = mat.shape[1]
        lam = torch.zeros(n, dtype=torch.float64)
        lam[: s.shape[0]] = s * s
        v = vh.conj().T
        vk = v[:, :k].contiguous()
        ctx.save_for_backward(mat, v, lam)
        ctx.k = k
        return vk, mat @ vk

    @staticmethod
    def backward(ctx, g_v, g_c):
        mat, v, lam = ctx.saved_tensors
        k = ctx.k
        vk, vp = v[:, :k], v[:, k:]
        vbar = torch.zeros_like(vk) if g_v is None else g_v.clone()
        mbar = torch.zeros_like(mat)
        if g_c is not None:
            vbar = vbar + mat.conj().T @ g_c
            mbar = mbar + g_c @ vk.conj().T
        if vp.shape[1] > 0:
            den = lam[None, :k] - lam[k:, None]
            # pairs closer than the eigenvector resolution carry no derivative
            keep = den > GAP_AD * lam[0]
            z = torch.where(keep, (vp.conj().T @ vbar) / torch.where(keep, den, torch.ones_like(den)),
                            torch.zeros((), dtype=CT))
            gbar = vp @ z @ vk.conj().T
            mbar = mbar + mat @ (gbar + gbar.conj().T)
        return mbar, None


def _keep(mat, cap, eps, tau):
    """Keep count of the truncation of ``mat`` (keep rule on sigma^2)."""
    s = torch.linalg.svdvals(mat.detach())
    return keep_count((s ** 2).numpy(), cap, eps, tau)


def zip_up(mps, mpo, chi_zip, eps=0.0, tau=TAU_F64):
    """Right-to-left zip-up (same steps as ``oracle.zipup.zip_up``)."""
    m = len(mps)
    out = [None] * m
    carry = torch.ones((1, 1, 1), dtype=CT)
    for k in range(m - 1, -1, -1):
        a = mps[k]
        w = torch.as_tensor(np.asarray(mpo[k]), dtype=CT)
        x = torch.tensordot(a, carry, dims=([2], [0]))           # [ra, s, db, beta]
        t = torch.tensordot(x, w, dims=([1, 2], [2, 3]))         # [ra, beta, da, t]
        t = t.permute(0, 2, 3, 1)                                # [ra, da, t, beta]
        ra, da, _, beta = t.shape
        mat = t.reshape(ra * da, 2 * beta)
        if k == 0:
            out[0] = mat.reshape(1, 2, beta)
            break
        r = _keep(mat, chi_zip, eps, tau)
        v, c = _KeepRight.apply(mat, r)
        out[k] = v.conj().T.reshape(r, 2, beta)          # B_k = V^H
        carry = c.reshape(ra, da, r)                     # M V = U S
    return out


def sweep(cores, chi, eps=0.0, tau=TAU_F64):
    """Left-to-right SVD truncation (same steps as ``oracle.zipup.sweep``)."""
    b = list(cores)
    m = len(b)
    for k in range(m - 1):
        r0, _, r1 = b[k].shape
        mat = b[k].reshape(2 * r0, r1)
        r = _keep(mat, chi, eps, tau)
        # left factor of mat = right factor of mat^H: U = V(mat^H), U^H mat = (mat^H U)^H
        u, c = _KeepRight.apply(mat.conj().T, r)
        b[k] = u.reshape(r0, 2, r)
        b[k + 1] = torch.tensordot(c.conj().T, b[k + 1], dims=([1], [0]))
    return b


def mpo_apply(mps, mpo, chi, chi_zip=None, eps=0.0, tau=TAU_F64):
    if chi_zip is None:
        chi_zip = chi
    return sweep(zip_up(mps, mpo, chi_zip, eps, tau), chi, eps, tau)


def to_dense(cores, n):
    """Contract the chain and undo the bit interleave: N x N field (Sec. 3)."""
    acc = cores[0].reshape(2, -1)
    for c in cores[1:]:
        acc = (acc @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    v = acc.reshape([2] * (2 * n))
    perm = list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2))
    return v.permute(perm).reshape(1 << n, 1 << n)


def intensity_loss(field, target):
    """Summed squared intensity error (the phase-retrieval objective)."""
    inten = field.real ** 2 + field.imag ** 2
    return torch.sum((inten - target) ** 2)


def propagate(mask, wx, wy, chi, chi_zip=None, tau=TAU_F64):
    """Plane wave x mask, then the x-axis and y-axis Fresnel MPOs, each a
    zip-up plus sweep to chi."""
    mid = mpo_apply(mask, wx, chi, chi_zip, tau=tau)
    return mpo_apply(mid, wy, chi, chi_zip, tau=tau)


def loss_and_grad(mask_cores, wx, wy, target, chi, n, chi_zip=None, tau=TAU_F64):
    """Float64 loss and its gradient w.r.t. every mask core (numpy arrays)."""
    ts = as_tensors(mask_cores, requires_grad=True)
    out = propagate(ts, wx, wy, chi, chi_zip, tau)
    loss = intensity_loss(to_dense(out, n), torch.as_tensor(np.asarray(target), dtype=torch.float64))
    grads = torch.autograd.grad(loss, ts)
    return float(loss.detach()), [g.detach().numpy() for g in grads]


def linear_grad(cores, wx, wy, probe, chi, n, chi_zip=None, tau=TAU_F64):
    """Gradient of Re <probe, dense(apply_y(apply_x(psi)))> w.r.t. the cores."""
    ts = as_tensors(cores, requires_grad=True)
    out = propagate(ts, wx, wy, chi, chi_zip, tau)
    e = to_dense(out, n)
    val = torch.sum(torch.conj(torch.as_tensor(np.asarray(probe), dtype=CT)) * e).real
    grads = torch.autograd.grad(val, ts)
    return float(val.detach()), [g.detach().numpy() for g in grads]


def dense_linear_grad(cores, probe, n):
    """Gradient of Re <probe, dense(psi)> w.r.t. the cores (decompression only)."""
    ts = as_tensors(cores, requires_grad=True)
    e = to_dense(ts, n)
    val = torch.sum(torch.conj(torch.as_tensor(np.asarray(probe), dtype=CT)) * e).real
    grads = torch.autograd.grad(val, ts)
    return [g.detach().numpy() for g in grads]
