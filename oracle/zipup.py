"""MPO x MPS application by zip-up followed by a truncation sweep.

The paper applies an operator MPO to a field MPS with a cutoff (Sec. 5: cost
O(2n chi_1^2 chi_2^2)) and obtains real-space propagation as the product of a
QFT MPO, a diagonal phase MPO and an inverse QFT MPO (Sec. 6.1).  The
contraction scheme is not spelled out there; the reading used by the whole
build (zip-up of Stoudenmire and White, then TT-rounding) is:

Zip-up, right to left, with the input left-canonical.  Carry C_m = 1.  At site
k = m..1 form T = A_k . W_k . C_k, reshape to M = [(a_(k-1), w_(k-1)),
(t_k, beta_k)].  For k > 1 take M = U S V^H, keep beta_(k-1) by the keep rule
with cap chi_zip, store B_k = V^H (right-orthonormal) and carry
C_(k-1) = U S.  At k = 1 the row dimension is 1 and B_1 = M.

Sweep, left to right.  At k = 1..m-1 reshape B_k to [(r_(k-1), t), beta_k],
take the SVD, keep r_k by the keep rule with cap chi, store B_k = U and absorb
S V^H into B_(k+1).  The result is left-canonical and its norm is ||B_m||_F.

With chi_zip large enough that nothing is dropped in the zip-up, the sweep is
exactly TT-rounding of an exact TT, which equals the TT-SVD of the dense
result; this is one of the pins in the tests.
"""
import numpy as np

from .ttsvd import keep_count, TAU_F64, tt_dense
from .quantics import from_quantics


def _svd(mat):
    return np.linalg.svd(mat, full_matrices=False)


def zip_up(mps, mpo, chi_zip, eps=0.0, tau=TAU_F64):
    """Right-to-left zip-up; returns right-canonical cores (centre at site 1)."""
    m = len(mps)
    assert len(mpo) == m
    out = [None] * m
    carry = np.ones((1, 1, 1), dtype=np.complex128)      # [a_k, w_k, beta_k]
    for k in range(m - 1, -1, -1):
        a = mps[k]                                         # [ra, s, rb]
        w = mpo[k]                                         # [da, t, s, db]
        # T[a_(k-1), w_(k-1), t, beta_k]
        x = np.tensordot(a, carry, axes=(2, 0))            # [ra, s, db, beta]
        t = np.tensordot(x, w, axes=([1, 2], [2, 3]))      # [ra, beta, da, t]
        t = t.transpose(0, 2, 3, 1)                        # [ra, da, t, beta]
        ra, da, _, beta = t.shape
        mat = t.reshape(ra * da, 2 * beta)
        if k == 0:
            assert ra * da == 1
            out[0] = mat.reshape(1, 2, beta)
            break
        u, s, vh = _svd(mat)
        r = keep_count(s * s, chi_zip, eps, tau)
        out[k] = vh[:r].reshape(r, 2, beta)
        carry = (u[:, :r] * s[:r]).reshape(ra, da, r)
    return out


def sweep(cores, chi, eps=0.0, tau=TAU_F64):
    """Left-to-right SVD truncation of a right-canonical MPS.

    Returns (left-canonical cores, float64 norm ||B_m||)."""
    b = [np.asarray(c, dtype=np.complex128) for c in cores]
    m = len(b)
    for k in range(m - 1):
        r0, _, r1 = b[k].shape
        u, s, vh = _svd(b[k].reshape(2 * r0, r1))
        r = keep_count(s * s, chi, eps, tau)
        b[k] = u[:, :r].reshape(r0, 2, r)
        rmat = s[:r, None] * vh[:r]
        b[k + 1] = np.tensordot(rmat, b[k + 1], axes=(1, 0))
    return b, float(np.linalg.norm(b[-1]))


def mpo_apply(mps, mpo, chi, chi_zip=None, eps=0.0, tau=TAU_F64):
    """Zip-up (cap chi_zip, default chi) then sweep (cap chi)."""
    if chi_zip is None:
        chi_zip = chi
    return sweep(zip_up(mps, mpo, chi_zip, eps, tau), chi, eps, tau)


def right_orthogonalize(cores):
    """QR sweep right to left: cores 2..m right-orthonormal, centre at 1."""
    b = [np.asarray(c, dtype=np.complex128) for c in cores]
    for k in range(len(b) - 1, 0, -1):
        r0, _, r1 = b[k].shape
        # M = L Q with Q having orthonormal rows: QR of M^H
        q, r = np.linalg.qr(b[k].reshape(r0, 2 * r1).conj().T)
        b[k] = q.conj().T.reshape(-1, 2, r1)
        b[k - 1] = np.tensordot(b[k - 1], r.conj().T, axes=(2, 0))
    return b


def tt_truncate(cores, chi, eps=0.0, tau=TAU_F64):
    """TT-rounding: right-orthogonalise by QR, then SVD sweep left to right."""
    return sweep(right_orthogonalize(cores), chi, eps, tau)


def to_dense(cores, n):
    """Decompress an MPS on a 2^n x 2^n grid to the N x N image (Sec. 3)."""
    return from_quantics(tt_dense(cores), n)


def bonds(cores):
    return [1] + [int(c.shape[2]) for c in cores]
