"""Sequential-SVD construction of a matrix product state (Sec. 4, App. A).

Every bond k is a Schmidt cut {1..k} | {k+1..m}.  Sweeping left to right, the
remainder is reshaped to (2 r_(k-1)) x 2^(m-k), an SVD is taken, the left
singular vectors become the left-orthonormal core A_k and S V^H is carried to
the next cut.  The last core holds the norm.

Keep rule (the paper mixes an MSE target with a library "cutoff"; the reading
used throughout the build): with lam_i = sigma_i^2 sorted descending,
    k = min(chi, k_eps, #{ lam_i > tau * lam_1 }),  and at least 1,
where k_eps is the smallest k with sum_(i>k) lam_i <= eps * sum_i lam_i
(eps = 0 disables it).  tau removes numerical zeros.
"""
import numpy as np

TAU_F64 = 1e-26          # relative to lam_1, i.e. sigma_i / sigma_1 > 1e-13


def keep_count(lam, chi, eps=0.0, tau=TAU_F64):
    """Number of singular values kept at one cut (keep rule above).

    ``lam`` are squared singular values sorted descending."""
    lam = np.asarray(lam, dtype=np.float64)
    if lam.size == 0 or not lam[0] > 0.0:
        return 1
    k = int(np.count_nonzero(lam > tau * lam[0]))
    k = min(k, int(chi))
    if eps > 0.0:
        total = lam.sum()
        # tail[k-1] = sum_{i>k} lam_i, summed from the small end (no cancellation)
        tail = np.append(np.cumsum(lam[::-1])[::-1][1:], 0.0)
        k_eps = int(np.argmax(tail <= eps * total)) + 1
        k = min(k, k_eps)
    return max(k, 1)


def tt_svd(vec, m, chi, eps=0.0, tau=TAU_F64):
    """Quantics vector (length 2^m) -> list of m cores [r_(k-1), 2, r_k].

    Output is left-canonical; the norm sits in the last core (App. A)."""
    rem = np.asarray(vec, dtype=np.complex128).reshape(1, -1)
    cores = []
    r_prev = 1
    for _k in range(m - 1):
        mat = rem.reshape(2 * r_prev, -1)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        r = keep_count(s * s, chi, eps, tau)
        cores.append(u[:, :r].reshape(r_prev, 2, r))
        rem = s[:r, None] * vh[:r]
        r_prev = r
    cores.append(rem.reshape(r_prev, 2, 1))
    return cores


def tt_dense(cores):
    """Contract an MPS back to its flat vector (the decompression of Sec. 3)."""
    acc = np.ones((1, 1), dtype=np.complex128)
    for c in cores:
        acc = np.tensordot(acc, c, axes=(acc.ndim - 1, 0))
    return acc.reshape(-1)


def bonds(cores):
    return [1] + [c.shape[2] for c in cores]


def param_count(cores):
    """Total number of parameters D = sum_k r_(k-1) * 2 * r_k (Sec. 4)."""
    return int(sum(c.size for c in cores))
