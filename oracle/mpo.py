"""Matrix product operators from dense matrices (Sec. 5, Sec. 6.1).

Core convention: W_k[D_(k-1), t, s, D_k] with t the output (row) bit and s the
input (column) bit of site k, most significant bit first, so that
(U psi)[i] = sum_j U[i, j] psi[j] and U[i, j] = W_1[t_1 s_1] ... W_n[t_n s_n].

``mpo_from_matrix`` is the brute-force construction of Sec. 6.1 (interleave the
row and column bits, then sequential SVD exactly as for a quantics MPS).
"""
import numpy as np

from .ttsvd import keep_count


def mpo_from_matrix(mat, n, rel_err=1e-12):
    """Dense 2^n x 2^n operator -> list of n cores [D, 2, 2, D'].

    The per-bond discarded weight is at most rel_err^2/(n-1) of the total, so
    the Frobenius error of the whole operator is at most rel_err * ||U||_F."""
    mat = np.asarray(mat, dtype=np.complex128)
    nn = 1 << n
    assert mat.shape == (nn, nn)
    t = mat.reshape((2,) * (2 * n))              # i_1..i_n, j_1..j_n
    order = []
    for p in range(n):
        order += [p, n + p]                       # i_p, j_p interleaved
    rem = np.ascontiguousarray(t.transpose(order)).reshape(1, -1)
    eps = rel_err * rel_err / max(n - 1, 1)
    cores = []
    d_prev = 1
    for _k in range(n - 1):
        m2 = rem.reshape(4 * d_prev, -1)
        u, s, vh = np.linalg.svd(m2, full_matrices=False)
        d = keep_count(s * s, chi=m2.shape[0], eps=eps)
        cores.append(u[:, :d].reshape(d_prev, 2, 2, d))
        rem = s[:d, None] * vh[:d]
        d_prev = d
    cores.append(rem.reshape(d_prev, 2, 2, 1))
    return cores


def mpo_dense(cores):
    """Contract an n-site MPO back to its 2^n x 2^n matrix."""
    n = len(cores)
    acc = np.ones((1, 1), dtype=np.complex128)
    for c in cores:
        acc = np.tensordot(acc, c, axes=(acc.ndim - 1, 0))
    acc = acc.reshape((2,) * (2 * n))            # t_1 s_1 t_2 s_2 ...
    order = [2 * p for p in range(n)] + [2 * p + 1 for p in range(n)]
    return acc.transpose(order).reshape(1 << n, 1 << n)


def identity_core(d):
    """Identity site with a bond of size d passed straight through."""
    return np.einsum("ab,ts->atsb", np.eye(d), np.eye(2)).astype(np.complex128)


def embed_axis(cores_1d, axis):
    """Per-axis MPO (n sites) -> 2n-site quantics MPO acting on one axis.

    Quantics site 2p-1 carries bit p of the row coordinate a (axis 'x') and
    site 2p bit p of the column coordinate b (axis 'y'); the other axis gets
    identity sites through which the operator bond passes (Sec. 6.1: the
    paraxial propagator is U^(x) (x) U^(y))."""
    out = []
    for c in cores_1d:
        if axis == "x":
            out += [c, identity_core(c.shape[3])]
        elif axis == "y":
            out += [identity_core(c.shape[0]), c]
        else:
            raise ValueError(axis)
    return out


def bit_reverse_perm(n):
    nn = 1 << n
    idx = np.arange(nn)
    rev = np.zeros(nn, dtype=np.int64)
    for p in range(n):
        rev |= ((idx >> p) & 1) << (n - 1 - p)
    return rev


def qft_br_matrix(n):
    """Unitary DFT with bit-reversed output order, P_rev F (Sec. 5).

    F[k, j] = exp(-2 pi i j k / N) / sqrt(N) (numpy "ortho" convention);
    the natural-order DFT is full rank as an MPO, its bit-reversed form is not.
    """
    f = np.fft.fft(np.eye(1 << n), axis=0, norm="ortho")
    return f[bit_reverse_perm(n), :]


def hadamard_mpo(n):
    """Hadamard transform H_1^(x)n as a bond-1 MPO (Sec. 5)."""
    h1 = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    return [h1.reshape(1, 2, 2, 1).astype(np.complex128) for _ in range(n)]


def diag_mpo_from_vector(v, n_sites, rel_err=1e-12):
    """diag(v) for a length-2^n_sites vector as an MPO by the brute-force
    construction of Sec. 6.1: the interleaved unfoldings of a diagonal matrix
    are those of v with zero rows and columns added, so the sequential SVD of
    v itself (same per-bond rule as mpo_from_matrix) gives its cores, each
    placed on the t = s diagonal."""
    from .ttsvd import tt_svd
    eps = rel_err * rel_err / max(n_sites - 1, 1)
    cores = tt_svd(np.asarray(v, dtype=np.complex128), n_sites, chi=1 << n_sites, eps=eps)
    out = []
    for c in cores:
        r0, _, r1 = c.shape
        w = np.zeros((r0, 2, 2, r1), dtype=np.complex128)
        w[:, 0, 0, :] = c[:, 0, :]
        w[:, 1, 1, :] = c[:, 1, :]
        out.append(w)
    return out
