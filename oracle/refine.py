"""One two-site variational fitting sweep: the FP32 refinement pass that
follows a reduced-precision (bfloat16) zip-up.

Test infrastructure, like the rest of ``oracle``.

Reading used by the build (the paper applies MPOs with a cutoff, Sec. 5, but
fixes no refinement scheme; the precision form with one full-precision
refinement sweep is the build's, so this is a definition, not a transcription):

    Given the input MPS psi (cores A_k), the operator W (cores W_k) and an
    initial state phi0 in right-canonical form (the zip-up output: cores B_k
    right-orthonormal, centre at site 1), sweep left to right over the pairs
    (k, k+1), k = 1..m-1.  With the left environment L_k built from the cores
    already fixed by this sweep and the right environment R_(k+2) built from
    phi0's cores k+2..m, the pair tensor maximising the overlap with W psi is
        Theta[(b, t1), (t2, b'')] = sum L_k[b, w, a] A_k[a, s1, a'] W_k[w, t1, s1, w']
                                        A_(k+1)[a', s2, a''] W_(k+1)[w', t2, s2, w'']
                                        R_(k+2)[b'', w'', a''],
    where both environments contract conj(phi) on their phi legs.  Theta is
    split by SVD with the keep rule (cap chi): the left factor U becomes core k
    (left-orthonormal) and the sweep moves on; at the last pair core m-1 =
    U and core m = U^H Theta.  The result is left-canonical with the norm in
    the last core, like the plain truncation sweep it replaces.

With the zip-up lossless and chi at least the exact ranks, the fit returns
W psi exactly; each pair update is the exact maximiser of the overlap given
the environments, so the distance to W psi never exceeds that of the state
the sweep starts from restricted to the same bond caps.  Both are pinned in
the tests.
"""
import numpy as np

from .ttsvd import keep_count, TAU_F64
from .zipup import zip_up


def _right_envs(mps, mpo, init):
    """R[k] = environment of sites k..m-1 (0-based), [b, w, a]; R[m] = 1."""
    m = len(mps)
    envs = [None] * (m + 1)
    envs[m] = np.ones((1, 1, 1), dtype=np.complex128)
    for k in range(m - 1, 0, -1):
        r = envs[k + 1]
        x = np.tensordot(mps[k], r, axes=(2, 2))                 # [a, s, b', w']
        x = np.tensordot(x, mpo[k], axes=([1, 3], [2, 3]))       # [a, b', w, t]
        envs[k] = np.tensordot(np.conj(init[k]), x, axes=([1, 2], [3, 1])).transpose(0, 2, 1)  # [b, w, a]
    return envs


def fit_sweep(mps, mpo, init, chi, eps=0.0, tau=TAU_F64):
    """Two-site fitting sweep, left to right, from the right-canonical init."""
    m = len(mps)
    R = _right_envs(mps, mpo, init)
    out = [None] * m
    L = np.ones((1, 1, 1), dtype=np.complex128)                  # [b, w, a]
    for k in range(m - 1):
        # left part: LX[b, t1, a', w'] = L[b, w, a] A_k[a, s1, a'] W_k[w, t1, s1, w']
        y = np.tensordot(L, mps[k], axes=(2, 0))                  # [b, w, s1, a']
        lx = np.tensordot(y, mpo[k], axes=([1, 2], [0, 2]))       # [b, a', t1, w']
        lx = lx.transpose(0, 2, 1, 3)                             # [b, t1, a', w']
        # right part: RM[a', w', t2, b''] = A_(k+1) W_(k+1) R_(k+2)
        x = np.tensordot(mps[k + 1], R[k + 2], axes=(2, 2))       # [a', s2, b'', w'']
        x = np.tensordot(x, mpo[k + 1], axes=([1, 3], [2, 3]))    # [a', b'', w', t2]
        rm = x.transpose(0, 2, 3, 1)                              # [a', w', t2, b'']
        rb, _, ra, rw = lx.shape
        theta = np.tensordot(lx, rm, axes=([2, 3], [0, 1]))       # [b, t1, t2, b'']
        b2 = theta.shape[3]
        mat = theta.reshape(rb * 2, 2 * b2)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        r = keep_count(s * s, chi, eps, tau)
        u = u[:, :r]
        out[k] = u.reshape(rb, 2, r)
        if k == m - 2:
            out[m - 1] = (u.conj().T @ mat).reshape(r, 2, b2)
        else:
            # L_(k+1)[i, w', a'] = conj(U)[(b, t1), i] LX[(b, t1), (a', w')]
            lxm = lx.reshape(rb * 2, ra * rw)
            L = (u.conj().T @ lxm).reshape(r, ra, rw).transpose(0, 2, 1)
    return out, float(np.linalg.norm(out[m - 1]))


def mpo_apply_refined(mps, mpo, chi, chi_zip=None, eps=0.0, tau=TAU_F64):
    """Zip-up (cap chi_zip, default chi), then one fitting sweep to chi."""
    if chi_zip is None:
        chi_zip = chi
    z = zip_up(mps, mpo, chi_zip, eps, tau)
    return fit_sweep(mps, mpo, z, chi, eps, tau)
