"""Pins for the oracle's two-site fitting sweep (oracle.refine).

Independent references: the dense FFT propagation (the fit of an exact,
untruncated zip-up returns W psi exactly), Eckart-Young at a single bond, and
the same sweep carried out with dense projections -- the left basis from the
cores the sweep has fixed, the right basis from the initial state, the
target W psi from the dense FFT oracle -- instead of environment
contractions through the MPO.
"""
import numpy as np
import pytest

from oracle import fresnel as F
from oracle import mpo as M
from oracle import quantics as Q
from oracle import refine as RF
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

LAM, DX = 500e-9, 1e-6
BIG = 1 << 20


def _axis_mpos(n, z):
    c = M.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    return M.embed_axis(c, "x"), M.embed_axis(c, "y")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _chain(cores):
    """Dense contraction of a list of cores -> [left bond, 2^len, right bond]."""
    acc = cores[0]
    for c in cores[1:]:
        acc = np.tensordot(acc, c, axes=(acc.ndim - 1, 0))
    return acc.reshape(acc.shape[0], -1, acc.shape[-1])


def _dense_route_fit(target_q, init, chi, m):
    """The fitting sweep by dense projections of the target vector."""
    out = []
    for k in range(m - 1):
        if k == 0:
            lb = np.ones((1, 1), dtype=np.complex128)
        else:
            lb = _chain(out[:k])[0]                                  # [2^k, r_k]
        if k + 2 <= m - 1:
            rb = _chain(init[k + 2:])[:, :, 0]                       # [b'', 2^(m-k-2)]
        else:
            rb = np.ones((1, 1), dtype=np.complex128)
        t = target_q.reshape(lb.shape[0], 4, rb.shape[1])
        theta = np.einsum("lr,lqc,bc->rqb", lb.conj(), t, rb.conj())   # [r_k, (t1 t2), b'']
        rk, _, b2 = theta.shape
        mat = theta.reshape(rk, 2, 2, b2).reshape(rk * 2, 2 * b2)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        r = T.keep_count(s * s, chi, 0.0, T.TAU_F64)
        u = u[:, :r]
        out.append(u.reshape(rk, 2, r))
        if k == m - 2:
            out.append((u.conj().T @ mat).reshape(r, 2, b2))
    return out


def test_lossless_fit_equals_fft():
    n, z = 3, 4e-6
    e0 = synth.random_field(4, 1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, BIG)
    wx, _ = _axis_mpos(n, z)
    out, nrm = RF.mpo_apply_refined(cores, wx, BIG, chi_zip=BIG)
    # the x-axis operator alone: propagate along the rows axis only
    ref = np.fft.ifft(np.fft.fft(e0, axis=0) * F.transfer_1d(1 << n, LAM, DX, z)[:, None], axis=0)
    assert _rel(Z.to_dense(out, n), ref) < 1e-12
    assert abs(nrm - np.linalg.norm(ref)) < 1e-12 * np.linalg.norm(ref)
    for c in out[:-1]:
        mat = c.reshape(-1, c.shape[2])
        assert np.allclose(mat.conj().T @ mat, np.eye(c.shape[2]), atol=1e-12)


def test_single_bond_is_eckart_young():
    rng = np.random.default_rng(2)
    psi = [rng.standard_normal((1, 2, 2)) + 1j * rng.standard_normal((1, 2, 2)),
           rng.standard_normal((2, 2, 1)) + 1j * rng.standard_normal((2, 2, 1))]
    w = [rng.standard_normal((1, 2, 2, 3)) + 1j * rng.standard_normal((1, 2, 2, 3)),
         rng.standard_normal((3, 2, 2, 1)) + 1j * rng.standard_normal((3, 2, 2, 1))]
    out, _ = RF.mpo_apply_refined(psi, w, chi=1, chi_zip=4)
    # W as a 4 x 4 matrix [(t1, t2), (s1, s2)]
    dense_w = np.einsum("atsw,wuvb->tusv", w[0], w[1]).reshape(4, 4)
    target = (dense_w @ T.tt_dense(psi)).reshape(2, 2)
    u, s, vh = np.linalg.svd(target)
    best = s[0] * np.outer(u[:, 0], vh[0])
    assert _rel(T.tt_dense(out).reshape(2, 2), best) < 1e-12


@pytest.mark.parametrize("n,chi,z,seed", [(3, 3, 6e-6, 0), (3, 5, 10e-6, 1), (4, 6, 30e-6, 2)])
def test_fit_matches_dense_projection_route(n, chi, z, seed):
    e0 = synth.random_field(seed, 1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi)
    wx, _ = _axis_mpos(n, z)
    init = Z.zip_up(cores, wx, chi)
    out, _ = RF.fit_sweep(cores, wx, init, chi)
    # target W psi from the dense FFT oracle (x axis only)
    tgt = np.fft.ifft(np.fft.fft(Z.to_dense(cores, n), axis=0) * F.transfer_1d(1 << n, LAM, DX, z)[:, None], axis=0)
    ref = _dense_route_fit(Q.to_quantics(tgt), init, chi, 2 * n)
    assert T.bonds(out) == T.bonds(ref)
    assert _rel(T.tt_dense(out), T.tt_dense(ref)) < 1e-9


def test_fit_not_worse_than_plain_sweep_on_aperture():
    n, chi, z = 5, 6, 40e-6
    e0 = synth.aperture_field(0, n=1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, 12)
    wx, _ = _axis_mpos(n, z)
    exact = np.fft.ifft(np.fft.fft(Z.to_dense(cores, n), axis=0) * F.transfer_1d(1 << n, LAM, DX, z)[:, None], axis=0)
    plain, _ = Z.mpo_apply(cores, wx, chi)
    fit, _ = RF.mpo_apply_refined(cores, wx, chi)
    e_plain = _rel(Z.to_dense(plain, n), exact)
    e_fit = _rel(Z.to_dense(fit, n), exact)
    assert e_fit <= e_plain * (1 + 1e-9)
