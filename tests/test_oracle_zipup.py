"""Pins for the oracle's zip-up / sweep / rounding / decompression.

References independent of the zip-up code: the dense FFT propagation (lossless
regime is exact), a fast Walsh-Hadamard transform written here, the identity
operator, and the textbook fact that TT-rounding of an exact TT equals the
TT-SVD of its dense vector.
"""
import numpy as np
import pytest

from oracle import fresnel as F
from oracle import mpo as M
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

LAM, DX = 500e-9, 1e-6
BIG = 1 << 20


def _axis_mpos(n, z):
    c = M.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    return M.embed_axis(c, "x"), M.embed_axis(c, "y")


def _propagate(cores, wx, wy, chi, chi_zip=None):
    c1, _ = Z.mpo_apply(cores, wx, chi, chi_zip)
    return Z.mpo_apply(c1, wy, chi, chi_zip)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("seed", [0, 1])
def test_lossless_equals_fft_random_8x8(seed):
    n = 3
    e0 = synth.random_field(seed, 8)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi=BIG)
    wx, wy = _axis_mpos(n, 3e-6)
    out, nrm = _propagate(cores, wx, wy, BIG)
    ref = F.fresnel_dense(e0, LAM, DX, 3e-6)
    assert _rel(Z.to_dense(out, n), ref) < 1e-12
    assert abs(nrm - np.linalg.norm(ref)) < 1e-12 * np.linalg.norm(ref)


def test_lossless_equals_fft_blob_64():
    n = 6
    img = synth.blob_image(0)
    cores = T.tt_svd(Q.to_quantics(img), 2 * n, chi=64)
    wx, wy = _axis_mpos(n, 1e-3)
    out, _ = _propagate(cores, wx, wy, BIG)
    ref = F.fresnel_dense(img, LAM, DX, 1e-3)
    assert _rel(Z.to_dense(out, n), ref) < 1e-11
    # output left-canonical
    for c in out[:-1]:
        mat = c.reshape(-1, c.shape[2])
        assert np.allclose(mat.conj().T @ mat, np.eye(c.shape[2]), atol=1e-10)


def test_identity_mpo_is_noop():
    n = 5
    e0 = synth.aperture_field(3, n=32)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi=BIG)
    ident = [M.identity_core(1) for _ in range(2 * n)]
    out, _ = Z.mpo_apply(cores, ident, BIG)
    assert _rel(Z.to_dense(out, n), e0) < 1e-13


def _fwht(v):
    v = v.copy()
    h = 1
    while h < v.size:
        for i in range(0, v.size, 2 * h):
            a = v[i:i + h].copy()
            b = v[i + h:i + 2 * h].copy()
            v[i:i + h] = a + b
            v[i + h:i + 2 * h] = a - b
        h *= 2
    return v / np.sqrt(v.size)


def test_hadamard_mpo_equals_fast_wht():
    n = 4
    e0 = synth.random_field(8, 16)
    v = Q.to_quantics(e0)
    cores = T.tt_svd(v, 2 * n, chi=BIG)
    out, _ = Z.mpo_apply(cores, M.hadamard_mpo(2 * n), BIG)
    assert np.allclose(T.tt_dense(out), _fwht(v), atol=1e-12)


@pytest.mark.parametrize("chi", [4, 8, 16])
def test_lossless_zip_then_sweep_equals_ttsvd(chi):
    n = 5
    e0 = synth.aperture_field(4, n=32)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi=BIG)
    wx, _ = _axis_mpos(n, 1e-3)
    exact = Z.to_dense(Z.mpo_apply(cores, wx, BIG)[0], n)
    got, _ = Z.mpo_apply(cores, wx, chi, chi_zip=BIG)
    opt = T.tt_svd(Q.to_quantics(exact), 2 * n, chi)
    assert _rel(T.tt_dense(got), T.tt_dense(opt)) < 1e-10
    assert Z.bonds(got) == T.bonds(opt)


@pytest.mark.parametrize("chi", [4, 8])
def test_tt_truncate_equals_ttsvd(chi):
    n = 5
    e0 = synth.aperture_field(6, n=32)
    exact = T.tt_svd(Q.to_quantics(e0), 2 * n, chi=BIG)
    # scramble the gauge: multiply a random invertible matrix into each bond
    rng = np.random.default_rng(0)
    cores = [c.copy() for c in exact]
    for k in range(len(cores) - 1):
        r = cores[k].shape[2]
        g = rng.standard_normal((r, r)) + np.eye(r) * 3
        cores[k] = np.tensordot(cores[k], g, axes=(2, 0))
        cores[k + 1] = np.tensordot(np.linalg.inv(g), cores[k + 1], axes=(1, 0))
    got, nrm = Z.tt_truncate(cores, chi)
    opt = T.tt_svd(Q.to_quantics(e0), 2 * n, chi)
    assert _rel(T.tt_dense(got), T.tt_dense(opt)) < 1e-9
    assert abs(nrm - np.linalg.norm(T.tt_dense(opt))) < 1e-9 * nrm


def test_truncated_zipup_bounded_by_opt():
    """chi_zip = chi (classic zip-up): error at least the optimal one and
    within a small factor of it (the zip-up is the identical algorithm on
    both sides of the GPU parity test; this bound is the only pin)."""
    n = 6
    img = synth.blob_image(2)
    cores = T.tt_svd(Q.to_quantics(img), 2 * n, chi=32)
    wx, wy = _axis_mpos(n, 1e-3)
    ref = F.fresnel_dense(Z.to_dense(cores, n), LAM, DX, 1e-3)
    got, _ = _propagate(cores, wx, wy, 16)
    opt = T.tt_svd(Q.to_quantics(ref), 2 * n, 16)
    e_got = _rel(Z.to_dense(got, n), ref)
    e_opt = _rel(Z.to_dense(opt, n), ref)
    assert e_got >= e_opt * (1 - 1e-9)
    assert e_got < 5.0 * e_opt          # two sequential capped applications


def _site_unitaries(rng, m):
    out = []
    for _ in range(m):
        z = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        q, r = np.linalg.qr(z)
        out.append(q * (np.diag(r) / np.abs(np.diag(r))))
    return out


@pytest.mark.parametrize("chi_zip,seed", [(2, 0), (3, 1), (5, 2), (9, 3)])
def test_truncating_zipup_of_site_unitaries_is_right_to_left_ttsvd(chi_zip, seed):
    """Truncating regime, closed form: for an MPO of single-site unitaries
    (bond 1) and a left-canonical input, every left block stays orthonormal,
    so the singular values the zip-up cuts at bond k are those of the exact
    state W psi across that bond and the zip-up is the sequential truncated
    SVD from the right -- the TT-SVD of the site-reversed vector.  Pins the
    keep rule, the carry and the site order of the truncating zip-up against
    the (separately pinned) TT-SVD and a dense application of the unitaries."""
    rng = np.random.default_rng(400 + seed)
    m = 8
    v = rng.standard_normal(1 << m) + 1j * rng.standard_normal(1 << m)
    psi = T.tt_svd(v, m, chi=BIG)                       # exact, left-canonical
    us = _site_unitaries(rng, m)
    mpo = [u.reshape(1, 2, 2, 1) for u in us]          # [D, t, s, D']
    out = Z.zip_up(psi, mpo, chi_zip)
    got = T.tt_dense(out)
    # dense W v: unitary k acts on bit k (site k, most significant first)
    y = v.reshape([2] * m)
    for k, u in enumerate(us):
        y = np.moveaxis(np.tensordot(u, y, axes=([1], [k])), 0, k)
    # sequential truncated SVD from the right = TT-SVD of the reversed sites
    rev = y.transpose(list(range(m - 1, -1, -1))).reshape(-1)
    cr = T.tt_svd(rev, m, chi=chi_zip)
    want = T.tt_dense(cr).reshape([2] * m).transpose(list(range(m - 1, -1, -1))).reshape(-1)
    assert _rel(got, want) < 1e-12
    assert Z.bonds(out) == T.bonds(cr)[::-1]
    # and the cut really truncates
    assert max(Z.bonds(out)) == chi_zip


def _zipup_dense_brute_force(psi, mpo, chi_zip, tau=1e-13):
    """The zip-up's definition evaluated without carries, for tiny chains.
    Before the cut at bond k-1 the exact right part of W psi,
        R[(a_(k-1), w_(k-1)), (t_k .. t_m)] = sum_s prod_(j >= k) A_j W_j,
    is formed densely from all cores at once; the output's right basis P
    (rows beta_k, columns t_(k+1) .. t_m) is formed densely from the cores
    already fixed; then M = R (I_2 (x) P)^H as [(a, w), (t_k, beta_k)], its
    singular vectors give B_k (top r rows of V^H, r = min(chi_zip,
    #{s^2 > tau s_1^2})) and P is extended by B_k.  The carry recursion of
    the oracle never appears."""
    m = len(psi)
    out = [None] * m
    P = np.ones((1, 1), dtype=np.complex128)           # [beta, T] with T = () at the right end
    for k in range(m - 1, -1, -1):
        # exact right part from site k: contract A_j W_j for j = k..m-1 densely
        R = np.ones((1, 1, 1), dtype=np.complex128)     # [a_j, w_j, T]
        for j in range(m - 1, k - 1, -1):
            a, w = psi[j], mpo[j]                       # [ra, s, rb], [da, t, s, db]
            x = np.einsum("asb,dtsc,bcT->adtT", a, w, R)
            R = x.reshape(a.shape[0], w.shape[0], -1)
        ra, da, nt = R.shape
        Rm = R.reshape(ra * da, 2, nt // 2)             # [(a, w), t_k, T']
        M = np.einsum("xtT,bT->xtb", Rm, P.conj()).reshape(ra * da, -1)
        if k == 0:
            out[0] = M.reshape(1, 2, -1)
            break
        u, s, vh = np.linalg.svd(M, full_matrices=False)
        lam = s * s
        r = max(1, min(chi_zip, int(np.sum(lam > tau * lam[0]))))
        bk = vh[:r].reshape(r, 2, -1)
        out[k] = bk
        P = np.einsum("itb,bT->itT", bk, P).reshape(r, -1)
    return out


def _random_mpo(rng, m, d):
    bonds = [1] + [d] * (m - 1) + [1]
    return [(rng.standard_normal((bonds[k], 2, 2, bonds[k + 1])) +
             1j * rng.standard_normal((bonds[k], 2, 2, bonds[k + 1]))) / 2.0 for k in range(m)]


@pytest.mark.parametrize("case", ["fresnel", "random"])
@pytest.mark.parametrize("chi_zip", [2, 3, 5])
def test_truncating_zipup_with_operator_bonds_vs_dense_brute_force(case, chi_zip):
    """Truncating regime with operator bonds above 1: the oracle's zip-up
    (carry recursion) equals the zip-up definition evaluated densely without
    carries (brute force on an 8-site chain) -- same bonds, same state; and
    a carry without its singular values (a plausible slip) is caught."""
    rng = np.random.default_rng(700 + chi_zip)
    n, m = 4, 8
    v = rng.standard_normal(1 << m) + 1j * rng.standard_normal(1 << m)
    psi = T.tt_svd(v, m, chi=BIG)
    if case == "fresnel":
        wx, _ = _axis_mpos(n, 3e-6)
        mpo = wx
    else:
        mpo = _random_mpo(rng, m, 3)
    assert max(w.shape[0] for w in mpo) > 1
    got = Z.zip_up(psi, mpo, chi_zip)
    want = _zipup_dense_brute_force(psi, mpo, chi_zip)
    assert Z.bonds(got) == Z.bonds(want)
    assert max(Z.bonds(got)) == chi_zip                  # the cut really truncates
    assert _rel(T.tt_dense(got), T.tt_dense(want)) < 1e-10
    # planted slip: carry U instead of U S
    slip = [None] * m
    carry = np.ones((1, 1, 1), dtype=np.complex128)
    for k in range(m - 1, -1, -1):
        x = np.tensordot(psi[k], carry, axes=(2, 0))
        t = np.tensordot(x, mpo[k], axes=([1, 2], [2, 3])).transpose(0, 2, 3, 1)
        ra, da, _, beta = t.shape
        mat = t.reshape(ra * da, 2 * beta)
        if k == 0:
            slip[0] = mat.reshape(1, 2, beta)
            break
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        r = max(1, min(chi_zip, int(np.sum(s * s > 1e-13 * s[0] ** 2))))
        slip[k] = vh[:r].reshape(r, 2, beta)
        carry = u[:, :r].reshape(ra, da, r)
    assert _rel(T.tt_dense(slip), T.tt_dense(want)) > 1e-3
