"""GPU parity of the three-stage propagator (QFT, diagonal transfer
function, inverse QFT: Sec. 6.1, Fig. of the MPO product), the diagonal-site
contraction, the non-paraxial angular-spectrum propagator (Sec. 6.1), the
element-wise product, the PSF and image formation (Sec. 5).

Bars: FP32 lossless 1e-5 against the dense FFT definitions; truncated 1e-4
against the oracle's zip-up + sweep of the same stages with the oracle's own
MPOs (sequential SVD of the dense operators, the same left-canonical form
as the library's), with equal bonds.
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import fresnel as F
from oracle import imaging as I
from oracle import mpo as OM
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

pytestmark = pytest.mark.gpu
LAM, DX = 500e-9, 1e-6


def _api():
    from paper_2510_23089_amd import api
    return api


def _oracle_stages(n, z, dispersion="parabolic"):
    qm = OM.qft_br_matrix(n)
    q = OM.mpo_from_matrix(qm, n)
    iq = OM.mpo_from_matrix(qm.conj().T, n)
    if dispersion == "parabolic":
        t = F.transfer_1d(1 << n, LAM, DX, z)
    else:
        t = F.transfer_lattice_1d(1 << n, LAM, DX, z)
    d = OM.diag_mpo_from_vector(t[OM.bit_reverse_perm(n)], n)
    return q, d, iq


def _oracle_three_stage(cores, n, z, chi, dispersion="parabolic"):
    q, d, iq = _oracle_stages(n, z, dispersion)
    out = cores
    for ax in ("x", "y"):
        for w in (q, d, iq):
            out, _ = Z.mpo_apply(out, OM.embed_axis(w, ax), chi, tau=1e-13)
    return out


@pytest.mark.parametrize("route", ["svd", "pauli"])
def test_three_stage_lossless_vs_fft(route):
    torch = need_gpu()
    api = _api()
    say("three-stage lossless", route)
    n, z = 6, 1e-3
    img = synth.blob_image(2)
    psi = api.tt_encode(torch.from_numpy(img).float().cuda(), 64)
    prop = api.FresnelThreeStage(n, LAM, DX, z, route=route)
    out = prop(psi, 64, chi_zip=128)
    got = api.tt_to_dense(out).cpu().numpy()
    api.check_status()
    assert rel(got, F.fresnel_dense(img, LAM, DX, z)) < 1e-5


def test_three_stage_lattice_bessel_lossless_vs_fft():
    torch = need_gpu()
    api = _api()
    n, z = 6, 2e-4
    e0 = synth.aperture_field(3, n=1 << n)
    psi = api.tt_encode(torch.from_numpy(e0).to(torch.complex64).cuda(), 64)
    prop = api.FresnelThreeStage(n, LAM, DX, z, route="bessel", dispersion="lattice")
    got = api.tt_to_dense(prop(psi, 64, chi_zip=128)).cpu().numpy()
    api.check_status()
    u = F.lattice_matrix_1d(1 << n, LAM, DX, z)
    assert rel(got, u @ e0 @ u.T) < 1e-5


@pytest.mark.parametrize("route", ["svd", "pauli"])
def test_three_stage_identically_truncated_vs_oracle(route):
    torch = need_gpu()
    api = _api()
    n, z, chi = 6, 1e-3, 12
    say("three-stage truncated", route)
    e0 = synth.aperture_field(5, n=1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi, tau=1e-13)
    psi = api.MPS.from_host(cores, chi_cap=chi)
    prop = api.FresnelThreeStage(n, LAM, DX, z, route=route)
    out = prop(psi, chi)
    got = api.tt_to_dense(out).cpu().numpy()
    api.check_status()
    ref = _oracle_three_stage(cores, n, z, chi)
    err = rel(got, Z.to_dense(ref, n))
    say("  rel err", err)
    assert err < 1e-4
    assert out.host_bonds() == Z.bonds(ref)


def test_diagonal_site_contraction_equals_the_general_one():
    """The same diagonal MPO applied with its sites marked diagonal (the
    per-bit product of half the depth) and marked general."""
    torch = need_gpu()
    api = _api()
    from paper_2510_23089_amd import mpo_build as B
    n, z, chi = 7, 2e-3, 24
    e0 = synth.aperture_field(6, n=1 << n)
    psi = api.tt_encode(torch.from_numpy(e0).to(torch.complex64).cuda(), chi)
    d = B.diag_fresnel(n, LAM, DX, z)
    c, kind = B.embed(d, "x", diag=True)
    w_diag = api.MPO(c, kind, d_cap=max(B.bonds(d)))
    w_gen = api.MPO(c, [0 if k == 2 else k for k in kind], d_cap=max(B.bonds(d)))
    a = api.mpo_apply(psi, w_diag, chi)
    b = api.mpo_apply(psi, w_gen, chi)
    da, db = api.tt_to_dense(a).cpu().numpy(), api.tt_to_dense(b).cpu().numpy()
    api.check_status()
    assert a.host_bonds() == b.host_bonds()
    assert rel(da, db) < 1e-6


def test_angular_spectrum_lossless_and_truncated_vs_oracle():
    torch = need_gpu()
    api = _api()
    n, z = 6, 60e-6
    say("angular spectrum")
    e0 = synth.aperture_field(7, n=1 << n)
    prop = api.AngularSpectrum(n, LAM, DX, z)
    psi = api.tt_encode(torch.from_numpy(e0).to(torch.complex64).cuda(), 64)
    # the 2-D diagonal has operator bond 64 here, and the zip-up's carry
    # (not yet orthogonalised on its left) needs 256 directions at one bond
    # to stay lossless (the oracle's lossless run needs the same)
    got = api.tt_to_dense(prop(psi, 64, chi_zip=256)).cpu().numpy()
    api.check_status()
    exact = F.angular_spectrum_dense(e0, LAM, DX, z)
    assert rel(got, exact) < 1e-5
    # it is not the paraxial propagator at this distance and pixel pitch
    assert rel(exact, F.fresnel_dense(e0, LAM, DX, z)) > 1e-3
    # truncated: the oracle's stages with its own MPOs
    chi = 10
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi, tau=1e-13)
    qm = OM.qft_br_matrix(n)
    q = OM.mpo_from_matrix(qm, n)
    iq = OM.mpo_from_matrix(qm.conj().T, n)
    tr = F.angular_spectrum_transfer(1 << n, LAM, DX, z)
    r = OM.bit_reverse_perm(n)
    d2 = OM.diag_mpo_from_vector(Q.to_quantics(tr[r][:, r]), 2 * n)
    ref = cores
    for w in (OM.embed_axis(q, "x"), OM.embed_axis(q, "y"), d2, OM.embed_axis(iq, "y"), OM.embed_axis(iq, "x")):
        ref, _ = Z.mpo_apply(ref, w, chi, tau=1e-13)
    out = prop(api.MPS.from_host(cores, chi_cap=chi), chi)
    got = api.tt_to_dense(out).cpu().numpy()
    api.check_status()
    err = rel(got, Z.to_dense(ref, n))
    say("  truncated rel err", err, "max diag bond", max(c.shape[3] for c in d2))
    assert err < 1e-4
    assert out.host_bonds() == Z.bonds(ref)


def test_hadamard_product_lossless_truncated_and_conjugate():
    torch = need_gpu()
    api = _api()
    n = 5
    ea = synth.aperture_field(8, n=1 << n)
    eb = synth.aperture_field(9, n=1 << n)
    a = api.tt_encode(torch.from_numpy(ea).to(torch.complex64).cuda(), 32)
    b = api.tt_encode(torch.from_numpy(eb).to(torch.complex64).cuda(), 32)
    out = api.tt_hadamard(a, b, 32, chi_zip=64)
    got = api.tt_to_dense(out).cpu().numpy()
    assert rel(got, ea * eb) < 1e-5
    pw = api.tt_to_dense(api.tt_hadamard(a, a, 32, conj_a=True, chi_zip=64)).cpu().numpy()
    assert rel(pw, np.abs(ea) ** 2) < 1e-5
    api.check_status()
    chi = 8
    ca = T.tt_svd(Q.to_quantics(ea), 2 * n, 32, tau=1e-13)
    cb = T.tt_svd(Q.to_quantics(eb), 2 * n, chi, tau=1e-13)
    ref, _ = Z.mpo_apply(cb, I.diag_mpo_from_mps(ca), chi, tau=1e-13)
    # bonds are compared in FP64: at bond 3 the oracle's sweep drops an
    # eigenvalue 0.998e-13 lambda_1, 0.2 % under the keep threshold (singular
    # value ratio 3.2e-7, about five FP32 ulps), which FP32 data cannot place
    # on either side of the threshold
    for dt, tol in ((torch.complex64, 1e-4), (torch.complex128, 1e-10)):
        out = api.tt_hadamard(api.MPS.from_host(ca, chi_cap=32, dtype=dt), api.MPS.from_host(cb, chi_cap=chi, dtype=dt),
                              chi)
        got = api.tt_to_dense(out).cpu().numpy()
        api.check_status()
        err = rel(got, Z.to_dense(ref, n))
        say("hadamard truncated rel err", dt, err)
        assert err < tol
        if dt == torch.complex128:
            assert out.host_bonds() == Z.bonds(ref)


def test_psf_and_image_formation_vs_oracle():
    torch = need_gpu()
    api = _api()
    n = 6
    N = 1 << n
    a, b = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    disk = (((a - N / 2) ** 2 + (b - N / 2) ** 2) <= (N / 4) ** 2).astype(np.float64)
    pupil = disk * np.exp(1j * synth.smoothed_phase(11, N, 3.0, 1.0))
    p = api.tt_encode(torch.from_numpy(pupil).to(torch.complex64).cuda(), 64)
    phi, ps = api.psf(p, 64, chi_zip=256)        # the product's zip-up needs 256 at one bond
    got_phi = api.tt_to_dense(phi).cpu().numpy()
    got_psf = api.tt_to_dense(ps).cpu().numpy()
    api.check_status()
    assert rel(got_phi, I.focal_field_br(pupil)) < 1e-5
    assert rel(got_psf, I.psf_br(pupil)) < 1e-5
    # image of a scene through a (natural-order) PSF: circular convolution / N
    obj = synth.blob_image(3)
    kern = np.fft.fftshift(I.psf_br(pupil)[np.argsort(OM.bit_reverse_perm(n))][:, np.argsort(OM.bit_reverse_perm(n))])
    o = api.tt_encode(torch.from_numpy(obj).float().cuda(), 64)
    k = api.tt_encode(torch.from_numpy(kern).to(torch.complex64).cuda(), 64)
    img = api.tt_to_dense(api.image_formation(o, k, 64, chi_zip=256)).cpu().numpy()
    api.check_status()
    assert rel(img, I.image_formation(obj, kern)) < 1e-5
