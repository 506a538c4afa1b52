"""GPU parity of the precision forms: bfloat16 contractions and the
full-precision two-site fitting sweep (refine), against the float64 oracle.

Bars (relative L2 of the dense result): BF16 zip-up + plain sweep against the
oracle's float64 zip-up + sweep <= 3e-3; refine after a BF16 zip-up against
the oracle's float64 zip-up + fitting sweep <= 1e-4; FP32 refine against the
same oracle <= 1e-4; FP64 refine <= 1e-10.  Inputs and MPO cores are the
oracle's, uploaded; the GPU side never feeds the oracle.
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import fresnel as F
from oracle import mpo as OM
from oracle import quantics as Q
from oracle import refine as RF
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

pytestmark = pytest.mark.gpu
LAM, DX = 500e-9, 1e-6


def _api():
    from paper_2510_23089_amd import api
    return api


def _bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", [(16, 16, 16), (64, 48, 80), (130, 70, 200), (7, 300, 33)])
def test_cgemm_bf16(shape):
    torch = need_gpu()
    import ctypes
    from paper_2510_23089_amd import _lib as L
    lib = L.load()
    M, N, K = shape
    rng = np.random.default_rng(M + N + K)
    a = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))).astype(np.complex64)
    b = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))).astype(np.complex64)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.zeros((M, N), dtype=torch.complex64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for ca, cb in ((0, 0), (1, 0), (0, 1)):
        L.check(lib.tt_cgemm(M, N, K, da.data_ptr(), K, ca, db.data_ptr(), N, cb, dc.data_ptr(), N, L.PREC_BF16, s),
                "tt_cgemm")
        torch.cuda.synchronize()
        ar = _bf16(a.real) + 1j * _bf16(a.imag)
        br = _bf16(b.real) + 1j * _bf16(b.imag)
        ar = ar.conj() if ca else ar
        br = br.conj() if cb else br
        ref = ar @ br
        got = dc.cpu().numpy()
        # bf16 x bf16 products are exact in FP32; only the FP32 sums round
        assert rel(got, ref) < 2e-6, (ca, cb, rel(got, ref))
        # and it is not the FP32 product
        full = (a.conj() if ca else a).astype(np.complex128) @ (b.conj() if cb else b).astype(np.complex128)
        assert rel(got, full) > 1e-4


def _case(n, z, chi_in, seed):
    e0 = synth.aperture_field(seed, n=1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi_in, tau=1e-13)
    c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    return cores, OM.embed_axis(c, "x"), OM.embed_axis(c, "y")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,chi,z", [(4, 6, 30e-6), (5, 12, 60e-6), (6, 16, 150e-6)])
def test_refine_vs_oracle(prec, n, chi, z):
    torch = need_gpu()
    api = _api()
    say("refine", prec, n, chi)
    cores, wx, wy = _case(n, z, 2 * chi, seed=n)
    ref, nref = RF.mpo_apply_refined(cores, wx, chi, tau=1e-13)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    psi = api.MPS.from_host(cores, chi_cap=2 * chi, dtype=dt)
    out = api.mpo_apply(psi, api.MPO(wx, dtype=dt), chi, refine=True)
    api.check_status()
    got = api.tt_to_dense(out).cpu().numpy()
    err = rel(got, Z.to_dense(ref, n))
    say("  rel err", err)
    assert out.host_bonds() == T.bonds(ref)
    assert err < (1e-4 if prec == "fp32" else 1e-10)
    assert abs(float(out.norm.cpu()[0]) - nref) < (1e-5 if prec == "fp32" else 1e-11) * nref
    # left-canonical output
    for c in out.host_cores()[:-1]:
        mat = c.reshape(-1, c.shape[2]).astype(np.complex128)
        assert np.allclose(mat.conj().T @ mat, np.eye(c.shape[2]), atol=1e-4 if prec == "fp32" else 1e-10)


@pytest.mark.parametrize("n,chi,z", [(5, 12, 60e-6), (6, 16, 150e-6), (7, 24, 300e-6)])
def test_bf16_then_refine_vs_oracle(n, chi, z):
    torch = need_gpu()
    api = _api()
    say("bf16", n, chi)
    cores, wx, wy = _case(n, z, 2 * chi, seed=10 + n)
    plain, _ = Z.mpo_apply(cores, wx, chi, tau=1e-13)
    fit, _ = RF.mpo_apply_refined(cores, wx, chi, tau=1e-13)
    psi = api.MPS.from_host(cores, chi_cap=2 * chi)
    W = api.MPO(wx)
    bf = api.mpo_apply(psi, W, chi, prec="bf16")
    bfr = api.mpo_apply(psi, W, chi, prec="bf16", refine=True)
    api.check_status()
    e_bf = rel(api.tt_to_dense(bf).cpu().numpy(), Z.to_dense(plain, n))
    e_bfr = rel(api.tt_to_dense(bfr).cpu().numpy(), Z.to_dense(fit, n))
    say("  bf16 vs oracle %.3e, bf16 + refine vs refined oracle %.3e" % (e_bf, e_bfr))
    assert e_bf < 3e-3
    assert e_bfr < 1e-4


def test_bf16_refine_full_size_propagation():
    """1024^2 aperture field, chi 64, both axes: the precision form at the
    benchmark's field size against the oracle's float64 zip-up + fit."""
    torch = need_gpu()
    api = _api()
    n, chi, z = 10, 64, 2e-3
    e0 = synth.aperture_field(0, n=1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi, tau=1e-13)
    c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    wx, wy = OM.embed_axis(c, "x"), OM.embed_axis(c, "y")
    r1, _ = RF.mpo_apply_refined(cores, wx, chi, tau=1e-13)
    r2, _ = RF.mpo_apply_refined(r1, wy, chi, tau=1e-13)
    ref = Z.to_dense(r2, n)
    psi = api.MPS.from_host(cores, chi_cap=chi)
    mid = api.mpo_apply(psi, api.MPO(wx), chi, prec="bf16", refine=True)
    out = api.mpo_apply(mid, api.MPO(wy), chi, prec="bf16", refine=True)
    api.check_status()
    err = rel(api.tt_to_dense(out).cpu().numpy(), ref)
    say("full size bf16 + refine rel err %.3e" % err)
    assert err < 1e-4
