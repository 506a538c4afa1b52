"""GPU parity of the hot path against the CPU float64 oracle.

Bars: FP32 path at untruncated bond dimension <= 1e-5 relative L2 against the
exact (dense FFT) result; against the oracle's identically truncated result
<= 1e-4; FP64 path <= 1e-10.  Inputs are seeded synthetic fields; every
oracle input (cores, MPOs) is computed by the oracle itself and uploaded.
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import fresnel as F
from oracle import mpo as OM
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

pytestmark = pytest.mark.gpu
LAM, DX = 500e-9, 1e-6
BIG = 1 << 20


def _api():
    from paper_2510_23089_amd import api
    return api


def _oracle_mpos(n, z):
    c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    return OM.embed_axis(c, "x"), OM.embed_axis(c, "y"), c


def _dev_mpo(api, torch, cores, dtype):
    return api.MPO(cores, None, dtype=dtype)


def _dense(api, psi):
    return api.tt_to_dense(psi).cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_encode_blob_vs_oracle(prec):
    torch = need_gpu()
    api = _api()
    img = synth.blob_image(0)
    dt = torch.float32 if prec == "fp32" else torch.float64
    d_img = torch.from_numpy(img).to(dt).cuda()
    for chi, tol in ((64, 1e-5), (32, 1e-4), (8, 1e-4)):
        say("encode", prec, chi)
        psi = api.tt_encode(d_img, chi, prec=prec)
        api.check_status()
        got = _dense(api, psi)
        ref_cores = T.tt_svd(Q.to_quantics(img), 12, chi, tau=1e-13)
        ref = Z.to_dense(ref_cores, 6)
        if prec == "fp64":
            tol = 1e-10
        assert rel(got, ref) < tol, (chi, rel(got, ref))
        if chi < 64:
            assert psi.host_bonds() == T.bonds(ref_cores)
        assert abs(float(psi.norm.cpu()[0]) - np.linalg.norm(ref)) < 1e-5 * np.linalg.norm(ref)


def test_to_dense_roundtrip_random():
    torch = need_gpu()
    api = _api()
    for n in (1, 2, 3, 5):
        say("to_dense", n)
        e0 = synth.random_field(n, 1 << n)
        cores = T.tt_svd(Q.to_quantics(e0), 2 * n, BIG)
        psi = api.MPS.from_host(cores, chi_cap=max(2, 1 << n))
        got = _dense(api, psi)
        assert rel(got, e0) < 1e-6


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_apply_lossless_random_8x8(prec):
    torch = need_gpu()
    api = _api()
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    n = 3
    z = 3e-6
    wx, wy, _ = _oracle_mpos(n, z)
    for seed in (0, 1):
        say("lossless 8x8", prec, seed)
        e0 = synth.random_field(seed, 8)
        cores = T.tt_svd(Q.to_quantics(e0), 2 * n, BIG)
        psi = api.MPS.from_host(cores, chi_cap=8, dtype=dt)
        mx = _dev_mpo(api, torch, wx, dt)
        my = _dev_mpo(api, torch, wy, dt)
        mid = api.mpo_apply(psi, mx, 64, chi_cap=64)
        out = api.mpo_apply(mid, my, 64, chi_cap=64)
        api.check_status()
        ref = F.fresnel_dense(e0, LAM, DX, z)
        tol = 1e-5 if prec == "fp32" else 1e-11
        assert rel(_dense(api, out), ref) < tol
        assert abs(float(out.norm.cpu()[0]) - np.linalg.norm(ref)) < tol * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_apply_lossless_blob_64(prec):
    """Untruncated bond dimension (chi = 64 = exact max rank of a 64x64 grid)."""
    torch = need_gpu()
    api = _api()
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    n = 6
    z = 1e-3
    img = synth.blob_image(0)
    cores = T.tt_svd(Q.to_quantics(img), 12, 64)
    wx, wy, _ = _oracle_mpos(n, z)
    psi = api.MPS.from_host(cores, chi_cap=64, dtype=dt)
    say("lossless blob", prec)
    mid = api.mpo_apply(psi, _dev_mpo(api, torch, wx, dt), 64, chi_zip=128, chi_cap=64)
    out = api.mpo_apply(mid, _dev_mpo(api, torch, wy, dt), 64, chi_zip=128, chi_cap=64)
    api.check_status()
    ref = F.fresnel_dense(img, LAM, DX, z)
    tol = 1e-5 if prec == "fp32" else 1e-10
    assert rel(_dense(api, out), ref) < tol


@pytest.mark.parametrize("chi", [8, 16, 32])
def test_apply_truncated_blob_vs_oracle(chi):
    """Identically truncated: GPU zip-up + sweep vs the oracle's, same input
    cores and MPO (both from the oracle)."""
    torch = need_gpu()
    api = _api()
    n = 6
    z = 1e-3
    img = synth.blob_image(3)
    cores = T.tt_svd(Q.to_quantics(img), 12, 32)
    wx, wy, _ = _oracle_mpos(n, z)
    c1, _ = Z.mpo_apply(cores, wx, chi, tau=1e-13)
    ref_cores, ref_norm = Z.mpo_apply(c1, wy, chi, tau=1e-13)
    ref = Z.to_dense(ref_cores, n)
    for prec, tol in (("fp32", 1e-4), ("fp64", 1e-10)):
        say("truncated blob", chi, prec)
        dt = torch.complex64 if prec == "fp32" else torch.complex128
        psi = api.MPS.from_host(cores, chi_cap=32, dtype=dt)
        mid = api.mpo_apply(psi, _dev_mpo(api, torch, wx, dt), chi)
        out = api.mpo_apply(mid, _dev_mpo(api, torch, wy, dt), chi)
        api.check_status()
        assert rel(_dense(api, out), ref) < tol, (prec, rel(_dense(api, out), ref))
        assert out.host_bonds() == Z.bonds(ref_cores)


def test_truncate_vs_oracle():
    torch = need_gpu()
    api = _api()
    n = 5
    e0 = synth.aperture_field(6, n=32)
    exact = T.tt_svd(Q.to_quantics(e0), 2 * n, BIG)
    for chi in (4, 8, 32):
        say("truncate", chi)
        ref_cores, _ = Z.tt_truncate(exact, chi, tau=1e-13)
        psi = api.MPS.from_host(exact, chi_cap=32)
        api.tt_truncate(psi, chi)
        api.check_status()
        assert rel(_dense(api, psi), Z.to_dense(ref_cores, n)) < (1e-4 if chi < 32 else 1e-5)
        if chi < 32:
            assert psi.host_bonds() == Z.bonds(ref_cores)


def test_product_mpo_end_to_end_blob():
    """The library's own host-built Fresnel MPO (QFT^H diag QFT route) with
    GPU encode and propagation, untruncated, vs the dense FFT oracle."""
    torch = need_gpu()
    api = _api()
    img = synth.blob_image(1)
    say("product end-to-end")
    d_img = torch.from_numpy(img).to(torch.float32).cuda()
    psi = api.tt_encode(d_img, 64)
    prop = api.FresnelPropagator(6, LAM, DX, 1e-3)
    out = prop(psi, 64, chi_zip=128)
    api.check_status()
    ref = F.fresnel_dense(img, LAM, DX, 1e-3)
    assert rel(_dense(api, out), ref) < 1e-5


def test_batched_apply_uneven_chi_vs_oracle():
    """Three fields in one batch: different input fields, different MPOs
    (different z, so different bond profiles, zero-padded to a common one)
    and different per-field bond caps; each field vs the oracle."""
    torch = need_gpu()
    api = _api()
    n = 6
    zs = (0.3e-3, 1e-3, 2e-3)
    chis = (8, 16, 32)
    imgs = [synth.blob_image(s) for s in (4, 5, 6)]
    cores = [T.tt_svd(Q.to_quantics(im), 12, 32) for im in imgs]
    mp = [_oracle_mpos(n, z) for z in zs]
    psi = api.MPSBatch(3, 12, 32)
    for f in range(3):
        psi.fill_from(api.MPS.from_host(cores[f], chi_cap=32), f)
    wx = api.MPOBatch([w[0] for w in mp])
    wy = api.MPOBatch([w[1] for w in mp])
    chi_dev = torch.tensor(chis, dtype=torch.int32, device="cuda")
    say("batched apply")
    mid = api.mpo_apply_batched(psi, wx, 32, chi_dev=chi_dev)
    out = api.mpo_apply_batched(mid, wy, 32, chi_dev=chi_dev)
    dense = api.tt_to_dense_batched(out).cpu().numpy()
    api.check_status()
    for f in range(3):
        c1, _ = Z.mpo_apply(cores[f], mp[f][0], chis[f], tau=1e-13)
        ref_cores, _ = Z.mpo_apply(c1, mp[f][1], chis[f], tau=1e-13)
        ref = Z.to_dense(ref_cores, n)
        assert rel(dense[f], ref) < 1e-4, (f, rel(dense[f], ref))
        assert [int(x) for x in out.bonds[f].cpu()] == Z.bonds(ref_cores)
        assert abs(float(out.norms[f].cpu()) - np.linalg.norm(ref)) < 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mixed_batch_full_rank_near_singular_and_capped(prec):
    """One batch holding a full-rank random field (every sweep step keeps all
    its directions), a smooth blob whose spectrum reaches the keep threshold
    (steps that drop near-zero directions) and a field under a per-field cap
    of 8.  Each field vs the oracle's identically truncated result with equal
    bonds and norm, and every output core left-orthonormal."""
    torch = need_gpu()
    api = _api()
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    n, z, cap = 5, 1e-3, 32
    fields = [synth.random_field(3, 32), synth.blob_image(9, n=32), synth.aperture_field(2, n=32)]
    chis = (32, 32, 8)
    cores = [T.tt_svd(Q.to_quantics(e), 2 * n, cap, tau=1e-13) for e in fields]
    wx, wy, _ = _oracle_mpos(n, z)
    psi = api.MPSBatch(3, 2 * n, cap, dtype=dt)
    for f in range(3):
        psi.fill_from(api.MPS.from_host(cores[f], chi_cap=cap, dtype=dt), f)
    mx = api.MPOBatch([wx] * 3, dtype=dt)
    my = api.MPOBatch([wy] * 3, dtype=dt)
    chi_dev = torch.tensor(chis, dtype=torch.int32, device="cuda")
    say("mixed batch", prec)
    mid = api.mpo_apply_batched(psi, mx, cap, chi_dev=chi_dev)
    out = api.mpo_apply_batched(mid, my, cap, chi_dev=chi_dev)
    dense = api.tt_to_dense_batched(out).cpu().numpy()
    api.check_status()
    # orthonormality is checked unweighted: a kept direction with singular
    # value sigma_i is resolved to about eps sigma_1 / sigma_i, and the blob
    # keeps directions down to the threshold's sigma_i / sigma_1 = 3e-7
    tol, otol = (1e-4, 1e-5) if prec == "fp32" else (1e-10, 1e-9)
    for f in range(3):
        c1, _ = Z.mpo_apply(cores[f], wx, chis[f], tau=1e-13)
        ref_cores, _ = Z.mpo_apply(c1, wy, chis[f], tau=1e-13)
        ref = Z.to_dense(ref_cores, n)
        assert rel(dense[f], ref) < tol, (f, rel(dense[f], ref))
        assert [int(x) for x in out.bonds[f].cpu()] == Z.bonds(ref_cores), f
        assert abs(float(out.norms[f].cpu()) - np.linalg.norm(ref)) < tol * np.linalg.norm(ref)
        for k, a in enumerate(out.field(f)[:-1]):
            a2 = a.reshape(-1, a.shape[2]).astype(np.complex128)
            err = np.abs(a2.conj().T @ a2 - np.eye(a2.shape[1])).max()
            assert err < otol, (f, k, err)


def test_batched_encode_matches_single():
    torch = need_gpu()
    api = _api()
    imgs = np.stack([synth.blob_image(s) for s in (7, 8)])
    d = torch.from_numpy(imgs).float().cuda()
    say("batched encode")
    chi_dev = torch.tensor([16, 64], dtype=torch.int32, device="cuda")
    b = api.tt_encode_batched(d, 64, chi_dev=chi_dev)
    dense = api.tt_to_dense_batched(b).cpu().numpy()
    api.check_status()
    for f, chi in enumerate((16, 64)):
        ref = Z.to_dense(T.tt_svd(Q.to_quantics(imgs[f]), 12, chi, tau=1e-13), 6)
        assert rel(dense[f], ref) < (1e-4 if chi < 64 else 1e-5)


@pytest.mark.parametrize("chi", [64, 128])
def test_bench_configuration_full_size_vs_oracle(chi):
    """The benchmark's workload at its full size and in the launch
    configuration it times: the 1024^2 aperture field (seed 0) encoded at
    chi, the three distances 0.5 / 2 / 8 mm propagated as one batch (one
    batched zip-up + sweep per axis) with the library's own Fresnel MPOs
    (FresnelBatch, as the benchmark runs them) and decompressed, against the
    oracle's float64 TT-SVD, zip-up and sweep with the oracle's MPO (the
    sequential SVD of the dense operator), distance by distance: the FP32 bar
    against the identically truncated result (1e-4) and the same bond
    profile.  Both MPOs are left-canonical with equal bonds, i.e. equal up to
    unitary changes of bond basis, which leave every cut of the zip-up
    unchanged.  The oracle's MPO cores uploaded to the GPU give the same
    result (checked too)."""
    torch = need_gpu()
    api = _api()
    n = 10
    zs = (0.5e-3, 2e-3, 8e-3)
    e0 = synth.aperture_field(0, n=1 << n)
    d = torch.from_numpy(e0).to(torch.complex64).cuda()
    say("bench configuration: encode + batch of", len(zs), "chi", chi)
    psi = api.tt_encode(d, chi)
    m = 2 * n
    bi = api.MPSBatch(len(zs), m, chi)
    mid = api.MPSBatch(len(zs), m, chi)
    out = api.MPSBatch(len(zs), m, chi)
    bi.fill_from(psi)
    prop = api.FresnelBatch(n, LAM, DX, zs, device="cuda")
    prop(bi, chi, tmp=mid, out=out)
    own = api.tt_to_dense_batched(out).cpu().numpy()
    own_bonds = out.bonds.cpu().numpy()
    api.check_status()
    mpos = [_oracle_mpos(n, z) for z in zs]
    wxb = api.MPOBatch([w[0] for w in mpos])
    wyb = api.MPOBatch([w[1] for w in mpos])
    api.mpo_apply_batched(bi, wxb, chi, out=mid)
    api.mpo_apply_batched(mid, wyb, chi, out=out)
    dens = api.tt_to_dense_batched(out).cpu().numpy()
    api.check_status()
    cores = T.tt_svd(Q.to_quantics(e0), m, chi, tau=1e-13)
    assert [int(x) for x in psi.bonds.cpu()] == T.bonds(cores)
    for i, z in enumerate(zs):
        wx, wy, c1 = mpos[i]
        r1, _ = Z.mpo_apply(cores, wx, chi, tau=1e-13)
        r2, _ = Z.mpo_apply(r1, wy, chi, tau=1e-13)
        ref = Z.to_dense(r2, n)
        e_own, e_orc = rel(own[i], ref), rel(dens[i], ref)
        say("z = %g mm: library MPO %.3e, oracle MPO %.3e vs the oracle's identical truncation" % (
            z * 1e3, e_own, e_orc))
        assert e_own < 1e-4
        assert e_orc < 1e-4
        assert [int(x) for x in own_bonds[i]] == T.bonds(r2)
        assert [int(x) for x in out.bonds[i].cpu()] == T.bonds(r2)


def test_concurrent_streams_with_separate_workspaces_match_serial():
    """Library calls on two streams at once (an encode with its own workspace
    on a second stream while a batched propagation runs on the current one)
    give bit-identical results to the same calls issued serially."""
    torch = need_gpu()
    api = _api()
    n, chi = 7, 24
    zs = (20e-6, 50e-6, 80e-6)
    m = 2 * n
    fa = torch.from_numpy(synth.aperture_field(5, n=1 << n)).to(torch.complex64).cuda()
    fb = torch.from_numpy(synth.aperture_field(6, n=1 << n)).to(torch.complex64).cuda()
    prop = api.FresnelBatch(n, LAM, DX, zs, device="cuda")
    bi, mid, out = (api.MPSBatch(len(zs), m, chi) for _ in range(3))
    # serial references
    pa = api.tt_encode(fa, chi)
    bi.fill_from(pa)
    prop(bi, chi, tmp=mid, out=out)
    ref_a = api.tt_to_dense_batched(out).clone()
    rb = api.tt_encode(fb, chi)
    torch.cuda.synchronize()
    # concurrent: encode B on a side stream while A propagates
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    pa2 = api.tt_encode(fa, chi)
    bi.fill_from(pa2)
    side.wait_stream(main)
    with torch.cuda.stream(side):
        pb = api.tt_encode(fb, chi, ws_key="side")
    prop(bi, chi, tmp=mid, out=out)
    da = api.tt_to_dense_batched(out)
    main.wait_stream(side)
    torch.cuda.synchronize()
    api.check_status()
    api.check_status("side")
    assert torch.equal(da, ref_a)
    assert torch.equal(pb.cores, rb.cores) and torch.equal(pb.bonds, rb.bonds)


@pytest.mark.gpu
def test_steps_in_flight_on_four_streams_match_serial():
    """Whole steps (encode, batched propagation, decompression) of different
    fields issued on four streams at once (the current stream and three
    more), each with its own buffers and workspace keys, as the benchmark's
    concurrent schedule issues them: every result is bit-identical to the
    same step run alone, and every workspace's status word stays clean."""
    torch = need_gpu()
    api = _api()
    say("steps in flight on four streams")
    n, chi = 7, 24
    zs = (20e-6, 50e-6, 80e-6)
    m = 2 * n
    prop = api.FresnelBatch(n, LAM, DX, zs, device="cuda")
    fields = [torch.from_numpy(synth.aperture_field(20 + i, n=1 << n)).to(torch.complex64).cuda()
              for i in range(8)]
    main = torch.cuda.current_stream()

    class Lane:
        def __init__(self, i):
            self.s = main if i == 0 else torch.cuda.Stream()
            self.psi = api.MPS(m, chi)
            self.inp, self.mid, self.out = (api.MPSBatch(len(zs), m, chi) for _ in range(3))
            self.key = "inflight%d" % i
            self.res = []

        def step(self, f):
            api.tt_encode(f, chi, out=self.psi, ws_key=self.key)
            self.inp.fill_from(self.psi)
            prop(self.inp, chi, tmp=self.mid, out=self.out, ws_key=self.key)
            self.res.append(api.tt_to_dense_batched(self.out, ws_key=self.key + ".dense"))

    refs = []
    for f in fields:
        bi, mid, out = (api.MPSBatch(len(zs), m, chi) for _ in range(3))
        bi.fill_from(api.tt_encode(f, chi))
        prop(bi, chi, tmp=mid, out=out)
        refs.append(api.tt_to_dense_batched(out).clone())
    torch.cuda.synchronize()
    lanes = [Lane(i) for i in range(4)]
    for ln in lanes:
        ln.s.wait_stream(main)
    for k, f in enumerate(fields):
        ln = lanes[k % 4]
        with torch.cuda.stream(ln.s):
            ln.step(f)
    for ln in lanes:
        main.wait_stream(ln.s)
    torch.cuda.synchronize()
    api.check_status()
    for ln in lanes:
        api.check_status(ln.key)
        api.check_status(ln.key + ".dense")
    for k in range(len(fields)):
        assert torch.equal(lanes[k % 4].res[k // 4], refs[k]), k
