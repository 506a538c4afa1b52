"""Fields too large to densify: separable encode, point evaluation and block
decompression, and the 16384^2 Gaussian-beam x grating propagation at chi
256 checked on sampled pixels and on the central 4096^2 window against the
exact separable solution (1-D float64 FFTs of length 16384 in the oracle,
plus the Gaussian-beam closed form for the grating-free factor).
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import fresnel as F
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

pytestmark = pytest.mark.gpu
LAM, DX = 500e-9, 1e-6


def _api():
    from paper_2510_23089_amd import api
    return api


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_separable_encode_small(prec):
    torch = need_gpu()
    api = _api()
    rng = np.random.default_rng(4)
    n = 6
    u = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    v = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    psi = api.tt_encode_separable(torch.from_numpy(u).to(dt).cuda(), torch.from_numpy(v).to(dt).cuda(), 64,
                                  prec=prec)
    api.check_status(key="separable")
    got = api.tt_to_dense(psi).cpu().numpy()
    assert rel(got, np.outer(u, v)) < (1e-5 if prec == "fp32" else 1e-12)
    b = psi.host_bonds()
    assert max(b) <= 64 and b[0] == 1 and b[-1] == 1


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_eval_points_and_blocks_vs_dense(prec):
    torch = need_gpu()
    api = _api()
    n = 5
    e0 = synth.random_field(3, 1 << n)         # nonzero everywhere: every block has a reference
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, 16, tau=1e-13)
    ref = Z.to_dense(cores, n)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    psi = api.MPS.from_host(cores, chi_cap=16, dtype=dt)
    rng = np.random.default_rng(0)
    rows = rng.integers(0, 1 << n, 500)
    cols = rng.integers(0, 1 << n, 500)
    rows[:4] = [0, 0, 31, 31]
    cols[:4] = [0, 31, 0, 31]
    vals = api.tt_eval_points(psi, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()).cpu().numpy()
    api.check_status(key="points")
    tol = 1e-5 if prec == "fp32" else 1e-12
    assert rel(vals, ref[rows, cols]) < tol
    for j in (1, 3, 5):
        side = 1 << j
        for br in range((1 << n) // side):
            for bc in range((1 << n) // side):
                blk = api.tt_to_dense_block(psi, j, br, bc).cpu().numpy()
                assert rel(blk, ref[br * side:(br + 1) * side, bc * side:(bc + 1) * side]) < tol, (j, br, bc)
    win = api.tt_to_dense_window(psi, 5, 9, 19, 13, log2_block=3).cpu().numpy()
    assert rel(win, ref[5:24, 9:22]) < tol
    api.check_status(key="block")


def _exact_factor(vec, z):
    return F.fresnel_1d(vec, LAM, DX, z)


# z_j = 0.1 * 100^(j/7) mm, j = 0..7: eight log-spaced distances 0.1 .. 10 mm
ZS_C4 = tuple(0.1e-3 * 100.0 ** (j / 7.0) for j in range(8))
# distances whose zip-up at chi_zip = 256 is lossless (measured: the result
# equals the exact separable propagation to FP32 rounding); beyond them the
# zip-up state left of the centre needs more than 256 directions (the Gram
# matrices of the eigensolver stop at 512 = 2 chi_zip), so the zip-up's own
# truncation shows and the comparison with the exact field measures that
# truncation, not parity (those distances are parity unpinned: an oracle
# zip-up at 28 sites, chi 256 and operator bond up to 88 is out of reach)
C4_LOSSLESS_MAX = 1.5e-3


def test_large_separable_propagation_16384():
    """16384^2 field (28 sites), chi 256, all eight log-spaced distances
    (0.1 .. 10 mm) as one batch, checked on 1e5 sampled pixels and on the
    central 4096^2 window against the exact separable solution (1-D FFTs of
    the factors; the grating-free factor also against the Gaussian-beam
    closed form): FP32 bar 2e-5 where the zip-up is lossless; elsewhere the
    error against the exact field is reported with a loose sanity bound."""
    torch = need_gpu()
    api = _api()
    n, chi = 14, 256
    zs = ZS_C4
    ua, vb = synth.grating_beam_1d(1 << n)
    say("encode")
    psi = api.tt_encode_separable(torch.from_numpy(ua).to(torch.complex64).cuda(),
                                  torch.from_numpy(vb).to(torch.complex64).cuda(), chi)
    api.check_status(key="separable")
    say("bonds", max(psi.host_bonds()))
    batch = api.MPSBatch(len(zs), 2 * n, chi)
    batch.fill_from(psi)
    say("mpo")
    prop = api.FresnelBatch(n, LAM, DX, zs)
    say("propagate")
    out = prop(batch, chi)
    api.check_status()
    rng = np.random.default_rng(7)
    npts = 100000
    rows = rng.integers(0, 1 << n, npts)
    cols = rng.integers(0, 1 << n, npts)
    for f, z in enumerate(zs):
        ex_a = _exact_factor(ua, z)
        ex_b = _exact_factor(vb, z)
        g_cf = F.gaussian_beam_exact_1d(1 << n, 2000.0, LAM, DX, z, (1 << n) / 2)
        assert rel(ex_b, g_cf) < 1e-8
        one = api.MPS.wrap(out.cores[f], out.bonds[f])
        vals = api.tt_eval_points(one, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()).cpu().numpy()
        api.check_status(key="points")
        ref = ex_a[rows] * ex_b[cols]
        e_pts = rel(vals, ref)
        lo = (1 << n) // 2 - 2048
        win = api.tt_to_dense_window(one, lo, lo, 4096, 4096).cpu().numpy()
        api.check_status(key="window")
        e_win = rel(win, np.outer(ex_a[lo:lo + 4096], ex_b[lo:lo + 4096]))
        say("z=%.3f mm: sampled rel err %.3e, window rel err %.3e, max bond %d" %
            (z * 1e3, e_pts, e_win, max(int(x) for x in out.bonds[f].cpu())))
        if z <= C4_LOSSLESS_MAX:
            assert e_pts < 2e-5
            assert e_win < 2e-5
        else:
            assert e_pts < 1e-2
            assert e_win < 1e-2
