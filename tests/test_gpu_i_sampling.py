"""GPU parity of perfect photon sampling (tt_sample, Sec. 5) against the
oracle's sampler: the same left-canonical cores (uploaded) and the same
uniforms give the same pixels wherever the oracle's decisions are not within
rounding of a tie (FP64: every sample with margin > 1e-9; FP32: margin
> 1e-4, at least 99 % of the samples); at the benchmark's size the samples
of a propagated 1024^2 field follow |E|^2 (chi-square on a 16 x 16 binning).
"""
import numpy as np
import pytest
from scipy import stats

from gpu_util import need_gpu, say
from oracle import quantics as Q
from oracle import sampling as S
from oracle import ttsvd as T
import synth

pytestmark = pytest.mark.gpu


def _api():
    from paper_2510_23089_amd import api
    return api


@pytest.mark.parametrize("prec,margin", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_samples_equal_the_oracle_sampler(prec, margin):
    torch = need_gpu()
    api = _api()
    n, chi, count = 6, 24, 8192
    e = synth.aperture_field(11, n=1 << n)
    cores = T.tt_svd(Q.to_quantics(e), 2 * n, chi, tau=1e-13)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    psi = api.MPS.from_host(cores, chi_cap=chi, dtype=dt)
    u = np.random.default_rng(12).random((count, 2 * n))
    rows, cols = api.tt_sample(psi, uniforms=torch.from_numpy(u).cuda(), ws_key="sample_test")
    api.check_status(key="sample_test")
    r_ref, c_ref = S.perfect_samples(cores, u)
    ok = S.decision_margins(cores, u) > margin
    got_r, got_c = rows.cpu().numpy(), cols.cpu().numpy()
    same = (got_r == r_ref) & (got_c == c_ref)
    say("%s: %d of %d samples beyond the margin, %d of them equal; %d equal overall"
        % (prec, ok.sum(), count, (same & ok).sum(), same.sum()))
    assert ok.mean() > 0.99
    assert np.all(same[ok])


def test_propagated_field_samples_follow_the_intensity():
    torch = need_gpu()
    api = _api()
    n, chi, count, z = 10, 128, 1 << 20, 2e-3
    e0 = synth.aperture_field(0, n=1 << n)
    psi = api.tt_encode(torch.from_numpy(e0).to(torch.complex64).cuda(), chi)
    prop = api.FresnelPropagator(n, 500e-9, 1e-6, z)
    out = prop(psi, chi)
    dense = api.tt_to_dense(out).cpu().numpy().astype(np.complex128)
    api.check_status()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    rows, cols = api.tt_sample(out, count=count, seed=3, ws_key="sample_test")
    ev1.record()
    torch.cuda.synchronize()
    api.check_status(key="sample_test")
    ms = ev0.elapsed_time(ev1)
    r, c = rows.cpu().numpy(), cols.cpu().numpy()
    bins = 16
    counts = np.zeros((bins, bins))
    np.add.at(counts, (r * bins >> n, c * bins >> n), 1)
    inten = np.abs(dense) ** 2
    expect = inten.reshape(bins, (1 << n) // bins, bins, (1 << n) // bins).sum(axis=(1, 3))
    expect = expect / expect.sum() * count
    keep = expect > 5
    chi2, p = stats.chisquare(counts[keep], expect[keep] * counts[keep].sum() / expect[keep].sum())
    say("1024^2 field, 2^20 samples in %.1f ms (%.2e samples/s); chi-square p %.3g over %d bins"
        % (ms, count / (ms * 1e-3), p, keep.sum()))
    assert p > 1e-6
