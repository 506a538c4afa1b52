"""GPU parity of the never-densified low-rank encoder (tt_encode_low_rank):
a field given as a sum of R separable terms, E0 = sum_r u_r v_r^T, encoded
term by term, summed as MPS and TT-rounded, against the oracle's TT-SVD of
the dense sum (Sec. 4; TT-rounding of an exact representation is the TT-SVD
of the tensor it represents, pinned on the CPU in test_oracle_ttsvd.py).

Bars (FP32): lossless (chi at least the field's ranks) 1e-5 against the
dense sum; truncated 1e-4 against the oracle's TT-SVD at the same chi with
equal bonds.  Every term's 1-D factors must encode losslessly at the term
cap for the comparison to be the identical algorithm; the test checks that
on the oracle first.  At 16384^2 (28 sites) the encode is checked at 1e5
sampled pixels and on a 2048^2 window against the sum of outer products.
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import quantics as Q
from oracle import ttsvd as T
import synth

pytestmark = pytest.mark.gpu


def _api():
    from paper_2510_23089_amd import api
    return api


def _c1(term_cap):
    c = 1
    while (c + 1) * (c + 1) <= term_cap:
        c += 1
    return c


@pytest.mark.parametrize("n,rank,term_cap,chi", [(4, 3, 64, 64), (6, 3, 64, 64), (6, 3, 64, 8), (8, 2, 128, 24),
                                                 (8, 4, 64, 128)])
def test_low_rank_encode_vs_oracle(n, rank, term_cap, chi):
    torch = need_gpu()
    api = _api()
    u, v = synth.beam_sum_1d(100 + n + rank, 1 << n, rank)
    c1 = _c1(term_cap)
    for x in list(u) + list(v):
        b = T.bonds(T.tt_svd(x, n, 1 << n, tau=1e-13))
        assert max(b) <= c1, (b, c1)          # each term's factors encode losslessly at the cap
    dense = np.einsum("ra,rb->ab", u, v)
    ref = T.tt_svd(Q.to_quantics(dense), 2 * n, chi, tau=1e-13)
    psi = api.tt_encode_low_rank(torch.from_numpy(u).to(torch.complex64).cuda(),
                                 torch.from_numpy(v).to(torch.complex64).cuda(), chi, term_cap=term_cap,
                                 chi_cap=256, tau=1e-13, ws_key="low_rank_test")
    api.check_status(key="low_rank_test")
    got = api.tt_to_dense(psi).cpu().numpy()
    bonds = [int(x) for x in psi.bonds.cpu()]
    e_ref = rel(got, Q.from_quantics(T.tt_dense(ref), n))
    e_dense = rel(got, dense)
    say("2^%d, rank %d, chi %d: vs TT-SVD %.2e, vs dense %.2e, bonds %s / %s"
        % (n, rank, chi, e_ref, e_dense, max(bonds), max(T.bonds(ref))))
    assert bonds == T.bonds(ref)
    assert e_ref < 1e-4
    if max(T.bonds(ref)) < chi:
        assert e_dense < 1e-5


def test_low_rank_encode_16384_never_densified():
    torch = need_gpu()
    api = _api()
    n, rank, term_cap, chi = 14, 3, 64, 192
    u, v = synth.beam_sum_1d(7, 1 << n, rank)
    psi = api.tt_encode_low_rank(torch.from_numpy(u).to(torch.complex64).cuda(),
                                 torch.from_numpy(v).to(torch.complex64).cuda(), chi, term_cap=term_cap,
                                 chi_cap=192, tau=1e-13, ws_key="low_rank_test")
    api.check_status(key="low_rank_test")
    say("bonds", max(int(x) for x in psi.bonds.cpu()))
    rng = np.random.default_rng(3)
    rows = rng.integers(0, 1 << n, 100000)
    cols = rng.integers(0, 1 << n, 100000)
    vals = api.tt_eval_points(psi, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()).cpu().numpy()
    api.check_status(key="points")
    ref = np.einsum("rp,rp->p", u[:, rows], v[:, cols])
    lo = (1 << n) // 2 - 1024
    win = api.tt_to_dense_window(psi, lo, lo, 2048, 2048).cpu().numpy()
    api.check_status(key="window")
    wref = u[:, lo:lo + 2048].T @ v[:, lo:lo + 2048]
    e_pts, e_win = rel(vals, ref), rel(win, wref)
    say("16384^2 rank 3: sampled %.2e, window %.2e" % (e_pts, e_win))
    assert e_pts < 1e-5
    assert e_win < 1e-5
