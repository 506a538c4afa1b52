"""Pins for the oracle's quantics map (Sec. 3) and TT-SVD (Sec. 4, App. A).

Each check compares the oracle with something other than itself: brute-force
bit manipulation written differently, closed-form parameter counts, the
Eckart-Young / Oseledets error bounds computed from independent SVDs of the
unfoldings, and exact reconstruction at full rank.
"""
import os

import numpy as np
import pytest

from oracle import quantics as Q
from oracle import ttsvd as T
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _interleave_string(a, b, n):
    sa = format(a, "0%db" % n)
    sb = format(b, "0%db" % n)
    return "".join(x + y for x, y in zip(sa, sb))


def test_quantics_bruteforce_8x8():
    n = 3
    img = np.arange(64, dtype=np.float64).reshape(8, 8) * (1 + 0.5j)
    v = Q.to_quantics(img)
    for a in range(8):
        for b in range(8):
            idx = int(_interleave_string(a, b, n), 2)     # string-based bit interleave
            assert v[idx] == img[a, b]
            assert Q.quantics_flat_index(a, b, n) == idx
    assert np.array_equal(Q.from_quantics(v, n), img)


def test_quantics_roundtrip_random():
    img = synth.random_field(3, 32)
    assert np.array_equal(Q.from_quantics(Q.to_quantics(img), 5), img)


def test_quantics_worked_example_golden():
    vals = {}
    with open(os.path.join(GOLD, "quantics_worked_example.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = v
    a, b, side = int(vals["a"]), int(vals["b"]), int(vals["side"])
    n = side.bit_length() - 1
    assert _interleave_string(a, b, n) == vals["interleaved"]
    assert format(a, "07b") + format(b, "07b") == vals["concatenated"]
    assert Q.quantics_flat_index(a, b, n) == int(vals["flat_index"])
    assert int(vals["interleaved"], 2) == int(vals["flat_index"])
    # the printed string matches neither reading (documented as garbled)
    assert vals["paper_printed"] not in (vals["interleaved"], vals["concatenated"])
    img = np.zeros((side, side))
    img[a, b] = 1.0
    v = Q.to_quantics(img)
    assert int(np.argmax(v)) == int(vals["flat_index"])


def test_keep_rule_hand_values():
    lam = np.array([8.0, 4.0, 2.0, 1.0, 1e-30])
    assert T.keep_count(lam, chi=10) == 4                     # tau removes the zero
    assert T.keep_count(lam, chi=2) == 2
    # eps: tails after k=1,2,3,4: 7, 3, 1, 1e-30 ; total 15
    assert T.keep_count(lam, chi=10, eps=3.0 / 15.0) == 2
    assert T.keep_count(lam, chi=10, eps=0.99 / 15.0) == 4
    assert T.keep_count(np.zeros(4), chi=5) == 1              # zero field keeps one


@pytest.mark.parametrize("m", [4, 6, 8, 10, 12])
def test_ttsvd_exact_and_parameter_count(m):
    rng = np.random.default_rng(m)
    v = rng.standard_normal(1 << m) + 1j * rng.standard_normal(1 << m)
    cores = T.tt_svd(v, m, chi=1 << m)
    err = np.linalg.norm(T.tt_dense(cores) - v) / np.linalg.norm(v)
    assert err < 1e-13
    # random MPS of m sites saturates r_k = min(2^k, 2^(m-k)); the total
    # parameter count is (8/3)(2^m - 1) for even m (Sec. 4, D_max = 8/3 2^n)
    assert T.param_count(cores) * 3 == 8 * ((1 << m) - 1)
    # left-orthonormal cores
    for c in cores[:-1]:
        mat = c.reshape(-1, c.shape[2])
        assert np.allclose(mat.conj().T @ mat, np.eye(c.shape[2]), atol=1e-12)


def _unfolding_tails(v, m, chi):
    tails = []
    for k in range(1, m):
        s = np.linalg.svd(v.reshape(1 << k, -1), compute_uv=False)
        tails.append(float(np.sum(s[chi:] ** 2)))
    return tails


@pytest.mark.parametrize("chi", [1, 2, 4, 8])
def test_ttsvd_error_bounds(chi):
    """Oseledets: max_k tail_k <= ||v - TT_chi(v)||^2 <= sum_k tail_k, with
    tail_k the discarded weight of the exact k-th unfolding."""
    m = 10
    img = synth.blob_image(7, n=32)
    v = Q.to_quantics(img).astype(np.complex128)
    cores = T.tt_svd(v, m, chi=chi)
    err2 = np.linalg.norm(T.tt_dense(cores) - v) ** 2
    tails = _unfolding_tails(v, m, chi)
    assert err2 <= sum(tails) * (1 + 1e-9) + 1e-20
    assert err2 >= max(tails) * (1 - 1e-9)


def test_ttsvd_eckart_young_single_cut():
    """m = 2: TT-SVD is the truncated SVD of a 2x2 matrix."""
    rng = np.random.default_rng(5)
    v = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    s = np.linalg.svd(v.reshape(2, 2), compute_uv=False)
    cores = T.tt_svd(v, 2, chi=1)
    err = np.linalg.norm(T.tt_dense(cores) - v)
    assert abs(err - s[1]) < 1e-13


def test_ttsvd_rank_one_product():
    rng = np.random.default_rng(11)
    m = 12
    factors = [rng.standard_normal(2) + 1j * rng.standard_normal(2) for _ in range(m)]
    v = factors[0]
    for f in factors[1:]:
        v = np.kron(v, f)
    cores = T.tt_svd(v, m, chi=64)
    assert T.bonds(cores) == [1] * (m + 1)
    assert np.linalg.norm(T.tt_dense(cores) - v) < 1e-12 * np.linalg.norm(v)


def test_ttsvd_blob_image_converges():
    """The 64x64 blob image is exact at full rank (max bond 2^6 = 64)."""
    img = synth.blob_image(0)
    v = Q.to_quantics(img)
    errs = []
    for chi in (8, 16, 32, 64):
        c = T.tt_svd(v, 12, chi)
        errs.append(np.linalg.norm(T.tt_dense(c) - v) / np.linalg.norm(v))
    assert errs[-1] < 1e-13
    assert errs[0] > errs[1] > errs[2] > errs[3]
