"""Pins of the oracle's perfect sampler (Sec. 5): the probability it assigns
to every outcome equals |E|^2 / ||E||^2 by brute-force enumeration; a point
mass is sampled exactly at its pixel (pins the bit-to-coordinate order); an
MPS of the same field that is not left-canonical gives wrong probabilities
(the sampler's precondition is load-bearing, so a missing orthogonalisation
would be caught); and drawn samples pass a chi-square test against |E|^2."""
import itertools

import numpy as np
from scipy import stats

from oracle import quantics as Q
from oracle import sampling as S
from oracle import ttsvd as T


def _field(seed, n):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))


def test_outcome_probabilities_equal_the_squared_field():
    n = 3
    e = _field(1, n)
    cores = T.tt_svd(Q.to_quantics(e), 2 * n, 64)
    dist = np.abs(e) ** 2 / np.sum(np.abs(e) ** 2)
    tot = 0.0
    for bits in itertools.product((0, 1), repeat=2 * n):
        a, b = S._coords(bits, n)
        p = S.sample_probability(cores, bits)
        assert abs(p - dist[a, b]) < 1e-12
        tot += p
    assert abs(tot - 1.0) < 1e-12


def test_point_mass_is_sampled_at_its_pixel():
    n = 4
    e = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    e[11, 6] = 2.0 - 1.0j
    cores = T.tt_svd(Q.to_quantics(e), 2 * n, 8)
    u = np.random.default_rng(2).random((50, 2 * n))
    rows, cols = S.perfect_samples(cores, u)
    assert np.all(rows == 11) and np.all(cols == 6)


def test_non_canonical_representation_is_caught():
    n = 3
    e = _field(3, n)
    cores = [c.copy() for c in T.tt_svd(Q.to_quantics(e), 2 * n, 64)]
    # the same state with a non-unitary change of basis on bond 2
    k = 2
    d = cores[k].shape[2]
    rng = np.random.default_rng(4)
    g = np.eye(d) + 0.5 * rng.standard_normal((d, d))
    cores[k] = np.einsum("rsc,cd->rsd", cores[k], g)
    cores[k + 1] = np.einsum("dc,csr->dsr", np.linalg.inv(g), cores[k + 1])
    assert np.abs(Q.from_quantics(T.tt_dense(cores), n) - e).max() < 1e-10
    dist = np.abs(e) ** 2 / np.sum(np.abs(e) ** 2)
    worst = 0.0
    for bits in itertools.product((0, 1), repeat=2 * n):
        a, b = S._coords(bits, n)
        worst = max(worst, abs(S.sample_probability(cores, bits) - dist[a, b]))
    assert worst > 1e-3


def test_samples_follow_the_squared_field_chi_square():
    n = 3
    e = _field(5, n)
    cores = T.tt_svd(Q.to_quantics(e), 2 * n, 64)
    u = np.random.default_rng(6).random((200000, 2 * n))
    rows, cols = S.perfect_samples(cores, u)
    counts = np.zeros((1 << n, 1 << n))
    np.add.at(counts, (rows, cols), 1)
    expect = np.abs(e) ** 2 / np.sum(np.abs(e) ** 2) * len(rows)
    chi2, p = stats.chisquare(counts.ravel(), expect.ravel())
    assert p > 1e-6, (chi2, p)
