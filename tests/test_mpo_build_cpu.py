"""CPU pins of the library's host-side Fresnel MPO builder (mpo_build).

The builder (QFT circuit -> diagonal -> QFT^H, then left-canonical rounding)
is product code; here it is checked against the oracle's dense operator
F^-1 diag(T) F (Sec. 6.1) and against the oracle's brute-force MPO (sequential
SVD of the dense operator, Sec. 6.1): same operator, left-orthonormal cores,
the same bond profile and the same Schmidt values at every bond.  Equal bonds
and left-orthonormal cores make the two MPOs differ only by unitary changes of
bond basis, under which the truncating zip-up's Gram matrices are invariant.
"""
import numpy as np
import pytest

from oracle import fresnel as F
from oracle import mpo as OM
from paper_2510_23089_amd import mpo_build as B

LAM, DX = 500e-9, 1e-6


def _bonds(cores):
    return [1] + [int(c.shape[3]) for c in cores]


def _apply_vec(cores, v):
    """(W v) for a 1-D MPO of n sites, contracted site by site (no densify):
    state[o, w, r] holds the output bits done so far (o), the open operator
    bond (w) and the input bits not yet consumed (r, most significant first)."""
    state = np.asarray(v, dtype=np.complex128).reshape(1, 1, -1)
    for w in cores:
        o, d, r = state.shape
        st = state.reshape(o, d, 2, r // 2)                       # split off the next input bit s
        nxt = np.einsum("odsr,dtse->oter", st, w)                 # [o, t, e, r']
        state = nxt.reshape(o * 2, w.shape[3], r // 2)
    return state.reshape(-1)


def _schmidt_values(cores):
    """Singular values at every inner bond of a left-canonical MPO.  With the
    cores left of a cut an isometry they are the singular values of the right
    part as a D_k x (rest) matrix; an LQ sweep from the right end makes every
    right part an isometry times a small D x D factor L, whose singular values
    (taken directly, not through a squared Gram matrix) are the bond's."""
    n = len(cores)
    lmat = np.ones((1, 1), dtype=np.complex128)
    out = [None] * (n - 1)
    for k in range(n - 1, 0, -1):
        w = np.tensordot(cores[k], lmat, axes=(3, 0))            # [D_(k-1), t, s, D']
        q, r = np.linalg.qr(w.reshape(w.shape[0], -1).conj().T)
        lmat = r.conj().T                                          # D_(k-1) x D'
        out[k - 1] = np.linalg.svd(lmat, compute_uv=False)
    return out


@pytest.mark.parametrize("n,z", [(2, 1e-4), (3, 2e-4), (4, 1e-3), (5, 2e-3), (6, 1e-3), (6, 8e-3)])
def test_dense_equals_fft_operator(n, z):
    w = B.fresnel_axis(n, LAM, DX, z)
    ref = F.fresnel_matrix_1d(1 << n, LAM, DX, z)
    assert np.abs(B.dense(w) - ref).max() < 1e-12


@pytest.mark.parametrize("z", [0.5e-3, 2e-3, 8e-3])
def test_n10_applied_to_random_vectors_equals_fft(z):
    n = 10
    w = B.fresnel_axis(n, LAM, DX, z)
    rng = np.random.default_rng(7)
    for _ in range(3):
        v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        got = _apply_vec(w, v)
        ref = F.fresnel_1d(v, LAM, DX, z)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11


@pytest.mark.parametrize("n,z", [(6, 1e-3), (10, 0.5e-3), (10, 2e-3), (10, 8e-3)])
def test_left_canonical_with_the_oracle_bonds_and_schmidt_values(n, z):
    w = B.fresnel_axis(n, LAM, DX, z)
    for k, c in enumerate(w[:-1]):
        q = c.reshape(-1, c.shape[3])
        assert np.abs(q.conj().T @ q - np.eye(q.shape[1])).max() < 1e-12, k
    # the operator is unitary: its squared Frobenius norm N sits in the last core
    assert abs(np.linalg.norm(w[-1]) ** 2 - (1 << n)) < 1e-9 * (1 << n)
    o = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    assert _bonds(w) == _bonds(o)
    for k, (a, b) in enumerate(zip(_schmidt_values(w), _schmidt_values(o))):
        assert a.shape == b.shape
        assert np.abs(a - b).max() < 1e-12 * b[0], k


def test_round_left_keeps_an_exact_operator_and_cuts_a_planted_redundancy():
    """A redundant representation (the product of the QFT MPO with its
    inverse, bond 49) rounds to the identity with bond 1; a generic operator
    of known rank profile keeps its bonds."""
    n = 5
    q = B.qft_br(n)
    eye = B.round_left(B.mul(B.dagger(q), q))
    assert _bonds(eye) == [1] * (n + 1)
    assert np.abs(B.dense(eye) - np.eye(1 << n)).max() < 1e-12
    rng = np.random.default_rng(3)
    cores = [rng.standard_normal((1 if k == 0 else 3, 2, 2, 1 if k == n - 1 else 3))
             + 1j * rng.standard_normal((1 if k == 0 else 3, 2, 2, 1 if k == n - 1 else 3)) for k in range(n)]
    r = B.round_left(cores)
    assert np.abs(B.dense(r) - B.dense(cores)).max() < 1e-12 * np.abs(B.dense(cores)).max()
    assert _bonds(r) == [1, 3, 3, 3, 3, 1]
