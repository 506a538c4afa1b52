"""Pins for the dense Fresnel oracle (Sec. 6.1) and the oracle's MPOs
(Sec. 5 Hadamard / QFT, Sec. 6.1 brute-force MPO construction).

Independent references: explicit O(N^4) DFT sums, unitarity and the
propagation semigroup, the Gaussian-beam closed form, a Sylvester-built
Hadamard matrix, and the bond ranks the paper states (Hadamard rank 1, QFT
finite rank, natural-order DFT full rank).
"""
import numpy as np
import pytest

from oracle import fresnel as F
from oracle import mpo as M
import synth

LAM, DX = 500e-9, 1e-6


def _bruteforce_propagate(e0, lam, dx, z):
    """Explicit DFT sums: E_z[a,b] = 1/N^2 sum_k H(k) sum_j E0[j] e^{2 pi i k (a-j)/N}."""
    n = e0.shape[0]
    out = np.zeros_like(e0, dtype=np.complex128)
    f = np.array([(k if k < n // 2 else k - n) / (n * dx) for k in range(n)])
    h1 = np.exp(-1j * np.pi * lam * z * f * f)
    for a in range(n):
        for b in range(n):
            acc = 0.0
            for ka in range(n):
                for kb in range(n):
                    s = 0.0
                    for ja in range(n):
                        for jb in range(n):
                            s += e0[ja, jb] * np.exp(2j * np.pi * (ka * (a - ja) + kb * (b - jb)) / n)
                    acc += h1[ka] * h1[kb] * s
            out[a, b] = acc / (n * n)
    return out


def test_fresnel_bruteforce_4x4():
    e0 = synth.random_field(1, 4)
    z = 3e-6                                  # large phase spread on a 4-px grid
    assert np.allclose(F.fresnel_dense(e0, LAM, DX, z),
                       _bruteforce_propagate(e0, LAM, DX, z), atol=1e-12)


def test_fresnel_invariants():
    e0 = synth.aperture_field(2, n=128)
    n0 = np.linalg.norm(e0)
    e1 = F.fresnel_dense(e0, LAM, DX, 1e-3)
    assert abs(np.linalg.norm(e1) - n0) < 1e-12 * n0                  # unitary (Parseval)
    assert np.allclose(F.fresnel_dense(e0, LAM, DX, 0.0), e0, atol=1e-13)
    e12 = F.fresnel_dense(F.fresnel_dense(e0, LAM, DX, 0.7e-3), LAM, DX, 0.3e-3)
    assert np.allclose(e12, e1, atol=1e-11 * n0)                      # semigroup
    # separability: rows then columns with the 1-D propagator
    u = F.fresnel_matrix_1d(128, LAM, DX, 1e-3)
    assert np.allclose(u @ e0 @ u.T, e1, atol=1e-11 * n0)
    # backward propagation inverts
    assert np.allclose(F.fresnel_dense(e1, LAM, DX, -1e-3), e0, atol=1e-11 * n0)


@pytest.mark.parametrize("n_side,w0,z,tol", [
    (4096, 300.0, 2e-3, 1e-12),
    (1024, 100.0, 8e-3, 1e-10),
    (256, 20.0, 0.5e-3, 1e-10),
])
def test_gaussian_beam_closed_form(n_side, w0, z, tol):
    c = n_side / 2
    e0 = synth.gaussian_beam(n_side, w0, c, c)
    num = F.fresnel_dense(e0, LAM, DX, z)
    ref = F.gaussian_beam_exact(n_side, w0, LAM, DX, z, c, c)
    assert np.max(np.abs(num - ref)) < tol


def test_bit_reversed_dft_bruteforce():
    n = 4
    nn = 1 << n
    qft = M.qft_br_matrix(n)
    for i in range(nn):
        k = int(format(i, "0%db" % n)[::-1], 2)               # bit-reversed row
        for j in range(nn):
            ref = np.exp(-2j * np.pi * j * k / nn) / np.sqrt(nn)
            assert abs(qft[i, j] - ref) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_qft_mpo_matches_dense(n):
    mat = M.qft_br_matrix(n)
    cores = M.mpo_from_matrix(mat, n, rel_err=1e-13)
    dense = M.mpo_dense(cores)
    assert np.max(np.abs(dense - mat)) < 1e-12
    assert np.allclose(dense.conj().T @ dense, np.eye(1 << n), atol=1e-12)


def test_qft_rank_finite_dft_full():
    """Bit-reversed DFT has small MPO rank, the natural-order DFT does not."""
    n = 8
    nat = M.mpo_from_matrix(np.fft.fft(np.eye(1 << n), axis=0, norm="ortho"), n, rel_err=1e-12)
    nat_bonds = [c.shape[3] for c in nat[:-1]]
    assert nat_bonds == [4 ** min(k + 1, n - k - 1) for k in range(n - 1)]
    # bit-reversed: the rank saturates as n grows (finite-rank QFT, Sec. 5)
    r8 = max(c.shape[3] for c in M.mpo_from_matrix(M.qft_br_matrix(8), 8, rel_err=1e-12))
    r10 = max(c.shape[3] for c in M.mpo_from_matrix(M.qft_br_matrix(10), 10, rel_err=1e-12))
    assert r8 <= 12 and r10 <= 12
    r10_loose = max(c.shape[3] for c in M.mpo_from_matrix(M.qft_br_matrix(10), 10, rel_err=1e-6))
    assert r10_loose <= 8


def _sylvester(n):
    h = np.array([[1.0]])
    for _ in range(n):
        h = np.block([[h, h], [h, -h]])
    return h / np.sqrt(1 << n)


def test_hadamard_mpo_rank_one():
    n = 6
    dense = M.mpo_dense(M.hadamard_mpo(n))
    assert np.allclose(dense, _sylvester(n), atol=1e-14)
    cores = M.mpo_from_matrix(_sylvester(n), n)
    assert all(c.shape[3] == 1 for c in cores)


@pytest.mark.parametrize("n,z", [(4, 1e-3), (6, 1e-3), (6, 5e-5), (8, 2e-3)])
def test_fresnel_mpo_dense(n, z):
    u = F.fresnel_matrix_1d(1 << n, LAM, DX, z)
    cores = M.mpo_from_matrix(u, n)
    dense = M.mpo_dense(cores)
    assert np.linalg.norm(dense - u) <= 1e-12 * np.linalg.norm(u) * 1.01
    assert np.allclose(dense.conj().T @ dense, np.eye(1 << n), atol=1e-11)


def test_fresnel_mpo_from_three_stage_product():
    """Real-space propagator = QFT_br^H diag_br(T) QFT_br (Sec. 6.1, Fig. of
    the MPO product), checked on dense matrices against the FFT form."""
    n = 6
    nn = 1 << n
    t = F.transfer_1d(nn, LAM, DX, 1e-3)
    qft = M.qft_br_matrix(n)
    d = np.diag(t[M.bit_reverse_perm(n)])
    assert np.allclose(qft.conj().T @ d @ qft, F.fresnel_matrix_1d(nn, LAM, DX, 1e-3), atol=1e-12)


def test_axis_embedding_is_kronecker():
    n = 3
    u = F.fresnel_matrix_1d(8, LAM, DX, 2e-6)
    c = M.mpo_from_matrix(u, n)
    wx = M.embed_axis(c, "x")
    wy = M.embed_axis(c, "y")
    e0 = synth.random_field(4, 8)
    from oracle import quantics as Q
    v = Q.to_quantics(e0)
    ux = M.mpo_dense(wx)
    uy = M.mpo_dense(wy)
    assert np.allclose(Q.from_quantics(ux @ v, n), u @ e0, atol=1e-12)
    assert np.allclose(Q.from_quantics(uy @ v, n), e0 @ u.T, atol=1e-12)


@pytest.mark.parametrize("n_side,w0,z", [(4096, 300.0, 2e-3), (16384, 2000.0, 10e-3), (1024, 60.0, 8e-3)])
def test_gaussian_beam_closed_form_1d(n_side, w0, z):
    """1-D factor: the FFT propagation of exp(-(u - c)^2 / w0^2) against the
    q^-1/2 closed form, and the 2-D closed form is the product of two."""
    c = n_side / 2
    u = np.arange(n_side) - c
    g = np.exp(-(u * u) / (w0 * w0)).astype(np.complex128)
    got = F.fresnel_1d(g, LAM, DX, z)
    ref = F.gaussian_beam_exact_1d(n_side, w0, LAM, DX, z, c)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9
    if n_side <= 1024:
        two = F.gaussian_beam_exact(n_side, w0, LAM, DX, z, c, c)
        assert np.allclose(np.outer(ref, ref), two, rtol=0, atol=1e-13)


def test_diag_mpo_from_vector_equals_the_brute_force_construction():
    """The diagonal shortcut gives the same operator, bonds and Schmidt
    values as the interleaved sequential SVD of the dense diagonal matrix."""
    from oracle import mpo as OM
    rng = np.random.default_rng(5)
    n = 5
    v = np.exp(1j * np.cumsum(rng.standard_normal(1 << n)) * 0.2)
    a = OM.diag_mpo_from_vector(v, n)
    b = OM.mpo_from_matrix(np.diag(v), n)
    assert np.abs(OM.mpo_dense(a) - np.diag(v)).max() < 1e-12
    assert [c.shape[3] for c in a] == [c.shape[3] for c in b]
