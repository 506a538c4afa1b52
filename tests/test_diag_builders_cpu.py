"""CPU pins of the host routes to diagonal operators and of the three-stage
factorisation of the propagator (Sec. 6.1 and 6.2).

* The library's fast Walsh-Hadamard transform equals the oracle's trace
  formula for the Pauli-Z coefficients; the oracle's closed form for the
  lattice dispersion (App. B) equals the trace formula.
* The parabolic phase on the two's-complement frequency register is a
  quadratic form in the bits, so its strings stop at two Z's (the transfer
  function is a product of one- and two-bit phase gates).
* Every route (sequential SVD of the diagonal, Pauli gate product, Bessel
  closed form for the lattice dispersion) gives the dense diagonal, and the
  three factors QFT^H . diag . QFT give the dense propagator F^-1 diag(T) F.
* The Bessel form at p_max = 14, t = 1 reproduces the unitary to below 1e-10
  for n = 4 .. 10 (the paper's statement for its Fig. of the MPO error), and
  its error never exceeds the tail sum of |J_p(t)| over |p| > p_max.
"""
import numpy as np
import pytest
from scipy.special import jv

from oracle import fresnel as F
from oracle import imaging as I
from paper_2510_23089_amd import mpo_build as B

LAM, DX = 500e-9, 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_walsh_hadamard_equals_trace_formula(n):
    rng = np.random.default_rng(n)
    phi = rng.standard_normal(1 << n)
    assert np.abs(B.walsh_hadamard(phi) - I.pauli_coefficients(phi)).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_cos_closed_form_equals_trace_formula(n):
    x = np.arange(1 << n) / (1 << n)
    assert np.abs(I.pauli_coefficients_cos(n) - I.pauli_coefficients(np.cos(2 * np.pi * x))).max() < 1e-14


@pytest.mark.parametrize("n,z", [(4, 1e-4), (6, 1e-3), (7, 2e-3)])
def test_parabolic_phase_has_at_most_two_body_strings(n, z):
    phi = B.fresnel_phase_br(n, LAM, DX, z)
    c = I.pauli_coefficients(phi)
    order = np.array([bin(m).count("1") for m in range(1 << n)])
    assert np.abs(c[order > 2]).max() < 1e-12 * np.abs(c).max()
    assert np.abs(c[order == 2]).max() > 1e-6 * np.abs(c).max()


@pytest.mark.parametrize("n", [3, 5, 6])
def test_pauli_route_gives_the_dense_diagonal(n):
    rng = np.random.default_rng(40 + n)
    phi = np.cumsum(rng.standard_normal(1 << n)) * 0.3
    d = B.dense(B.diag_pauli(phi))
    assert np.abs(d - np.diag(np.exp(-1j * phi))).max() < 1e-12


@pytest.mark.parametrize("route", ["svd", "pauli"])
@pytest.mark.parametrize("n,z", [(3, 3e-5), (5, 1e-4), (6, 1e-3), (6, 4e-3)])
def test_three_factors_give_the_dense_propagator(route, n, z):
    q, d, iq = B.fresnel_three_stage(n, LAM, DX, z, route)
    u = B.dense(iq) @ B.dense(d) @ B.dense(q)
    assert np.abs(u - F.fresnel_matrix_1d(1 << n, LAM, DX, z)).max() < 1e-12
    # the diagonal factor is diagonal, the outer ones are the bit-reversed DFT and its inverse
    dd = B.dense(d)
    assert np.abs(dd - np.diag(np.diag(dd))).max() < 1e-14
    r = I.bit_reverse_index(n)
    fr = np.fft.fft(np.eye(1 << n), axis=0, norm="ortho")[r]
    assert np.abs(B.dense(q) - fr).max() < 1e-12


@pytest.mark.parametrize("n,z", [(4, 1e-4), (6, 2e-4)])
def test_bessel_route_gives_the_lattice_propagator(n, z):
    q, d, iq = B.fresnel_three_stage(n, LAM, DX, z, "bessel", "lattice")
    u = B.dense(iq) @ B.dense(d) @ B.dense(q)
    assert np.abs(u - F.lattice_matrix_1d(1 << n, LAM, DX, z)).max() < 1e-12


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_bessel_pmax14_t1_error_below_1e10_and_within_the_tail_bound(n):
    """The closed form itself (unrounded, bond 29): its error is the
    truncation of the Jacobi-Anger series, bounded by the tail sum; the
    rounded MPO adds at most its 1e-12 rounding."""
    t, pm = 1.0, 14
    x = np.arange(1 << n) / (1 << n)
    exact = np.exp(-1j * t * np.cos(2 * np.pi * x))

    def diagonal(cores):
        got = np.empty(1 << n, dtype=np.complex128)
        for i in range(1 << n):
            v = np.ones(1, dtype=np.complex128)
            for j, c in enumerate(cores):
                s = (i >> (n - 1 - j)) & 1
                v = v @ c[:, s, s, :]
            got[i] = v[0]
        return got

    raw = diagonal(B.diag_bessel(n, t, pm, rel=0))
    ps = np.arange(pm + 1, 200)
    tail = 2 * np.abs(jv(ps, t)).sum()
    err = np.abs(raw - exact).max()
    assert err < 1e-10
    assert err <= tail + 1e-14
    rounded = diagonal(B.diag_bessel(n, t, pm))
    assert np.abs(rounded - exact).max() < 1e-10


def test_angular_spectrum_diagonal_mpo_is_the_transfer_function():
    n, z = 4, 2e-4
    d = B.angular_spectrum_diag(n, LAM, DX, z)
    assert len(d) == 2 * n
    diag = np.diag(B.dense(d))
    t = F.angular_spectrum_transfer(1 << n, LAM, DX, z)
    r = I.bit_reverse_index(n)
    tq = t[r][:, r].reshape((2,) * (2 * n))
    order = []
    for p in range(n):
        order += [p, n + p]
    tq = tq.transpose(order).reshape(-1)
    assert np.abs(diag - tq).max() < 1e-12
