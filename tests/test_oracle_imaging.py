"""Pins of the oracle's image-formation, PSF and angular-spectrum functions
against brute force and invariants (Sec. 5, Sec. 6.1)."""
import numpy as np
import pytest

from oracle import fresnel as F
from oracle import imaging as I

LAM, DX = 500e-9, 1e-6


def _dft2_brute(e):
    n = e.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    for ka in range(n):
        for kb in range(n):
            acc = 0.0
            for a in range(n):
                for b in range(n):
                    acc += e[a, b] * np.exp(-2j * np.pi * (ka * a + kb * b) / n)
            out[ka, kb] = acc / n
    return out


def test_focal_field_is_the_bit_reversed_unitary_dft():
    rng = np.random.default_rng(1)
    e = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    ref = _dft2_brute(e)
    r = [0, 4, 2, 6, 1, 5, 3, 7]
    assert np.abs(I.focal_field_br(e) - ref[r][:, r]).max() < 1e-12


def test_psf_is_real_nonnegative_and_keeps_the_power():
    rng = np.random.default_rng(2)
    e = rng.standard_normal((16, 16)) * np.exp(1j * rng.standard_normal((16, 16)))
    p = I.psf_br(e)
    assert np.abs(p.imag).max() == 0.0 and p.real.min() >= 0.0
    assert abs(p.real.sum() - np.sum(np.abs(e) ** 2)) < 1e-10 * np.sum(np.abs(e) ** 2)


def test_image_formation_is_the_circular_convolution_over_n():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    b = rng.standard_normal((8, 8))
    assert np.abs(I.image_formation(a, b) * 8 - I.circular_convolution(a, b)).max() < 1e-12


def test_angular_spectrum_brute_force_unitary_and_paraxial_limit():
    rng = np.random.default_rng(4)
    e = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    z = 3e-6
    t = F.angular_spectrum_transfer(8, LAM, DX, z)
    # brute force: inverse DFT of the product, each by explicit sums
    fe = _dft2_brute(e) * 8
    prod = fe * t
    ref = np.zeros((8, 8), dtype=np.complex128)
    for a in range(8):
        for b in range(8):
            acc = 0.0
            for ka in range(8):
                for kb in range(8):
                    acc += prod[ka, kb] * np.exp(2j * np.pi * (ka * a + kb * b) / 8)
            ref[a, b] = acc / 64
    got = F.angular_spectrum_dense(e, LAM, DX, z)
    assert np.abs(got - ref).max() < 1e-12
    # no evanescent frequency on this grid (f_max^2 * 2 < 1 / lam^2): unitary
    assert abs(np.linalg.norm(got) - np.linalg.norm(e)) < 1e-12 * np.linalg.norm(e)
    assert np.abs(F.angular_spectrum_dense(e, LAM, DX, 0.0) - e).max() < 1e-13
    # a field of low spatial frequencies: the paraxial form is its limit
    n = 256
    g = np.exp(-((np.arange(n) - n / 2) / 40.0) ** 2)
    e2 = np.outer(g, g)
    z2 = 20e-6
    ang = F.angular_spectrum_dense(e2, LAM, DX, z2)
    par = F.fresnel_dense(e2, LAM, DX, z2)
    assert np.linalg.norm(ang - par) / np.linalg.norm(par) < 1e-3


def test_evanescent_components_decay():
    t = F.angular_spectrum_transfer(16, 2e-6, 1e-6, 1e-6)     # 1 / lam = 5e5 < f_max
    f = np.fft.fftfreq(16, d=1e-6)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    assert np.all(np.abs(t[f2 > 1 / (2e-6) ** 2]) < 1.0)
    assert np.allclose(np.abs(t[f2 < 1 / (2e-6) ** 2]), 1.0)


def test_lattice_transfer_function_has_the_parabolic_limit():
    n = 1024
    t_lat = F.transfer_lattice_1d(n, LAM, DX, 1e-3)
    t_par = F.transfer_1d(n, LAM, DX, 1e-3)
    k = np.abs(np.fft.fftfreq(n)) * n
    small = k < 20
    # phases agree to O(k^4): lam z / (2 pi dx^2) (2 pi k / N)^4 / 24
    kk = 2 * np.pi * k[small] / n
    bound = LAM * 1e-3 / (2 * np.pi * DX * DX) * kk ** 4 / 24 * 1.01 + 1e-12
    assert np.all(np.abs(np.angle(t_lat[small] / t_par[small])) <= bound)
