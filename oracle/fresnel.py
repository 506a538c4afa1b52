"""Dense FFT Fresnel propagation (Sec. 6.1).

The paraxial transfer function is separable: T(f_x, f_y) = e^(ikz) T(f_x) T(f_y)
with T(f) = exp(-i pi lambda z f^2).  The constant phase e^(ikz) is dropped
(reading), the grid is periodic with no zero padding (the FFT and the lattice
models of Sec. 6.2 are both periodic), and f runs over numpy's ``fftfreq``
ordering, i.e. bin N/2 is the negative Nyquist frequency.

E_z = IFFT2( FFT2(E_0) * T ) is the plain definition of what the MPO path
computes: in the lossless regime the MPS/MPO result equals it exactly (Sec. 5,
image formation is "exactly equivalent" to the grid FFT computation).
"""
import numpy as np


def transfer_1d(n_side, lam, dx, z):
    """T(f) = exp(-i pi lam z f^2) on the FFT frequency grid (Sec. 6.1)."""
    f = np.fft.fftfreq(n_side, d=dx)
    return np.exp(-1j * np.pi * lam * z * f * f)


def fresnel_dense(e0, lam, dx, z):
    """Propagate an N x N field by distance z (complex128)."""
    e0 = np.asarray(e0, dtype=np.complex128)
    n_side = e0.shape[0]
    t = transfer_1d(n_side, lam, dx, z)
    h = t[:, None] * t[None, :]
    return np.fft.ifft2(np.fft.fft2(e0) * h)


def fresnel_1d(u, lam, dx, z):
    """1-D propagation of a length-N vector (periodic)."""
    u = np.asarray(u, dtype=np.complex128)
    t = transfer_1d(u.shape[0], lam, dx, z)
    return np.fft.ifft(np.fft.fft(u) * t)


def fresnel_matrix_1d(n_side, lam, dx, z):
    """Dense N x N real-space propagator F^-1 diag(T) F (Sec. 6.1, Fig. MPO of
    the optical propagation): column j is the propagated unit vector e_j."""
    eye = np.eye(n_side, dtype=np.complex128)
    t = transfer_1d(n_side, lam, dx, z)
    return np.fft.ifft(np.fft.fft(eye, axis=0) * t[:, None], axis=0)


def gaussian_beam_exact(n_side, w0, lam, dx, z, ca, cb):
    """Closed-form paraxial propagation of exp(-r^2/w0^2) (r in pixels).

    Derived from the transfer function of Sec. 6.1: the Fourier transform of a
    Gaussian is Gaussian, the quadratic phase adds to its exponent, giving
    E_z = q^-1 exp(-r^2 / (w0^2 q)),  q = 1 + i z / z_R,  z_R = pi w0^2 / lam,
    with w0 and r converted to metres by dx.  Valid on the periodic grid while
    the beam tails stay negligible at the grid edge.
    """
    w = w0 * dx
    zr = np.pi * w * w / lam
    q = 1.0 + 1j * z / zr
    a = (np.arange(n_side)[:, None] - ca) * dx
    b = (np.arange(n_side)[None, :] - cb) * dx
    r2 = a * a + b * b
    return np.exp(-r2 / (w * w * q)) / q


def gaussian_beam_exact_1d(n_side, w0, lam, dx, z, c):
    """1-D closed form of the same propagation: q^-1/2 exp(-u^2 / (w0^2 q)),
    u = (index - c) dx, for the factor exp(-u^2 / w0^2) of a separable beam
    (each axis contributes q^-1/2, their product the 2-D q^-1)."""
    w = w0 * dx
    zr = np.pi * w * w / lam
    q = 1.0 + 1j * z / zr
    u = (np.arange(n_side) - c) * dx
    return np.exp(-u * u / (w * w * q)) / np.sqrt(q)


def transfer_lattice_1d(n_side, lam, dx, z):
    """Transfer function of the tight-binding (discrete Laplacian) model of
    Sec. 6.2: energies -2J cos(2 pi k / N) with hopping J = lam / (4 pi dx^2)
    (the constant shift, a global phase, chosen so that k = 0 has phase 0):
    T(k) = exp(-i 2 J z (1 - cos(2 pi k / N))).  Its small-k limit is the
    parabolic transfer function exp(-i pi lam z f^2)."""
    k = np.arange(n_side)
    two_jz = lam * z / (2.0 * np.pi * dx * dx)
    return np.exp(-1j * two_jz * (1.0 - np.cos(2.0 * np.pi * k / n_side)))


def lattice_matrix_1d(n_side, lam, dx, z):
    """Dense N x N lattice propagator F^-1 diag(T) F (periodic)."""
    eye = np.eye(n_side, dtype=np.complex128)
    t = transfer_lattice_1d(n_side, lam, dx, z)
    return np.fft.ifft(np.fft.fft(eye, axis=0) * t[:, None], axis=0)


def angular_spectrum_transfer(n_side, lam, dx, z):
    """Angular-spectrum transfer function of Sec. 6.1 on the FFT frequency
    grid, T(f_a, f_b) = exp(2 pi i z (sqrt(1/lam^2 - f_a^2 - f_b^2) - 1/lam)):
    the constant phase e^{ikz} is dropped as for the Fresnel form; where
    f_a^2 + f_b^2 > 1/lam^2 the square root is i sqrt(f^2 - 1/lam^2), so the
    evanescent components decay."""
    f = np.fft.fftfreq(n_side, d=dx)
    arg = 1.0 / lam ** 2 - (f[:, None] ** 2 + f[None, :] ** 2)
    kz = np.sqrt(arg.astype(np.complex128))          # principal root: i sqrt(|arg|) for arg < 0
    return np.exp(2j * np.pi * z * (kz - 1.0 / lam))


def angular_spectrum_dense(e0, lam, dx, z):
    """Propagate an N x N field by the angular-spectrum transfer function
    (periodic grid, no padding): IFFT2(FFT2(E0) T)."""
    e0 = np.asarray(e0, dtype=np.complex128)
    t = angular_spectrum_transfer(e0.shape[0], lam, dx, z)
    return np.fft.ifft2(np.fft.fft2(e0) * t)
