"""Seeded generators for the synthetic workloads.

Recipes (all on an N x N grid, pixel (a, b) with a = row):

* ``blob_image``      64x64 real image: 20 Gaussian blobs + a linear ramp +
                      1/|f|-amplitude noise at 5 % of the clean RMS.
* ``aperture_field``  complex field: hard disk of radius 300*N/1024 px whose
                      amplitude is modulated by a 1/|f|^2-power random field,
                      times exp(i phi) with phi = iid U(0, 2 pi) smoothed by a
                      Gaussian (sigma 4 px, periodic).
* ``beam_grating_field`` Gaussian beam (off-centre, to break the x/y symmetry)
                      times a binary grating along the rows.
* ``batch_specs``     (side exponent, bond cap) draws for a batch of fields.
* ``grating_beam_1d`` the two 1-D factors of the separable 16384^2 field.
* ``smoothed_phase``  iid N(0,1) smoothed with a periodic Gaussian, scaled to
                      a given standard deviation (phase masks / targets).
"""
import numpy as np
from scipy import ndimage


def _power_law_noise(rng, n, exponent):
    """Real random field whose Fourier amplitude falls as |f|^-exponent.

    White Gaussian noise is filtered in Fourier space; the DC term is removed
    and the result standardised to zero mean, unit variance.
    """
    white = rng.standard_normal((n, n))
    fa = np.fft.fftfreq(n)[:, None]
    fb = np.fft.fftfreq(n)[None, :]
    fr = np.sqrt(fa * fa + fb * fb)
    filt = np.zeros_like(fr)
    nz = fr > 0
    filt[nz] = fr[nz] ** (-exponent)
    out = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
    out -= out.mean()
    sd = out.std()
    return out / sd if sd > 0 else out


def blob_image(seed, n=64, n_blobs=20):
    """Real n x n test image (float64): blobs + ramp + 1/f noise at 5 % RMS.

    Draw order: centres, widths, amplitudes, ramp gradient, noise.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, n, size=(n_blobs, 2))
    sig = rng.uniform(1.0, 6.0, size=n_blobs)
    amp = rng.uniform(0.0, 1.0, size=n_blobs)
    grad = rng.uniform(0.0, 0.5, size=2)
    a = np.arange(n, dtype=np.float64)[:, None]
    b = np.arange(n, dtype=np.float64)[None, :]
    img = np.zeros((n, n))
    for (ca, cb), s, h in zip(centres, sig, amp):
        d2 = (a - ca) ** 2 + (b - cb) ** 2
        img += h * np.exp(-d2 / (2.0 * s * s))
    img += grad[0] * a / (n - 1) + grad[1] * b / (n - 1)
    rms = np.sqrt(np.mean(img * img))
    img += 0.05 * rms * _power_law_noise(rng, n, 1.0)
    return img


def aperture_field(seed, n=1024, radius=None, phase_sigma=4.0):
    """Complex n x n field (complex128): disk aperture x 1/f^2-power amplitude
    modulation x smoothed random phase."""
    rng = np.random.default_rng(seed)
    if radius is None:
        radius = round(300 * n / 1024)
    c = n // 2
    a = np.arange(n)[:, None] - c
    b = np.arange(n)[None, :] - c
    disk = (a * a + b * b) <= radius * radius
    mod = _power_law_noise(rng, n, 1.0)          # |f|^-1 amplitude = |f|^-2 power
    amp = disk * np.maximum(0.0, 1.0 + 0.5 * mod)
    raw = rng.uniform(0.0, 2.0 * np.pi, size=(n, n))
    phase = ndimage.gaussian_filter(raw, phase_sigma, mode="wrap")
    return amp * np.exp(1j * phase)


def gaussian_beam(n, w0, ca, cb):
    """exp(-r^2 / w0^2) centred at pixel (ca, cb) (float64), no wrap."""
    a = np.arange(n, dtype=np.float64)[:, None] - ca
    b = np.arange(n, dtype=np.float64)[None, :] - cb
    return np.exp(-(a * a + b * b) / (w0 * w0))


def beam_grating_field(n=1024, w0=100.0, period=64, offset=(37.0, -21.0)):
    """Off-centre Gaussian beam times a binary row grating (complex128).

    The grating m(a) = 1 if a mod period < period/2 depends on few quantics
    bits only, and the off-centre beam breaks the x <-> y symmetry so that
    singular values at the bond cuts are not exactly degenerate.
    """
    g = gaussian_beam(n, w0, n / 2 + offset[0], n / 2 + offset[1])
    m = ((np.arange(n) % period) < period // 2).astype(np.float64)[:, None]
    return (g * m).astype(np.complex128)


def grating_beam_1d(n=16384, w0=2000.0, period=64):
    """The separable factors (row vector, column vector) of the large field
    E0[a, b] = m(a) g(a) * g(b), g(u) = exp(-(u - n/2)^2 / w0^2)."""
    u = np.arange(n, dtype=np.float64)
    g = np.exp(-((u - n / 2) ** 2) / (w0 * w0))
    m = ((np.arange(n) % period) < period // 2).astype(np.float64)
    return (m * g).astype(np.complex128), g.astype(np.complex128)


def batch_specs(seed, count=256, k_lo=8, k_hi=11, chis=(16, 32, 64, 128)):
    """Independent draws of the side exponent k (U{k_lo..k_hi}) and bond cap
    (uniform over ``chis``) for a batch of fields.  Returns a list of
    (k, chi, field_seed)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(k_lo, k_hi + 1, size=count)
    cs = rng.choice(np.asarray(chis), size=count)
    fseeds = rng.integers(0, 2**31 - 1, size=count)
    return [(int(k), int(c), int(s)) for k, c, s in zip(ks, cs, fseeds)]


def smoothed_phase(seed, n, sigma, std):
    """iid N(0,1) smoothed by a periodic Gaussian of width ``sigma`` px,
    rescaled to standard deviation ``std`` (float64)."""
    rng = np.random.default_rng(seed)
    raw = rng.standard_normal((n, n))
    ph = ndimage.gaussian_filter(raw, sigma, mode="wrap")
    ph -= ph.mean()
    s = ph.std()
    return ph * (std / s) if s > 0 else ph


def random_field(seed, n):
    """iid complex Gaussian n x n field (complex128), for brute-force tests."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


def beam_sum_1d(seed, n, rank, w_frac=(0.05, 0.2), tilt_max=0.05):
    """Factors of a field of separation rank ``rank``: a sum of Gaussian beams
    with tilts, E0[a, b] = sum_r u_r(a) v_r(b), each u_r, v_r a 1-D Gaussian
    exp(-(x - c)^2 / w^2) times a tilt exp(2 pi i f x) (centre c ~ U(0.2, 0.8) n,
    width w ~ U(w_frac) n, tilt f ~ U(-tilt_max, tilt_max) cycles/px, complex
    amplitude of unit modulus on u_r).  Returns two complex128 arrays
    (rank, n)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n, dtype=np.float64)
    us, vs = [], []
    for _ in range(rank):
        facs = []
        for _axis in range(2):
            c = rng.uniform(0.2, 0.8) * n
            w = rng.uniform(*w_frac) * n
            f = rng.uniform(-tilt_max, tilt_max)
            facs.append(np.exp(-((x - c) ** 2) / (w * w)) * np.exp(2j * np.pi * f * x))
        amp = np.exp(2j * np.pi * rng.uniform())
        us.append(amp * facs[0])
        vs.append(facs[1])
    return np.stack(us), np.stack(vs)
