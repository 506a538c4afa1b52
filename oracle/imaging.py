"""Image formation and point spread functions (Sec. 5), and the Pauli-Z
expansion of diagonal operators (Sec. 6.2, App. B), as plain definitions.

Test infrastructure, like the rest of ``oracle``.

* The focal-plane field of a pupil field E0 is its 2-D Fourier transform
  (Fraunhofer, Sec. 5); the quantum Fourier transform MPO produces it with
  every frequency register in bit-reversed order, so the oracle states it in
  that order: phi = (P F) E0 (P F)^T, F the unitary DFT, P the bit reversal.
* PSF = phi (.) conj(phi): the element-wise product (the local contraction
  of physical indices of Sec. 5).
* Image formation, Eq. of the convolution: IQFT(QFT(PSF) (.) QFT(S)); with
  unitary transforms this is the circular convolution PSF * S divided by N
  (each axis contributes sqrt(N)), written here exactly as composed.
* Pauli-Z coefficients of a diagonal phi over n bits: the trace formula
  c_S = 2^-n sum_s phi(s) (-1)^(sum_{j in S} s_j), and for phi = cos(2 pi x_s)
  the closed form of App. B.
"""
import numpy as np


def bit_reverse_index(n):
    idx = np.arange(1 << n)
    rev = np.zeros(1 << n, dtype=np.int64)
    for p in range(n):
        rev |= ((idx >> p) & 1) << (n - 1 - p)
    return rev


def focal_field_br(e0):
    """Unitary 2-D DFT of e0 with both frequency registers bit-reversed."""
    n = int(e0.shape[0]).bit_length() - 1
    r = bit_reverse_index(n)
    f = np.fft.fft2(np.asarray(e0, dtype=np.complex128), norm="ortho")
    return f[r][:, r]


def psf_br(e0):
    """PSF = |focal field|^2 in the bit-reversed frequency order (Sec. 5)."""
    phi = focal_field_br(e0)
    return (phi * np.conj(phi)).real


def image_formation(obj, psf):
    """IQFT(QFT(psf) (.) QFT(obj)) on an N x N grid with unitary transforms
    (the bit reversals of the QFT MPO cancel in the element-wise product)."""
    a = np.fft.fft2(np.asarray(psf, dtype=np.complex128), norm="ortho")
    b = np.fft.fft2(np.asarray(obj, dtype=np.complex128), norm="ortho")
    return np.fft.ifft2(a * b, norm="ortho")


def circular_convolution(a, b):
    """Brute-force 2-D circular convolution (small grids only)."""
    n = a.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                for l in range(n):
                    acc += a[k, l] * b[(i - k) % n, (j - l) % n]
            out[i, j] = acc
    return out


def diag_mpo_from_mps(cores, conj=False):
    """The element-wise product with an MPS as a diagonal operator:
    W_k[w, t, s, w'] = delta_ts A_k[w, s, w'] (conjugated if conj)."""
    out = []
    for c in cores:
        a = np.conj(c) if conj else np.asarray(c)
        r0, _, r1 = a.shape
        w = np.zeros((r0, 2, 2, r1), dtype=np.complex128)
        w[:, 0, 0, :] = a[:, 0, :]
        w[:, 1, 1, :] = a[:, 1, :]
        out.append(w)
    return out


def pauli_coefficients(phi):
    """c_S for every bitmask S (bit j of S = register bit j, the index's
    own bit order), from the trace formula, one subset at a time."""
    phi = np.asarray(phi, dtype=np.float64)
    size = phi.size
    out = np.zeros(size)
    for mask in range(size):
        acc = 0.0
        for s in range(size):
            sign = -1.0 if bin(s & mask).count("1") % 2 else 1.0
            acc += phi[s] * sign
        out[mask] = acc / size
    return out


def pauli_coefficients_cos(n):
    """Closed form (App. B) for phi(s) = cos(2 pi x_s), x_s = sum_j s_j 2^-j
    (s_1 the most significant bit): c_S = 0 unless the most significant bit
    is in S, else 2^(1-n) Re[gamma_n prod_{j in S, j > 1} x_j] with
    x_j = -i tan(theta_j / 2), theta_j = 2 pi / 2^j and
    gamma_n = e^{i pi (1/2 - 1/2^n)} / sin(pi / 2^n)."""
    size = 1 << n
    gamma = np.exp(1j * np.pi * (0.5 - 1.0 / size)) / np.sin(np.pi / size)
    xs = [-1j * np.tan(np.pi / 2.0 ** (j + 1)) for j in range(n)]   # x_j, j = 1..n (0-based index j-1)
    out = np.zeros(size)
    for mask in range(size):
        if not (mask >> (n - 1)) & 1:
            continue
        prod = gamma
        for j in range(1, n):
            if (mask >> (n - 1 - j)) & 1:
                prod *= xs[j]
        out[mask] = 2.0 ** (1 - n) * prod.real
    return out
