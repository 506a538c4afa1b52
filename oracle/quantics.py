"""Quantics (bit-interleaved) index map, Sec. 3.

An image h[a, b] on a 2^n x 2^n grid is written with the binary digits of its
two coordinates, a = (a_1 ... a_n)_2 and b = (b_1 ... b_n)_2 (digit 1 is the
most significant, i.e. the coarsest scale).  The quantics tensor has 2n binary
indices ordered a_1 b_1 a_2 b_2 ... a_n b_n, so that each consecutive pair of
sites describes one length scale.  Reading choices (the figure caption and the
footnote example in Sec. 3 are not self-consistent): most significant bit first,
row coordinate a before column coordinate b, a = first array axis.

The flat quantics vector is the C-order flattening of that 2n-index tensor, so
flat index i = sum_k s_k 2^(2n-k) with s_(2p-1) = a_p, s_(2p) = b_p.
"""
import numpy as np


def to_quantics(img):
    """N x N array -> length N^2 vector in quantics order (Sec. 3)."""
    img = np.asarray(img)
    n_side = img.shape[0]
    assert img.shape == (n_side, n_side)
    n = int(round(np.log2(n_side)))
    assert 1 << n == n_side, "side must be a power of two"
    t = img.reshape((2,) * (2 * n))            # axes: a_1..a_n, b_1..b_n
    order = []
    for p in range(n):
        order += [p, n + p]                      # a_p then b_p
    return np.ascontiguousarray(t.transpose(order)).reshape(-1)


def from_quantics(v, n):
    """Inverse of :func:`to_quantics` for a 2^n x 2^n grid."""
    v = np.asarray(v)
    t = v.reshape((2,) * (2 * n))               # axes: a_1 b_1 a_2 b_2 ...
    order = [2 * p for p in range(n)] + [2 * p + 1 for p in range(n)]
    return np.ascontiguousarray(t.transpose(order)).reshape(1 << n, 1 << n)


def quantics_flat_index(a, b, n):
    """Flat quantics index of pixel (a, b) on a 2^n grid (integer arithmetic)."""
    i = 0
    for p in range(n):
        ap = (a >> (n - 1 - p)) & 1
        bp = (b >> (n - 1 - p)) & 1
        i = (i << 2) | (ap << 1) | bp
    return i
