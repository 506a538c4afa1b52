"""Perfect sampling of photon detection events from a field MPS (Sec. 5):
samples (a, b) drawn with probability |E(a, b)|^2 / ||E||^2 without forming
the distribution, by drawing the quantics bits one site at a time from their
conditional probabilities.

Test infrastructure, like the rest of ``oracle``.

The MPS must be left-canonical (every core but the last an isometry from its
left bond and physical index to its right bond), as TT-SVD and the truncation
sweep leave it.  Sites are then visited from the last to the first: with the
cores left of site k an isometry, the squared norm of the partial state with
bits s_k .. s_(m-1) fixed is |A_k[s_k] R|^2, R the product of the chosen
cores right of k applied to the right boundary, so the conditional
probability of s_k is that norm over its sum for both values.  The random
numbers are inputs: bit s_k = 0 when u_k * (p0 + p1) < p0.
"""
import numpy as np


def _coords(bits, n):
    """Row and column of a quantics bit string (site 2q = bit q of the row,
    site 2q + 1 = bit q of the column, most significant first)."""
    a = b = 0
    for q in range(n):
        a |= int(bits[2 * q]) << (n - 1 - q)
        b |= int(bits[2 * q + 1]) << (n - 1 - q)
    return a, b


def perfect_samples(cores, uniforms):
    """Samples (rows, cols) for every row of ``uniforms`` (count x m), all
    samples advanced together site by site (float64)."""
    m = len(cores)
    n = m // 2
    u = np.asarray(uniforms, dtype=np.float64)
    count = u.shape[0]
    R = np.ones((count, 1), dtype=np.complex128)
    bits = np.zeros((count, m), dtype=np.int64)
    for k in range(m - 1, -1, -1):
        c = np.einsum("rsc,pc->prs", np.asarray(cores[k], dtype=np.complex128), R)
        p0 = np.sum(np.abs(c[:, :, 0]) ** 2, axis=1)
        p1 = np.sum(np.abs(c[:, :, 1]) ** 2, axis=1)
        tot = p0 + p1
        s = np.where((tot > 0) & ~(u[:, k] * tot < p0), 1, 0)
        ps = np.where(s == 1, p1, p0)
        sc = np.where(ps > 0, 1.0 / np.sqrt(np.where(ps > 0, ps, 1.0)), 0.0)
        R = c[np.arange(count), :, s] * sc[:, None]
        bits[:, k] = s
    rows = np.zeros(count, dtype=np.int64)
    cols = np.zeros(count, dtype=np.int64)
    for q in range(n):
        rows |= bits[:, 2 * q] << (n - 1 - q)
        cols |= bits[:, 2 * q + 1] << (n - 1 - q)
    return rows, cols


def sample_probability(cores, bits):
    """Probability that the sampler returns the bit string ``bits`` (product of
    its conditional probabilities, visited from the last site to the first)."""
    m = len(cores)
    R = np.ones(1, dtype=np.complex128)
    prob = 1.0
    for k in range(m - 1, -1, -1):
        c = np.einsum("rsc,c->rs", np.asarray(cores[k], dtype=np.complex128), R)
        p = np.sum(np.abs(c) ** 2, axis=0)
        s = int(bits[k])
        if p.sum() == 0:
            return 0.0
        prob *= p[s] / p.sum()
        R = c[:, s] / np.sqrt(p[s]) if p[s] > 0 else c[:, s]
    return prob


def decision_margins(cores, uniforms):
    """Smallest |u_k - p0 / (p0 + p1)| over the sites of every sample (how far
    each sample's decisions were from a tie), float64."""
    m = len(cores)
    u = np.asarray(uniforms, dtype=np.float64)
    count = u.shape[0]
    R = np.ones((count, 1), dtype=np.complex128)
    marg = np.full(count, np.inf)
    for k in range(m - 1, -1, -1):
        c = np.einsum("rsc,pc->prs", np.asarray(cores[k], dtype=np.complex128), R)
        p0 = np.sum(np.abs(c[:, :, 0]) ** 2, axis=1)
        p1 = np.sum(np.abs(c[:, :, 1]) ** 2, axis=1)
        tot = np.where(p0 + p1 > 0, p0 + p1, 1.0)
        marg = np.minimum(marg, np.abs(u[:, k] - p0 / tot))
        s = np.where(~(u[:, k] * (p0 + p1) < p0), 1, 0)
        ps = np.where(s == 1, p1, p0)
        R = c[np.arange(count), :, s] / np.sqrt(np.where(ps > 0, ps, 1.0))[:, None]
    return marg
