"""Host (float64) construction of the Fresnel propagator as matrix product operators.

Route of Sec. 6.1 (figure of the MPO product): the real-space propagator of one
axis is U = QFT_br^H . diag_br(T) . QFT_br, where
  * QFT_br is the unitary DFT with bit-reversed output, finite-rank as an MPO
    (Sec. 5).  It is built here from its circuit: for each qubit, a Hadamard
    followed by controlled phases with every later qubit; each such layer is
    a bond-2 MPO (the control bit rides along the bond) and the layers are
    multiplied in and recompressed one at a time;
  * diag_br(T) is diagonal in the bit-reversed frequency register, with
    T(f) = exp(-i pi lambda z f^2) (paraxial transfer function, Sec. 6.1) on
    the FFT frequency grid; its MPO is the sequential-SVD tensor train of the
    length-N diagonal (each core delta_{ts} V[a, t, b]);
  * the two products are formed pairwise with SVD recompression.
The 2-D operator is U^(x) (x) U^(y) (Sec. 6.1, separability): each axis MPO is
embedded in the 2n-site quantics chain with identity sites on the other axis.

Core convention: W[D_l, t, s, D_r], t = output bit, s = input bit, MSB first.
This module is host setup (not timed); it shares no code with the test oracle.
"""
import numpy as np

H1 = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)


# ------------------------------------------------------------------ helpers
def _keep(s, rel):
    """Smallest rank whose discarded squared weight is <= rel^2 of the total."""
    w = s * s
    tot = w.sum()
    if tot <= 0.0:
        return 1
    tail = np.append(np.cumsum(w[::-1])[::-1][1:], 0.0)
    return max(1, int(np.argmax(tail <= rel * rel * tot)) + 1)


def round_left(cores, rel=1e-12):
    """Left-canonical rounding of an operator MPO: an LQ sweep right to left
    (every core right of the cut an isometry), then an SVD sweep left to
    right keeping at each bond the singular values whose discarded squared
    weight is at most rel^2 / (n-1) of the total, minus numerical zeros
    (sigma_i <= 1e-13 sigma_1).  The left singular vectors stay as the cores
    and S V^H moves right, so the result is the form the sequential SVD of
    the dense operator produces (Sec. 6.1, brute-force MPO construction): every
    core but the last left-orthonormal as a (D_l * 4) x D_r matrix, the
    operator's weight in the last core, bonds equal to the Schmidt ranks at
    that cutoff.  The truncating zip-up sees the operator's left bond through
    its Gram matrices, which are invariant only under unitary changes of the
    bond basis, so this canonical form fixes what the zip-up computes."""
    c = [np.asarray(x, dtype=np.complex128) for x in cores]
    n = len(c)
    if n == 1:
        return c
    for k in range(n - 1, 0, -1):
        dl, _, _, dr = c[k].shape
        q, r = np.linalg.qr(c[k].reshape(dl, 4 * dr).conj().T)
        c[k] = q.conj().T.reshape(-1, 2, 2, dr)
        c[k - 1] = np.tensordot(c[k - 1], r.conj().T, axes=(3, 0))
    per = rel / np.sqrt(n - 1)
    for k in range(n - 1):
        dl, _, _, dr = c[k].shape
        u, s, vh = np.linalg.svd(c[k].reshape(dl * 4, dr), full_matrices=False)
        d = _keep(s, per)
        if s[0] > 0.0:
            d = min(d, max(1, int(np.count_nonzero(s > 1e-13 * s[0]))))
        c[k] = u[:, :d].reshape(dl, 2, 2, d)
        c[k + 1] = np.tensordot(s[:d, None] * vh[:d], c[k + 1], axes=(1, 0))
    return c


def compress(cores, rel=1e-13):
    """Recompress an MPO: QR sweep left to right, then SVD sweep right to left
    keeping per bond a relative discarded weight <= rel^2 / (n-1)."""
    c = [np.asarray(x, dtype=np.complex128) for x in cores]
    n = len(c)
    if n == 1:
        return c
    for k in range(n - 1):
        dl, _, _, dr = c[k].shape
        q, r = np.linalg.qr(c[k].reshape(dl * 4, dr))
        c[k] = q.reshape(dl, 2, 2, -1)
        c[k + 1] = np.tensordot(r, c[k + 1], axes=(1, 0))
    per = rel / np.sqrt(n - 1)
    for k in range(n - 1, 0, -1):
        dl, _, _, dr = c[k].shape
        u, s, vh = np.linalg.svd(c[k].reshape(dl, 4 * dr), full_matrices=False)
        r = _keep(s, per)
        c[k] = vh[:r].reshape(r, 2, 2, dr)
        c[k - 1] = np.tensordot(c[k - 1], u[:, :r] * s[:r], axes=(3, 0))
    return c


def mul(a, b):
    """Operator product A . B of two MPOs (bond dimensions multiply)."""
    out = []
    for wa, wb in zip(a, b):
        t = np.einsum("atub,cusd->actsbd", wa, wb)
        al, cl, _, _, ar, cr = t.shape
        out.append(t.reshape(al * cl, 2, 2, ar * cr))
    return out


def dagger(a):
    return [np.conj(w.transpose(0, 2, 1, 3)) for w in a]


def dense(cores):
    """Densify (small n only; used by tests and checks)."""
    n = len(cores)
    acc = np.ones((1, 1), dtype=np.complex128)
    for c in cores:
        acc = np.tensordot(acc, c, axes=(acc.ndim - 1, 0))
    acc = acc.reshape((2,) * (2 * n))
    order = [2 * p for p in range(n)] + [2 * p + 1 for p in range(n)]
    return acc.transpose(order).reshape(1 << n, 1 << n)


# ------------------------------------------------------------------ QFT
def _layer(n, q):
    """Hadamard on qubit q then controlled phases exp(-2 pi i c x / 2^(d+1))
    between its output bit c and the (untransformed) input bit x of qubit q+d."""
    cores = []
    for p in range(n):
        if p < q:
            w = np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1)
        elif p == q:
            if q == n - 1:
                w = H1.astype(np.complex128).reshape(1, 2, 2, 1)
            else:
                w = np.zeros((1, 2, 2, 2), dtype=np.complex128)
                for t in range(2):
                    w[0, t, :, t] = H1[t, :]
        else:
            d = p - q
            last = p == n - 1
            w = np.zeros((2, 2, 2, 1 if last else 2), dtype=np.complex128)
            for c in range(2):
                for x in range(2):
                    w[c, x, x, 0 if last else c] = np.exp(-2j * np.pi * c * x / 2.0 ** (d + 1))
        cores.append(w)
    return cores


def qft_br(n, rel=1e-14):
    """P_rev F as an MPO: F[k, j] = exp(-2 pi i j k / N)/sqrt(N) with the
    output register in bit-reversed order."""
    acc = _layer(n, 0)
    for q in range(1, n):
        acc = compress(mul(_layer(n, q), acc), rel)
    return acc


# ------------------------------------------------------------------ diagonal
def _vec_tt(v, rel):
    """Sequential-SVD tensor train of a length-2^n vector (MSB first)."""
    n = int(round(np.log2(v.size)))
    rem = v.reshape(1, -1).astype(np.complex128)
    cores = []
    r = 1
    per = rel / np.sqrt(max(n - 1, 1))
    for _ in range(n - 1):
        u, s, vh = np.linalg.svd(rem.reshape(2 * r, -1), full_matrices=False)
        k = _keep(s, per)
        cores.append(u[:, :k].reshape(r, 2, k))
        rem = s[:k, None] * vh[:k]
        r = k
    cores.append(rem.reshape(r, 2, 1))
    return cores


def bit_reverse(n):
    idx = np.arange(1 << n)
    rev = np.zeros_like(idx)
    for p in range(n):
        rev |= ((idx >> p) & 1) << (n - 1 - p)
    return rev


def transfer(n, lam, dx, z):
    """T(f) = exp(-i pi lambda z f^2) on numpy's FFT frequency grid."""
    f = np.fft.fftfreq(1 << n, d=dx)
    return np.exp(-1j * np.pi * lam * z * f * f)


def diag_br(n, lam, dx, z, rel=1e-14):
    v = transfer(n, lam, dx, z)[bit_reverse(n)]
    out = []
    for c in _vec_tt(v, rel):
        r0, _, r1 = c.shape
        w = np.zeros((r0, 2, 2, r1), dtype=np.complex128)
        w[:, 0, 0, :] = c[:, 0, :]
        w[:, 1, 1, :] = c[:, 1, :]
        out.append(w)
    return out


# ------------------------------------------------------------------ propagator
def fresnel_axis(n, lam, dx, z, rel=1e-12):
    """Per-axis real-space Fresnel propagator QFT_br^H diag_br(T) QFT_br, in
    the left-canonical form of `round_left` (discarded weight rel^2 / (n-1)
    per bond)."""
    q = qft_br(n)
    d = diag_br(n, lam, dx, z)
    dq = compress(mul(d, q), rel * 1e-2)
    return round_left(compress(mul(dagger(q), dq), rel * 1e-2), rel)


def identity_core(d):
    return np.einsum("ab,ts->atsb", np.eye(d), np.eye(2)).astype(np.complex128)


def embed(cores_1d, axis, diag=False):
    """2n-site quantics MPO for one axis; returns (cores, site_kind) with
    site_kind 1 on the identity (pass-through) sites and, for an operator
    diagonal in the computational basis (diag=True), 2 on its own sites."""
    cores, kind = [], []
    own = 2 if diag else 0
    for c in cores_1d:
        if axis == "x":
            cores += [c, identity_core(c.shape[3])]
            kind += [own, 1]
        else:
            cores += [identity_core(c.shape[0]), c]
            kind += [1, own]
    return cores, kind


def bonds(cores):
    return [1] + [int(c.shape[3]) for c in cores]


# ------------------------------------------------------------------ diagonal operators, other routes
# Sec. 6.2: a diagonal operator U = diag(exp(-i phi(s))) on an n-bit register
# (bits s_1..s_n, most significant first) has three constructions as an MPO:
#   * the sequential SVD of its diagonal (diag_br above);
#   * the Pauli-Z expansion phi = sum_S c_S prod_{j in S} Z_j, whose
#     coefficients are the Walsh-Hadamard transform of phi; since the strings
#     commute, U = prod_S (cos c_S I - i sin c_S P_S), each factor a bond-2
#     MPO, absorbed one after the other into the identity with recompression
#     (the gate-product circuit of the paper);
#   * for the lattice dispersion phi = t cos(2 pi x_s), x_s = sum_j s_j 2^-j,
#     the Jacobi-Anger expansion exp(-i t cos a) = sum_p (-i)^p J_p(t) e^{ipa},
#     a closed-form MPO of bond 2 p_max + 1 (phases e^{i p theta_j s_j} per
#     site, theta_j = 2 pi / 2^j, Bessel weights on the left boundary).
Z1 = np.array([1.0, -1.0])


def walsh_hadamard(phi):
    """c_S = 2^-n sum_s phi(s) (-1)^(sum_{j in S} s_j) for every subset S of
    the n register bits, indexed like the register (bit j of the index is
    bit j of the bitmask S); fast transform in n butterfly passes."""
    c = np.array(phi, dtype=np.float64).copy()
    n = int(round(np.log2(c.size)))
    h = 1
    for _ in range(n):
        c = c.reshape(-1, 2, h)
        a, b = c[:, 0, :].copy(), c[:, 1, :].copy()
        c[:, 0, :] = a + b
        c[:, 1, :] = a - b
        c = c.reshape(-1)
        h *= 2
    return c / c.size


def _string_factor(n, mask, omega):
    """MPO of exp(-i omega P_S) = cos(omega) I - i sin(omega) P_S, P_S the
    product of Z over the register bits in S (bitmask, MSB = site 0)."""
    sites = [j for j in range(n) if (mask >> (n - 1 - j)) & 1]
    eye = np.eye(2, dtype=np.complex128)
    z = np.diag(Z1).astype(np.complex128)
    cores = [eye.reshape(1, 2, 2, 1).copy() for _ in range(n)]
    if not sites:
        cores[0] = cores[0] * np.exp(-1j * omega)
        return cores
    j0, j1 = sites[0], sites[-1]
    if j0 == j1:
        cores[j0] = (np.cos(omega) * eye - 1j * np.sin(omega) * z).reshape(1, 2, 2, 1)
        return cores
    w = np.zeros((1, 2, 2, 2), dtype=np.complex128)
    w[0, :, :, 0] = np.cos(omega) * eye
    w[0, :, :, 1] = -1j * np.sin(omega) * z
    cores[j0] = w
    for j in range(j0 + 1, j1):
        w = np.zeros((2, 2, 2, 2), dtype=np.complex128)
        w[0, :, :, 0] = eye
        w[1, :, :, 1] = z if j in sites else eye
        cores[j] = w
    w = np.zeros((2, 2, 2, 1), dtype=np.complex128)
    w[0, :, :, 0] = eye
    w[1, :, :, 0] = z
    cores[j1] = w
    return cores


def diag_pauli(phi, gate_cutoff=0.0, rel=1e-12):
    """MPO of diag(exp(-i phi)) from the gates of its Pauli-Z expansion:
    strings with |c_S| > gate_cutoff (0 keeps every nonzero one), absorbed
    one by one with recompression; left-canonical result."""
    phi = np.asarray(phi, dtype=np.float64)
    n = int(round(np.log2(phi.size)))
    c = walsh_hadamard(phi)
    scale = max(np.abs(c).max(), 1e-300)
    acc = [np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1) for _ in range(n)]
    for mask in np.flatnonzero(np.abs(c) > max(gate_cutoff, 1e-15 * scale)):
        acc = compress(mul(_string_factor(n, int(mask), float(c[mask])), acc), rel * 1e-2)
    return round_left(acc, rel)


def diag_bessel(n, t, p_max, bitrev=False, rel=1e-12):
    """MPO of diag(exp(-i t cos(2 pi x))) on n register bits by the
    Jacobi-Anger expansion truncated at |p| <= p_max, x the register read
    most significant bit first (x = sum_j s_j 2^-j), or with the register in
    bit-reversed order (bitrev: site j carries the bit of weight 2^(j-1) / N,
    as the output register of QFT_br).  Closed form, then left-canonical
    rounding (the closed form's bond 2 p_max + 1 is far above the rank);
    rel = 0 returns the closed form unrounded."""
    from scipy.special import jv
    ps = np.arange(-p_max, p_max + 1)
    chi = ps.size
    left = ((-1j) ** ps) * jv(ps, t)
    theta = [2.0 * np.pi / 2.0 ** (j + 1) for j in range(n)]
    if bitrev:
        theta = theta[::-1]
    cores = []
    for j in range(n):
        w = np.zeros((chi, 2, 2, chi), dtype=np.complex128)
        for s in range(2):
            w[np.arange(chi), s, s, np.arange(chi)] = np.exp(1j * ps * theta[j] * s)
        cores.append(w)
    cores[0] = np.tensordot(left, cores[0], axes=(0, 0))[None]
    cores[-1] = cores[-1].sum(axis=3)[..., None]
    if not rel:
        return cores                                  # the closed form itself, bond 2 p_max + 1
    return round_left(compress(cores, rel * 1e-2), rel)


def transfer_lattice(n, lam, dx, z):
    """Transfer function of the lattice (tight-binding) model of Sec. 6.2 on
    the FFT frequency grid: exp(-i 2 J z (1 - cos(2 pi k / N))), hopping
    J = lam / (4 pi dx^2); the parabolic form is its small-k limit."""
    k = np.arange(1 << n)
    t = lam * z / (2.0 * np.pi * dx * dx)
    return np.exp(-1j * t * (1.0 - np.cos(2.0 * np.pi * k / (1 << n))))


def fresnel_phase_br(n, lam, dx, z, dispersion="parabolic"):
    """Phase phi with T = exp(-i phi) in the bit-reversed frequency register."""
    if dispersion == "parabolic":
        f = np.fft.fftfreq(1 << n, d=dx)
        phi = np.pi * lam * z * f * f
    else:
        k = np.arange(1 << n)
        phi = lam * z / (2.0 * np.pi * dx * dx) * (1.0 - np.cos(2.0 * np.pi * k / (1 << n)))
    return phi[bit_reverse(n)]


def diag_fresnel(n, lam, dx, z, route="svd", dispersion="parabolic", p_max=None, rel=1e-12):
    """The transfer function between the two Fourier transforms (Sec. 6.1,
    Fig. of the MPO product) as a diagonal MPO on the bit-reversed frequency
    register, by one of the routes above; left-canonical."""
    phi = fresnel_phase_br(n, lam, dx, z, dispersion)
    if route == "svd":
        return round_left(_diag_cores(_vec_tt(np.exp(-1j * phi), rel * 1e-2)), rel)
    if route == "pauli":
        return diag_pauli(phi, rel=rel)
    if route == "bessel":
        if dispersion != "lattice":
            raise ValueError("the Bessel closed form is that of the lattice dispersion")
        t = lam * z / (2.0 * np.pi * dx * dx)
        pm = p_max if p_max is not None else int(np.ceil(abs(t) + 12.0 * max(abs(t), 1.0) ** (1.0 / 3.0) + 14))
        # exp(-i t (1 - cos a)) = exp(-i t) exp(+i t cos a): the expansion at -t
        cores = diag_bessel(n, -t, pm, bitrev=True, rel=rel)
        cores[0] = cores[0] * np.exp(-1j * t)
        return cores
    raise ValueError(route)


def _diag_cores(vec_cores):
    out = []
    for c in vec_cores:
        r0, _, r1 = c.shape
        w = np.zeros((r0, 2, 2, r1), dtype=np.complex128)
        w[:, 0, 0, :] = c[:, 0, :]
        w[:, 1, 1, :] = c[:, 1, :]
        out.append(w)
    return out


def fresnel_three_stage(n, lam, dx, z, route="svd", dispersion="parabolic", rel=1e-12):
    """Per-axis factors (QFT_br, diag_br(T), QFT_br^H) of the propagator,
    each left-canonical, applied right to left: U = QFT^H . diag . QFT."""
    q = round_left(qft_br(n), rel)
    d = diag_fresnel(n, lam, dx, z, route, dispersion, rel=rel)
    return q, d, round_left(dagger(q), rel)


def angular_spectrum_diag(n, lam, dx, z, rel=1e-12):
    """Angular-spectrum transfer function exp(2 pi i z (sqrt(1/lam^2 - f^2) -
    1/lam)) (Sec. 6.1, global phase e^{ikz} dropped; evanescent components
    decay as exp(-2 pi z sqrt(f^2 - 1/lam^2))) on the 2n interleaved sites of
    the two bit-reversed frequency registers, as a diagonal MPO by the
    sequential SVD of its diagonal: not separable, so one 2-D operator."""
    fr = np.fft.fftfreq(1 << n, d=dx)[bit_reverse(n)]
    f2 = fr[:, None] ** 2 + fr[None, :] ** 2
    arg = 1.0 / lam ** 2 - f2
    kz = np.where(arg >= 0.0, np.sqrt(np.abs(arg)) + 0j, 1j * np.sqrt(np.abs(arg)))
    t = np.exp(2j * np.pi * z * (kz - 1.0 / lam))
    # quantics order: bit p of the row register then bit p of the column one
    v = t.reshape((2,) * (2 * n))
    order = []
    for p in range(n):
        order += [p, n + p]
    v = np.ascontiguousarray(v.transpose(order)).reshape(-1)
    return round_left(_diag_cores(_vec_tt(v, rel * 1e-2)), rel)
