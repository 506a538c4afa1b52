"""Pins for the oracle's differentiable twin (oracle.grad).

Independent references:
* the numpy oracle's forward result (same algorithm, other library);
* brute-force environments of the decompression: the gradient of a linear
  functional of the dense field with respect to core k is the contraction of
  the probe with the conjugated other cores, evaluated here pixel by pixel;
* in the lossless regime the propagation is exactly the unitary Fresnel
  operator, so the gradient of Re <probe, P_z dense(psi)> equals the gradient
  of Re <P_z^H probe, dense(psi)>, and P_z^H is propagation by -z (dense FFT);
* central finite differences of the float64 loss in the truncated regime.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fresnel as F
from oracle import grad as OG
from oracle import mpo as M
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

LAM, DX = 500e-9, 1e-6
BIG = 1 << 20


def _axis_mpos(n, z):
    c = M.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    return M.embed_axis(c, "x"), M.embed_axis(c, "y")


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _rand_cores(rng, m, chi):
    bonds = [1] + [min(chi, 2 ** min(k, m - k)) for k in range(1, m)] + [1]
    return [(rng.standard_normal((bonds[k], 2, bonds[k + 1])) +
             1j * rng.standard_normal((bonds[k], 2, bonds[k + 1]))) / np.sqrt(2 * bonds[k])
            for k in range(m)]


def test_forward_twin_matches_numpy_oracle():
    n, z, chi = 4, 40e-6, 6
    e0 = synth.random_field(3, 1 << n)
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi=8)
    wx, wy = _axis_mpos(n, z)
    c1, _ = Z.mpo_apply(cores, wx, chi)
    c2, _ = Z.mpo_apply(c1, wy, chi)
    ref = Z.to_dense(c2, n)
    with torch.no_grad():
        got = OG.to_dense(OG.propagate(OG.as_tensors(cores), wx, wy, chi), n).numpy()
    assert _rel(got, ref) < 1e-12


def _brute_dense_grad(cores, probe_q):
    """d Re<probe, dense(psi)> / d core_k, pixel by pixel (torch convention:
    grad = probe contracted with the conjugated other cores)."""
    m = len(cores)
    grads = [np.zeros_like(c) for c in cores]
    for idx in range(1 << m):
        bits = [(idx >> (m - 1 - k)) & 1 for k in range(m)]
        left = [np.ones((1,), dtype=np.complex128)]
        for k in range(m):
            left.append(left[-1] @ cores[k][:, bits[k], :])
        right = [np.ones((1,), dtype=np.complex128)]
        for k in range(m - 1, -1, -1):
            right.append(cores[k][:, bits[k], :] @ right[-1])
        right = right[::-1]                       # right[k] = A_k ... A_(m-1) applied to 1
        for k in range(m):
            env = np.outer(left[k], right[k + 1])
            grads[k][:, bits[k], :] += probe_q[idx] * np.conj(env)
    return grads


def test_decompression_gradient_vs_brute_force():
    n = 3
    rng = np.random.default_rng(11)
    cores = _rand_cores(rng, 2 * n, 4)
    probe = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    got = OG.dense_linear_grad(cores, probe, n)
    ref = _brute_dense_grad(cores, Q.to_quantics(probe))
    for g, r in zip(got, ref):
        assert _rel(g, r) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_lossless_apply_gradient_equals_fft_adjoint(seed):
    n, z = 3, 4e-6
    rng = np.random.default_rng(seed)
    cores = _rand_cores(rng, 2 * n, 4)
    probe = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    wx, wy = _axis_mpos(n, z)
    val, got = OG.linear_grad(cores, wx, wy, probe, BIG, n, chi_zip=BIG)
    back = F.fresnel_dense(probe, LAM, DX, -z)            # P_z^H probe
    ref = OG.dense_linear_grad(cores, back, n)
    dense_in = Z.to_dense(cores, n)
    assert abs(val - np.real(np.vdot(back, dense_in))) < 1e-12 * abs(val) + 1e-12
    for g, r in zip(got, ref):
        assert _rel(g, r) < 1e-9


@pytest.mark.parametrize("chi,seed", [(5, 5), (3, 6), (8, 7)])
def test_truncated_loss_gradient_vs_finite_differences(chi, seed):
    n, z = 4, 30e-6
    rng = np.random.default_rng(seed)
    mask = T.tt_svd(Q.to_quantics(np.exp(1j * synth.smoothed_phase(2, 1 << n, 1.5, np.pi / 4))), 2 * n, chi)
    tgt_field = np.exp(1j * synth.smoothed_phase(3, 1 << n, 1.5, np.pi / 2))
    tcores = T.tt_svd(Q.to_quantics(tgt_field), 2 * n, chi)
    wx, wy = _axis_mpos(n, z)
    t1, _ = Z.mpo_apply(tcores, wx, chi)
    t2, _ = Z.mpo_apply(t1, wy, chi)
    target = np.abs(Z.to_dense(t2, n)) ** 2
    loss, grads = OG.loss_and_grad(mask, wx, wy, target, chi, n)

    def loss_at(cores):
        with torch.no_grad():
            out = OG.propagate(OG.as_tensors(cores), wx, wy, chi)
            return float(OG.intensity_loss(OG.to_dense(out, n), torch.as_tensor(target)))

    assert abs(loss_at(mask) - loss) < 1e-12 * loss
    h = 1e-6
    errs = []
    for _ in range(20):
        k = int(rng.integers(0, 2 * n))
        idx = tuple(int(rng.integers(0, d)) for d in mask[k].shape)
        for unit, part in ((1.0, "re"), (1j, "im")):
            cp = [c.copy() for c in mask]
            cm = [c.copy() for c in mask]
            cp[k][idx] += h * unit
            cm[k][idx] -= h * unit
            fd = (loss_at(cp) - loss_at(cm)) / (2 * h)
            g = grads[k][idx]
            ad = g.real if part == "re" else g.imag
            errs.append(abs(fd - ad) / max(1e-3, max(abs(g) for g in np.concatenate([q.ravel() for q in grads]))))
    assert max(errs) < 1e-6


def test_loss_gradient_where_the_keep_threshold_binds_vs_finite_differences():
    """A keep threshold that binds (tau = 1e-8 on lam_i / lam_1: the ranks of
    a smooth mask's propagation drop below those kept at the float64 floor)
    leaves the twin's gradient equal to central finite differences of its own
    loss: the threshold selects the kept pairs, the derivative stays exact
    (no pair of this problem straddles the cut closer than GAP_AD lam_1; at
    tau = 1e-10 some do, and dropping them moves the gradient by 8e-4 of its
    largest entry)."""
    n, z, chi = 5, 40e-6, 32
    rng = np.random.default_rng(11)
    mask = T.tt_svd(Q.to_quantics(np.exp(1j * synth.smoothed_phase(21, 1 << n, 6.0, np.pi / 8))), 2 * n, chi)
    tgt = np.exp(1j * synth.smoothed_phase(22, 1 << n, 3.0, np.pi / 2))
    wx, wy = _axis_mpos(n, z)
    tc = T.tt_svd(Q.to_quantics(tgt), 2 * n, chi)
    t1, _ = Z.mpo_apply(tc, wx, chi)
    t2, _ = Z.mpo_apply(t1, wy, chi)
    target = np.abs(Z.to_dense(t2, n)) ** 2
    with torch.no_grad():
        floor = OG.propagate(OG.as_tensors(mask), wx, wy, chi)
        ad_map = OG.propagate(OG.as_tensors(mask), wx, wy, chi, tau=1e-8)
    b_floor = [1] + [int(c.shape[2]) for c in floor]
    b_ad = [1] + [int(c.shape[2]) for c in ad_map]
    assert any(x < y for x, y in zip(b_ad, b_floor)), (b_ad, b_floor)
    loss, grads = OG.loss_and_grad(mask, wx, wy, target, chi, n, tau=1e-8)

    def loss_at(cores):
        with torch.no_grad():
            out = OG.propagate(OG.as_tensors(cores), wx, wy, chi, tau=1e-8)
            return float(OG.intensity_loss(OG.to_dense(out, n), torch.as_tensor(target)))

    gmax = max(np.abs(g).max() for g in grads)
    h = 1e-6
    worst = 0.0
    for _ in range(20):
        k = int(rng.integers(0, 2 * n))
        idx = tuple(int(rng.integers(0, d)) for d in mask[k].shape)
        for unit in (1.0, 1j):
            cp = [c.copy() for c in mask]
            cm = [c.copy() for c in mask]
            cp[k][idx] += h * unit
            cm[k][idx] -= h * unit
            fd = (loss_at(cp) - loss_at(cm)) / (2 * h)
            ad = grads[k][idx].real if unit == 1.0 else grads[k][idx].imag
            worst = max(worst, abs(fd - ad) / gmax)
    assert worst < 1e-6
