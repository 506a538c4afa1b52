"""GPU parity of the adjoint (mpo_apply_backward, tt_to_dense_backward, the
intensity loss) against the float64 oracle gradient (oracle.grad), plus
central finite differences of the GPU's own FP64 forward.

Both sides start from the same cores and the same (oracle-built) MPO cores,
so the truncations are identical; the compared quantity is the gradient on
the input cores, which is gauge invariant.  Bars (relative L2 over all
entries): linear functional through two truncated applications 1e-10 (FP64)
and 1e-4 (FP32); phase-retrieval loss gradient 1e-8 (FP64) and 2e-4 (FP32),
the FP32 bar being tighter than the 1e-3 proposed for this adjoint.
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import fresnel as F
from oracle import grad as OG
from oracle import mpo as OM
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

pytestmark = pytest.mark.gpu
LAM, DX = 500e-9, 1e-6


def _api():
    from paper_2510_23089_amd import api
    return api


def _mpos(n, z):
    c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << n, LAM, DX, z), n)
    return OM.embed_axis(c, "x"), OM.embed_axis(c, "y")


def _grad_list(api, g):
    return g.host_cores()


def _rel_list(a, b):
    num = sum(np.linalg.norm(x - y) ** 2 for x, y in zip(a, b))
    den = sum(np.linalg.norm(y) ** 2 for y in b)
    return float(np.sqrt(num / den))


def _rand_cores(rng, m, chi):
    bonds = [1] + [min(chi, 2 ** min(k, m - k)) for k in range(1, m)] + [1]
    return [(rng.standard_normal((bonds[k], 2, bonds[k + 1])) +
             1j * rng.standard_normal((bonds[k], 2, bonds[k + 1]))) / np.sqrt(2 * bonds[k])
            for k in range(m)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,chi", [(1, 2), (3, 4), (4, 7), (5, 16)])
def test_dense_backward_vs_oracle(prec, n, chi):
    torch = need_gpu()
    api = _api()
    say("dense_backward", prec, n, chi)
    rng = np.random.default_rng(n * 10 + chi)
    cores = _rand_cores(rng, 2 * n, chi)
    probe = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    psi = api.MPS.from_host(cores, chi_cap=chi + 1, dtype=dt)
    g = api.tt_to_dense_backward(psi, torch.from_numpy(probe).to(dt).cuda())
    api.check_status()
    got = g.host_cores()
    ref = OG.dense_linear_grad(cores, probe, n)
    assert g.host_bonds() == psi.host_bonds()
    tol = 1e-5 if prec == "fp32" else 1e-12
    assert _rel_list(got, ref) < tol
    # padding outside the bonds is zeroed
    full = g.cores.cpu().numpy()
    b = g.host_bonds()
    for k in range(2 * n):
        blk = full[k].copy()
        blk[:b[k], :, :b[k + 1]] = 0
        assert np.all(blk == 0)


def test_intensity_loss_kernel():
    torch = need_gpu()
    api = _api()
    rng = np.random.default_rng(3)
    e = rng.standard_normal((3, 32, 32)) + 1j * rng.standard_normal((3, 32, 32))
    t = rng.uniform(0, 2, (3, 32, 32))
    for dt in (torch.complex64, torch.complex128):
        ee = torch.from_numpy(e).to(dt).cuda()
        loss, grad = api.intensity_loss(ee, torch.from_numpy(t).cuda())
        ei = ee.cpu().numpy().astype(np.complex128)
        d = np.abs(ei) ** 2 - t
        ref = np.sum(d * d, axis=(1, 2))
        tol = 1e-6 if dt == torch.complex64 else 1e-13
        assert np.max(np.abs(loss.cpu().numpy() - ref) / ref) < tol
        assert rel(grad.cpu().numpy(), 4 * d * ei) < tol


def _linear_case(n, z, chi, seed, field="random"):
    rng = np.random.default_rng(seed)
    if field == "random":
        e0 = synth.random_field(seed, 1 << n)
    else:
        e0 = np.exp(1j * synth.smoothed_phase(seed, 1 << n, 1.5, np.pi / 3))
    cores = T.tt_svd(Q.to_quantics(e0), 2 * n, chi, tau=1e-13)
    probe = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    return cores, probe


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,chi,z", [(3, 3, 5e-6), (4, 5, 30e-6), (5, 8, 60e-6)])
def test_apply_backward_linear_functional_vs_oracle(prec, n, chi, z):
    """d Re<probe, dense(W^y W^x psi)> / d psi through both truncated applications."""
    torch = need_gpu()
    api = _api()
    say("apply_backward", prec, n, chi, z)
    cores, probe = _linear_case(n, z, chi, seed=n)
    wx, wy = _mpos(n, z)
    _, ref = OG.linear_grad(cores, wx, wy, probe, chi, n, tau=1e-13)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    Wx, Wy = api.MPO(wx, dtype=dt), api.MPO(wy, dtype=dt)
    psi = api.MPS.from_host(cores, chi_cap=chi, dtype=dt)
    s1 = api.saved_buffer(psi, Wx, chi)
    mid = api.mpo_apply(psi, Wx, chi, saved=s1)
    s2 = api.saved_buffer(mid, Wy, chi)
    out = api.mpo_apply(mid, Wy, chi, saved=s2)
    g_out = api.tt_to_dense_backward(out, torch.from_numpy(probe).to(dt).cuda())
    s1c, s2c = s1.clone(), s2.clone()
    g_mid = api.mpo_apply_backward(mid, Wy, chi, s2, out, g_out)
    g_in = api.mpo_apply_backward(psi, Wx, chi, s1, mid, g_mid)
    api.check_status()
    got = g_in.host_cores()
    assert g_in.host_bonds() == psi.host_bonds()
    err = _rel_list(got, ref)
    say("  rel err", err)
    assert err < (1e-4 if prec == "fp32" else 1e-10)
    # the saved buffers are only read: a second adjoint from them repeats the first bit for bit
    assert torch.equal(s1, s1c) and torch.equal(s2, s2c)
    g_in2 = api.mpo_apply_backward(psi, Wx, chi, s1, mid, api.mpo_apply_backward(mid, Wy, chi, s2, out, g_out))
    api.check_status()
    assert torch.equal(g_in2.cores, g_in.cores)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_phase_retrieval_gradient_vs_oracle(prec):
    torch = need_gpu()
    api = _api()
    from paper_2510_23089_amd import autograd as AG
    n, z, chi = 5, 40e-6, 8
    say("phase retrieval grad", prec)
    mask = T.tt_svd(Q.to_quantics(np.exp(1j * synth.smoothed_phase(2, 1 << n, 2.0, np.pi / 8))), 2 * n, chi,
                    tau=1e-13)
    tgt = np.exp(1j * synth.smoothed_phase(3, 1 << n, 2.0, np.pi / 2))
    wx, wy = _mpos(n, z)
    tc = T.tt_svd(Q.to_quantics(tgt), 2 * n, chi, tau=1e-13)
    t1, _ = Z.mpo_apply(tc, wx, chi, tau=1e-13)
    t2, _ = Z.mpo_apply(t1, wy, chi, tau=1e-13)
    target = np.abs(Z.to_dense(t2, n)) ** 2
    loss_ref, gref = OG.loss_and_grad(mask, wx, wy, target, chi, n, tau=1e-13)
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    rt = torch.float32 if prec == "fp32" else torch.float64
    pr = AG.PhaseRetrieval(api.MPO(wx, dtype=dt), api.MPO(wy, dtype=dt), chi, tau=1e-13)
    psi = api.MPS.from_host(mask, chi_cap=chi, dtype=dt)
    loss, g = pr.loss_and_grad(psi.cores, psi.bonds, torch.from_numpy(target).to(rt).cuda())
    api.check_status()
    b = psi.host_bonds()
    gn = g.cpu().numpy()
    got = [gn[k, :b[k], :, :b[k + 1]] for k in range(2 * n)]
    lt = 1e-5 if prec == "fp32" else 1e-11
    assert abs(float(loss) - loss_ref) < lt * loss_ref
    err = _rel_list(got, gref)
    say("  rel err", err)
    assert err < (2e-4 if prec == "fp32" else 1e-8)


def test_phase_retrieval_fd_on_gpu_fp64():
    """Central differences of the GPU's own FP64 loss vs its adjoint."""
    torch = need_gpu()
    api = _api()
    from paper_2510_23089_amd import autograd as AG
    n, z, chi = 4, 30e-6, 5
    mask = T.tt_svd(Q.to_quantics(np.exp(1j * synth.smoothed_phase(4, 1 << n, 1.5, np.pi / 4))), 2 * n, chi,
                    tau=1e-13)
    wx, wy = _mpos(n, z)
    target = np.abs(synth.random_field(9, 1 << n)) ** 2
    dt, rt = torch.complex128, torch.float64
    pr = AG.PhaseRetrieval(api.MPO(wx, dtype=dt), api.MPO(wy, dtype=dt), chi, tau=1e-13)
    psi = api.MPS.from_host(mask, chi_cap=chi, dtype=dt)
    tg = torch.from_numpy(target).to(rt).cuda()
    loss, g = pr.loss_and_grad(psi.cores, psi.bonds, tg)
    gn = g.cpu().numpy()
    gmax = np.abs(gn).max()
    rng = np.random.default_rng(1)
    b = psi.host_bonds()
    h = 1e-6
    worst = 0.0
    for _ in range(12):
        k = int(rng.integers(0, 2 * n))
        idx = (k, int(rng.integers(0, b[k])), int(rng.integers(0, 2)), int(rng.integers(0, b[k + 1])))
        for unit in (1.0, 1j):
            cp = psi.cores.clone()
            cm = psi.cores.clone()
            cp[idx] += h * unit
            cm[idx] -= h * unit
            with torch.no_grad():
                lp = float(pr.loss(cp, psi.bonds, tg))
                lm = float(pr.loss(cm, psi.bonds, tg))
            fd = (lp - lm) / (2 * h)
            ad = gn[idx].real if unit == 1.0 else gn[idx].imag
            worst = max(worst, abs(fd - ad) / gmax)
    api.check_status()
    assert worst < 1e-5


def test_batched_backward_equals_single():
    torch = need_gpu()
    api = _api()
    n, z, chi = 4, 30e-6, 6
    wx, wy = _mpos(n, z)
    fields = [_linear_case(n, z, chi, seed=s) for s in (1, 2, 3)]
    dt = torch.complex64
    Wx = api.MPO(wx, dtype=dt)
    Wxb = api.MPOBatch([wx] * 3, dtype=dt)
    batch = api.MPSBatch(3, 2 * n, chi, dtype=dt)
    for f, (cores, _) in enumerate(fields):
        batch.fill_from(api.MPS.from_host(cores, chi_cap=chi, dtype=dt), f)
    probes = torch.from_numpy(np.stack([p for _, p in fields])).to(dt).cuda()
    sb = api.saved_buffer(batch, Wxb, chi)
    outb = api.mpo_apply_batched(batch, Wxb, chi, saved=sb)
    gob = api.tt_to_dense_backward_batched(outb, probes)
    gib = api.mpo_apply_backward_batched(batch, Wxb, chi, sb, outb, gob)
    api.check_status()
    for f, (cores, _) in enumerate(fields):
        psi = api.MPS.from_host(cores, chi_cap=chi, dtype=dt)
        s1 = api.saved_buffer(psi, Wx, chi)
        out = api.mpo_apply(psi, Wx, chi, saved=s1)
        go = api.tt_to_dense_backward(out, probes[f])
        gi = api.mpo_apply_backward(psi, Wx, chi, s1, out, go)
        api.check_status()
        a = gib.field(f)
        bb = gi.host_cores()
        assert _rel_list(a, bb) < 1e-5


def test_phase_retrieval_gradient_at_the_c5_bond_shape():
    """The phase-retrieval gradient at the bond and operator shapes of the
    4096^2 benchmark problem, on its 1024^2 stand-in (20 sites; mask and
    application caps chi = 64, so the same 128 x 128 Gram eigenproblems;
    Fresnel MPO at z = 2 mm, operator bond 32): two problems, each in four
    of eight batch slots (every slot seeds inverse iteration differently):
    masks exp(i phi) with phi smoothed over 16 px at std pi/8, targets the
    oracle's propagated intensity of masks at std pi/2; keep rule with
    tau = 1e-13 on both sides.  Bars, every slot: GPU FP32 gradient vs the
    FP64 oracle gradient 1e-3 relative L2, GPU FP64 vs oracle 1e-5, GPU FP32
    vs GPU FP64 1e-3 (measured: FP32 1.0-3.1e-4, FP64 4e-9 to 2.5e-7; with
    the adjoint's pair cutoff at 1e-12 lam_1 instead of 1e-10 some slots
    reached 4e-3 in FP32 and 6e-3 in FP64); central differences of the GPU
    FP64 loss on 50 seeded entries agree with the adjoint to 2e-3 of the
    largest gradient entry at h = 1e-3 and to 1e-6 at h = 1e-6, on the same
    problem with tau = 1e-8 (at tau = 1e-13 kept eigenvalues near 1e-13 lam_1
    cross the threshold under a step of 1e-6, so the loss is not smooth at
    that scale, and at tau = 1e-10 pairs straddle the cut closer than the
    pair cutoff): the cuts at chi = 64 separate eigenvalues only 2-5 % apart,
    so a step of 1e-3 in a core entry leaves the linear regime of the
    truncation (measured: 1.9e-4 at h = 1e-3, 3.5e-8 at 1e-6)."""
    torch = need_gpu()
    api = _api()
    from paper_2510_23089_amd import autograd as AG
    n, z, chi = 10, 2e-3, 64
    tau = 1e-13
    say("phase retrieval at the C5 bond shape (1024^2 stand-in, chi 64)")
    wx, wy = _mpos(n, z)
    masks, targets = [], []
    for p in range(2):
        ph = synth.smoothed_phase(1000 + p, 1 << n, 16.0, np.pi / 8)
        masks.append(T.tt_svd(Q.to_quantics(np.exp(1j * ph)), 2 * n, chi, tau=1e-13))
        tph = synth.smoothed_phase(2000 + p, 1 << n, 16.0, np.pi / 2)
        tc = T.tt_svd(Q.to_quantics(np.exp(1j * tph)), 2 * n, chi, tau=1e-13)
        t1, _ = Z.mpo_apply(tc, wx, chi, tau=1e-13)
        t2, _ = Z.mpo_apply(t1, wy, chi, tau=1e-13)
        targets.append(np.abs(Z.to_dense(t2, n)) ** 2)
    refs = [OG.loss_and_grad(masks[p], wx, wy, targets[p], chi, n, tau=tau) for p in range(2)]

    slots = [0, 1, 1, 0, 0, 1, 1, 0]

    def run(prec, tau=tau):
        dt = torch.complex64 if prec == "fp32" else torch.complex128
        rt = torch.float32 if prec == "fp32" else torch.float64
        ns = len(slots)
        psi = api.MPSBatch(ns, 2 * n, chi, dtype=dt)
        for i, p in enumerate(slots):
            psi.fill_from(api.MPS.from_host(masks[p], chi_cap=chi, dtype=dt), i)
        pr = AG.PhaseRetrieval(api.MPOBatch([wx] * ns, dtype=dt), api.MPOBatch([wy] * ns, dtype=dt), chi, tau=tau)
        tg = torch.from_numpy(np.stack([targets[p] for p in slots])).to(rt).cuda()
        loss, g = pr.loss_and_grad(psi.cores, psi.bonds, tg)
        api.check_status()
        b = psi.bonds.cpu().numpy()
        gn = g.cpu().numpy()
        grads = [[gn[i, k, :b[i, k], :, :b[i, k + 1]].astype(np.complex128) for k in range(2 * n)]
                 for i in range(ns)]
        return float(loss), grads, (pr, psi, tg, gn, b)

    l32, g32, _ = run("fp32")
    l64, g64, _ = run("fp64")
    lref = sum(refs[p][0] for p in slots)
    assert abs(l64 - lref) < 1e-10 * lref
    assert abs(l32 - lref) < 1e-5 * lref
    errs = []
    for i, p in enumerate(slots):
        e32, e64, e3264 = _rel_list(g32[i], refs[p][1]), _rel_list(g64[i], refs[p][1]), _rel_list(g32[i], g64[i])
        say("  slot %d (problem %d): fp32 vs oracle %.2e, fp64 vs oracle %.2e, fp32 vs fp64 %.2e"
            % (i, p, e32, e64, e3264))
        errs.append((e32, e64, e3264))
    for e32, e64, e3264 in errs:
        assert e32 < 1e-3
        assert e64 < 1e-5
        assert e3264 < 1e-3
    _, _, (pr, psi, tg, gn, b) = run("fp64", 1e-8)
    rng = np.random.default_rng(5)
    gmax = np.abs(gn).max()
    h = 1e-3

    def dq(idx, unit, step):
        cp, cm = psi.cores.clone(), psi.cores.clone()
        cp[idx] += step * unit
        cm[idx] -= step * unit
        with torch.no_grad():
            return (float(pr.loss(cp, psi.bonds, tg)) - float(pr.loss(cm, psi.bonds, tg))) / (2 * step)

    worst, worst_small = 0.0, 0.0
    for _ in range(50):
        p = int(rng.integers(0, len(slots)))
        k = int(rng.integers(0, 2 * n))
        idx = (p, k, int(rng.integers(0, b[p, k])), int(rng.integers(0, 2)), int(rng.integers(0, b[p, k + 1])))
        unit = 1.0 if rng.integers(0, 2) == 0 else 1j
        ad = gn[idx].real if unit == 1.0 else gn[idx].imag
        worst = max(worst, abs(dq(idx, unit, h) - ad) / gmax)
        worst_small = max(worst_small, abs(dq(idx, unit, 1e-6) - ad) / gmax)
    api.check_status()
    say("  FD h=1e-3: %.2e of max|g|, h=1e-6: %.2e" % (worst, worst_small))
    assert worst < 2e-3
    assert worst_small < 1e-6


def test_phase_retrieval_gradient_4096_batch_of_32_every_position():
    """The benchmark's gradient step at its own shape: 32 problems of 4096^2
    (24 sites, chi 64, the library's Fresnel MPO at z = 2 mm, operator bond
    42) as one batch.  Two problems whose gradients once depended on their
    position in the batch (the forward then factored some bonds on the other
    Gram side than the adjoint, so the two disagreed on small-sigma kept
    directions) fill all 32 slots, 16 copies each, with the oracle's FP64
    mask cores; every slot's FP32 gradient matches the FP64 oracle gradient of
    its problem to 1e-3 relative L2, and the copies agree with each other to
    the same bar (measured 4e-5 against the oracle and 7e-6 between copies:
    the slots' eigensolvers start inverse iteration from different vectors,
    so FP32 rounding lands differently; the position-dependent failure it
    guards against was 1e4 to 1e9 times the gradient's norm)."""
    torch = need_gpu()
    api = _api()
    from paper_2510_23089_amd import autograd as AG
    n, z, chi, nb = 12, 2e-3, 64, 32
    say("phase retrieval 4096^2, batch of 32")
    prop = api.FresnelPropagator(n, LAM, DX, z)
    probs = (14, 24)
    masks, targets, refs = {}, {}, {}
    wx, wy = _mpos(n, z)
    for p in probs:
        ph = synth.smoothed_phase(1000 + p, 1 << n, 16.0, np.pi / 8)
        masks[p] = T.tt_svd(Q.to_quantics(np.exp(1j * ph)), 2 * n, chi, tau=1e-13)
        tph = synth.smoothed_phase(2000 + p, 1 << n, 16.0, np.pi / 2)
        tc = T.tt_svd(Q.to_quantics(np.exp(1j * tph)), 2 * n, chi, tau=1e-13)
        t1, _ = Z.mpo_apply(tc, wx, chi, tau=1e-13)
        t2, _ = Z.mpo_apply(t1, wy, chi, tau=1e-13)
        targets[p] = np.abs(Z.to_dense(t2, n)) ** 2
        refs[p] = OG.loss_and_grad(masks[p], wx, wy, targets[p], chi, n, tau=1e-13)
        say("  oracle problem %d done" % p)
    slot = [probs[(i // 2) % 2] if i not in probs else i for i in range(nb)]
    psi = api.MPSBatch(nb, 2 * n, chi)
    one = {p: api.MPS.from_host(masks[p], chi_cap=chi) for p in probs}
    for i, p in enumerate(slot):
        psi.fill_from(one[p], i)
    tg = torch.from_numpy(np.stack([targets[p] for p in slot])).float().cuda()
    pr = AG.PhaseRetrieval(api.MPOBatch([prop.wx] * nb), api.MPOBatch([prop.wy] * nb), chi)
    loss, g = pr.loss_and_grad(psi.cores, psi.bonds, tg)
    api.check_status()
    b = psi.bonds.cpu().numpy()
    gn = g.cpu().numpy()
    worst = {p: 0.0 for p in probs}
    spread = {p: 0.0 for p in probs}
    first = {}
    for i, p in enumerate(slot):
        got = [gn[i, k, :b[i, k], :, :b[i, k + 1]].astype(np.complex128) for k in range(2 * n)]
        worst[p] = max(worst[p], _rel_list(got, refs[p][1]))
        if p in first:
            spread[p] = max(spread[p], _rel_list(got, first[p]))
        else:
            first[p] = got
    say("  worst FP32 vs oracle over the slots: %s" % {p: "%.2e" % worst[p] for p in probs})
    say("  largest disagreement between copies: %s" % {p: "%.2e" % spread[p] for p in probs})
    for p in probs:
        assert worst[p] < 1e-3
        assert spread[p] < 1e-3
