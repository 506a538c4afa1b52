"""GPU unit tests of the two building blocks behind every step of the path:
the MFMA complex contraction (tt_cgemm) and the FP64 Hermitian eigensolver
with the keep rule (tt_heev).  References: numpy matmul / eigh in float64."""
import ctypes

import numpy as np
import pytest

from gpu_util import need_gpu, say, rel

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2510_23089_amd import _lib as L
    return L, L.load()


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 7), (64, 64, 16), (100, 37, 53), (130, 200, 70), (17, 300, 129)])
@pytest.mark.parametrize("conj", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_cgemm(prec, shape, conj):
    torch = need_gpu()
    L, lib = _lib()
    M, N, K = shape
    say("cgemm", prec, shape, conj)
    rng = np.random.default_rng(M * 1000 + N + K)
    a = rng.standard_normal((M, K + 3)) + 1j * rng.standard_normal((M, K + 3))
    b = rng.standard_normal((K, N + 2)) + 1j * rng.standard_normal((K, N + 2))
    dt = torch.complex64 if prec == "fp32" else torch.complex128
    da = torch.from_numpy(a).to(dt).cuda()
    db = torch.from_numpy(b).to(dt).cuda()
    dc = torch.zeros((M, N + 1), dtype=dt, device="cuda")
    code = L.PREC_FP32 if prec == "fp32" else L.PREC_FP64
    rc = lib.tt_cgemm(M, N, K, da.data_ptr(), K + 3, conj[0], db.data_ptr(), N + 2, conj[1], dc.data_ptr(), N + 1,
                      code, _stream(torch))
    L.check(rc, "tt_cgemm")
    torch.cuda.synchronize()
    aa = a[:, :K].conj() if conj[0] else a[:, :K]
    bb = b[:, :N].conj() if conj[1] else b[:, :N]
    if prec == "fp32":
        aa = aa.astype(np.complex64).astype(np.complex128)
        bb = bb.astype(np.complex64).astype(np.complex128)
    ref = aa @ bb
    got = dc.cpu().numpy()[:, :N]
    tol = 2e-6 if prec == "fp32" else 1e-13
    assert rel(got, ref) < tol


@pytest.mark.parametrize("shape", [(300, 260, 70), (129, 129, 33), (1000, 100, 300), (64, 513, 17)])
def test_cgemm_every_tile_variant_bit_identical(shape):
    """Every output-tile variant of the FP32 contraction (the two wide ones
    included), forced through the tuning table, gives the default variant's
    bits: the variants differ only in how the output is partitioned."""
    torch = need_gpu()
    L, lib = _lib()
    M, N, K = shape
    say("cgemm variants", shape)
    rng = np.random.default_rng(M + 7 * N + 13 * K)
    a = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    b = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    da = torch.from_numpy(a).to(torch.complex64).cuda()
    db = torch.from_numpy(b).to(torch.complex64).cuda()

    def run():
        dc = torch.zeros((M, N), dtype=torch.complex64, device="cuda")
        L.check(lib.tt_cgemm(M, N, K, da.data_ptr(), K, 0, db.data_ptr(), N, 0, dc.data_ptr(), N, L.PREC_FP32,
                             _stream(torch)), "tt_cgemm")
        torch.cuda.synchronize()
        return dc.cpu()

    from paper_2510_23089_amd import api
    L.check(lib.tt_autotune_clear(), "clear")
    base = run()
    ref = a.astype(np.complex64).astype(np.complex128) @ b.astype(np.complex64).astype(np.complex128)
    assert rel(base.numpy(), ref) < 2e-6
    assert api.autotune(run) >= 1
    table = api.autotune_table()
    assert all(e[0] == 0 and 0 <= e[5] < 5 for e in table)
    try:
        for v in range(5):
            L.check(lib.tt_autotune_clear(), "clear")
            api.autotune_load([list(e[:5]) + [v] for e in table])
            assert torch.equal(run(), base), v
    finally:
        L.check(lib.tt_autotune_clear(), "clear")


def _heev(torch, L, lib, mats, kcap, cutoff=0.0, tau=0.0):
    batch, n, _ = mats.shape
    g = torch.from_numpy(np.ascontiguousarray(mats)).to(torch.complex128).cuda()
    kept = torch.zeros(batch, dtype=torch.int32, device="cuda")
    ev = torch.zeros((batch, kcap), dtype=torch.float64, device="cuda")
    vec = torch.zeros((batch, n, kcap), dtype=torch.complex128, device="cuda")
    nb = lib.tt_heev_workspace_size(n, kcap, batch)
    ws = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    rc = lib.tt_heev(g.data_ptr(), n, batch, kcap, cutoff, tau, kept.data_ptr(), ev.data_ptr(), vec.data_ptr(),
                     ws.data_ptr(), nb, _stream(torch))
    L.check(rc, "tt_heev")
    torch.cuda.synchronize()
    st = int(ws[:4].view(torch.int32).cpu()[0])
    return kept.cpu().numpy(), ev.cpu().numpy(), vec.cpu().numpy(), st


def _rand_herm(rng, n, spectrum=None):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, _ = np.linalg.qr(x)
    if spectrum is None:
        spectrum = np.sort(rng.uniform(0.0, 1.0, n))[::-1]
    return (q * spectrum) @ q.conj().T


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 64, 100, 128, 129, 200, 256, 300, 512])
def test_heev_random(n):
    torch = need_gpu()
    L, lib = _lib()
    say("heev", n)
    rng = np.random.default_rng(n)
    # a Gram-like spectrum decaying over many decades, and a flat one
    specs = [np.sort(10.0 ** rng.uniform(-9, 2, n))[::-1], np.sort(rng.uniform(0.1, 1.0, n))[::-1]]
    mats = np.stack([_rand_herm(rng, n, s) for s in specs])
    kcap = max(1, min(n, 96))
    kept, ev, vec, st = _heev(torch, L, lib, mats, kcap)
    assert st == 0
    for b in range(2):
        w, v = np.linalg.eigh(mats[b])
        w = w[::-1]
        v = v[:, ::-1]
        k = int(kept[b])
        assert k == min(n, kcap)
        assert np.max(np.abs(ev[b, :k] - w[:k])) < 1e-12 * abs(w[0])
        u = vec[b, :, :k]
        # orthogonality, weighted by the singular values the vectors carry in a
        # truncation (sqrt of the eigenvalues), and unweighted at a looser bar
        e = np.abs(u.conj().T @ u - np.eye(k))
        wgt = np.sqrt(np.outer(ev[b, :k], ev[b, :k])) / abs(w[0])
        assert np.max(e * wgt) < 1e-12
        assert np.max(e) < 1e-6
        # eigen-equation residual
        res = mats[b] @ u - u * ev[b, :k]
        assert np.max(np.abs(res)) < 1e-10 * abs(w[0])


def _check_heev(mats, kept, ev, vec, kcap):
    for b in range(mats.shape[0]):
        w, v = np.linalg.eigh(mats[b])
        w = w[::-1]
        k = int(kept[b])
        assert k == min(mats.shape[1], kcap)
        assert np.max(np.abs(ev[b, :k] - w[:k])) < 1e-12 * abs(w[0])
        u = vec[b, :, :k]
        e = np.abs(u.conj().T @ u - np.eye(k))
        wgt = np.sqrt(np.outer(ev[b, :k], ev[b, :k])) / abs(w[0])
        assert np.max(e * wgt) < 1e-12
        assert np.max(np.abs(mats[b] @ u - u * ev[b, :k])) < 1e-10 * abs(w[0])


@pytest.mark.parametrize("n,batch", [(64, 2), (200, 2), (300, 2), (200, 40)])
def test_heev_reads_lower_triangle_only(n, batch):
    """Every reduction form (LDS n <= 128, multi-workgroup, and the streaming
    one that 40 matrices of n = 200 force: 40 x 7 workgroups exceed the
    chip) must reference only the lower triangle: garbage above the diagonal
    changes nothing."""
    torch = need_gpu()
    L, lib = _lib()
    say("heev lower", n, batch)
    rng = np.random.default_rng(1000 + n + batch)
    mats = np.stack([_rand_herm(rng, n, np.sort(10.0 ** rng.uniform(-6, 1, n))[::-1]) for _ in range(batch)])
    dirty = mats.copy()
    iu = np.triu_indices(n, 1)
    for b in range(batch):
        dirty[b][iu] = rng.standard_normal(len(iu[0])) * 1e3 + 1j * rng.standard_normal(len(iu[0]))
    kcap = min(n, 64)
    kept, ev, vec, st = _heev(torch, L, lib, dirty, kcap)
    assert st == 0
    _check_heev(mats, kept, ev, vec, kcap)


def test_heev_keep_rule_and_degenerate():
    torch = need_gpu()
    L, lib = _lib()
    rng = np.random.default_rng(7)
    n = 40
    spec = np.concatenate([[5.0, 3.0, 3.0, 3.0, 1.0], 1e-16 * np.ones(n - 5)])
    spec2 = np.concatenate([[8.0, 4.0, 2.0, 1.0], np.zeros(n - 4)])
    mats = np.stack([_rand_herm(rng, n, spec), _rand_herm(rng, n, spec2), np.zeros((n, n)), np.eye(n)])
    kept, ev, vec, st = _heev(torch, L, lib, mats, 10)
    assert st == 0
    assert kept[0] == 5                 # tau drops the 1e-16 tail
    assert kept[1] == 4
    assert kept[2] == 1                 # zero matrix keeps one
    assert kept[3] == 10                # identity: capped, degenerate cluster
    u = vec[0, :, :5]
    assert np.max(np.abs(u.conj().T @ u - np.eye(5))) < 1e-9
    assert np.max(np.abs(mats[0] @ u - u * ev[0, :5])) < 1e-10
    u = vec[3, :, :10]
    assert np.max(np.abs(u.conj().T @ u - np.eye(10))) < 1e-9
    # relative discarded-weight rule: total 15, tails 7, 3, 1, 0 (cutoffs kept
    # off the exact boundaries, which rounding of the trace decides)
    kept, ev, vec, st = _heev(torch, L, lib, mats[1:2].copy(), 10, cutoff=3.05 / 15.0)
    assert kept[0] == 2
    kept, ev, vec, st = _heev(torch, L, lib, mats[1:2].copy(), 10, cutoff=2.95 / 15.0)
    assert kept[0] == 3


def test_heev_nonfinite_flags_status():
    torch = need_gpu()
    L, lib = _lib()
    m = np.eye(8, dtype=np.complex128)
    m[3, 3] = np.nan
    kept, ev, vec, st = _heev(torch, L, lib, m[None], 4)
    assert st == -7


@pytest.mark.parametrize("n,kcap", [(200, 160), (256, 200)])
def test_heev_degenerate_runs_across_bitmask_words(n, kcap):
    """Clusters of exactly equal eigenvalues found from the joined-neighbour
    bitmask (one 64-bit word per 64 eigenvalues): a run straddling indices
    63/64, a run starting inside the second word, a run after index 128 and
    one straddling 127/128, with singletons between them.  Every kept vector
    is orthonormal to 1e-12 and satisfies the eigen-equation to 1e-10 ||G||,
    and each run's vectors span that eigenvalue's eigenspace."""
    torch = need_gpu()
    L, lib = _lib()
    say("heev degenerate runs", n, kcap)
    rng = np.random.default_rng(31 + n)
    spec = list(np.linspace(10.0, 6.0, 60))            # singletons 0..59
    spec += [5.0] * 8                                  # run 60..67 across the 63/64 boundary
    spec += list(np.linspace(4.9, 4.0, 10))            # singletons 68..77
    spec += [3.5] * 5                                  # run 78..82 inside word 1
    spec += list(np.linspace(3.4, 2.5, 43))            # singletons 83..125
    spec += [2.0] * 4                                  # run 126..129 across 127/128
    spec += list(np.linspace(1.9, 1.5, 6))             # singletons 130..135
    spec += [1.0] * 7                                  # run 136..142 after 128
    spec += list(np.linspace(0.9, 0.1, n - len(spec)))
    spec = np.array(spec[:n])
    assert np.all(np.diff(spec) <= 0)
    mats = _rand_herm(rng, n, spec)[None]
    kept, ev, vec, st = _heev(torch, L, lib, mats, kcap)
    assert st == 0
    k = int(kept[0])
    assert k == kcap
    assert np.max(np.abs(ev[0, :k] - spec[:k])) < 1e-12 * spec[0]
    u = vec[0, :, :k]
    assert np.max(np.abs(u.conj().T @ u - np.eye(k))) < 1e-12
    assert np.max(np.abs(mats[0] @ u - u * ev[0, :k])) < 1e-10 * spec[0]
    w, v = np.linalg.eigh(mats[0])
    w, v = w[::-1], v[:, ::-1]
    for a, b in ((60, 68), (78, 83), (126, 130), (136, 143)):
        if b > k:
            continue
        # projector onto the exact eigenspace equals the projector onto the kept run
        pe = v[:, a:b] @ v[:, a:b].conj().T
        pk = u[:, a:b] @ u[:, a:b].conj().T
        assert np.max(np.abs(pe - pk)) < 1e-10, (a, b)
