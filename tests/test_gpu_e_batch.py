"""Uneven batches (fields of different side and bond cap, one lockstep pass)
and HIP-graph replay of the whole pipeline.

Parity: every member of a padded batch equals the oracle's zip-up + sweep on
the member's own grid with the same (oracle-built) MPO cores, to the FP32 bar
1e-4 (truncated) / 1e-5 (lossless, against the dense FFT).  Graph replays are
compared with the eager result after eager work in between (several replays).
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say, rel
from oracle import fresnel as F
from oracle import mpo as OM
from oracle import quantics as Q
from oracle import ttsvd as T
from oracle import zipup as Z
import synth

pytestmark = pytest.mark.gpu
LAM, DX = 500e-9, 1e-6


def _ident(d):
    return np.einsum("ab,ts->atsb", np.eye(d), np.eye(2)).astype(np.complex128)


def _oracle_padded(k, K, z):
    """Oracle-built axis MPOs of a 2^k field padded into a 2^K batch."""
    c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << k, LAM, DX, z), k)
    pad = [_ident(1)] * (2 * (K - k))
    return pad + OM.embed_axis(c, "x"), pad + OM.embed_axis(c, "y"), c


def _run_batch(api, torch, fields, ks, chis, z, prec="fp32", refine=False):
    K = max(ks)
    count = len(ks)
    mx, my = [], []
    for k in ks:
        wx, wy, _ = _oracle_padded(k, K, z)
        mx.append(wx)
        my.append(wy)
    Wx, Wy = api.MPOBatch(mx), api.MPOBatch(my)
    side = 1 << K
    img = torch.zeros((count, side, side), dtype=torch.complex64, device="cuda")
    for i, f in enumerate(fields):
        n = f.shape[0]
        img[i, :n, :n] = torch.from_numpy(f).to(torch.complex64)
    chi = max(chis)
    chi_dev = torch.tensor(chis, dtype=torch.int32, device="cuda")
    psi = api.tt_encode_batched(img, chi, chi_dev=chi_dev)
    mid = api.mpo_apply_batched(psi, Wx, chi, chi_dev=chi_dev, prec=prec, refine=refine)
    out = api.mpo_apply_batched(mid, Wy, chi, chi_dev=chi_dev, prec=prec, refine=refine)
    dense = api.tt_to_dense_batched(out)
    api.check_status()
    return psi, out, dense


def test_uneven_batch_vs_oracle_per_field():
    torch = need_gpu()
    from paper_2510_23089_amd import api
    ks = [3, 5, 4, 5, 3, 4]
    chis = [4, 16, 8, 6, 8, 16]
    z = 20e-6
    fields = [synth.aperture_field(10 + i, n=1 << k) for i, k in enumerate(ks)]
    psi, out, dense = _run_batch(api, torch, fields, ks, chis, z)
    K = max(ks)
    for i, (k, chi, f) in enumerate(zip(ks, chis, fields)):
        say("member", i, k, chi)
        cores = T.tt_svd(Q.to_quantics(f), 2 * k, chi, tau=1e-13)
        _, _, c = _oracle_padded(k, K, z)
        wx, wy = OM.embed_axis(c, "x"), OM.embed_axis(c, "y")
        r1, _ = Z.mpo_apply(cores, wx, chi, tau=1e-13)
        r2, _ = Z.mpo_apply(r1, wy, chi, tau=1e-13)
        ref = Z.to_dense(r2, k)
        n = 1 << k
        got = dense[i].cpu().numpy()
        assert rel(got[:n, :n], ref) < 1e-4
        if n < got.shape[0]:
            assert np.abs(got[n:, :]).max() == 0 and np.abs(got[:, n:]).max() == 0
        # the padded sites stay bond 1
        b = [int(x) for x in out.bonds[i].cpu()]
        assert b[:2 * (K - k) + 1] == [1] * (2 * (K - k) + 1)
        assert b[2 * (K - k):] == T.bonds(r2)


def test_uneven_batch_lossless_vs_fft():
    torch = need_gpu()
    from paper_2510_23089_amd import api
    # caps at least the largest zip-up bond a 2k-site member can need
    # (left of the centre the zip-up state is not yet in Schmidt form)
    ks = [2, 4, 3, 4]
    chis = [8, 64, 32, 64]
    z = 10e-6
    fields = [synth.random_field(20 + i, 1 << k) for i, k in enumerate(ks)]
    _, _, dense = _run_batch(api, torch, fields, ks, chis, z)
    for i, (k, f) in enumerate(zip(ks, fields)):
        n = 1 << k
        ref = F.fresnel_dense(f, LAM, DX, z)
        assert rel(dense[i, :n, :n].cpu().numpy(), ref) < 1e-5


@pytest.mark.parametrize("prec,refine", [("fp32", False), ("bf16x3", True)])
def test_graph_replay_matches_eager(prec, refine):
    torch = need_gpu()
    from paper_2510_23089_amd import batch as BT
    ks = [4, 6, 5, 6, 4]
    chis = [8, 32, 16, 12, 16]
    z = 50e-6
    b = BT.UnevenBatch(ks, chis, LAM, DX, z, prec=prec, refine=refine)
    fields = [synth.aperture_field(30 + i, n=1 << k) for i, k in enumerate(ks)]
    b.load(fields)
    eager = b.run().clone()
    from paper_2510_23089_amd import api
    api.check_status()
    b.capture()
    for rep in range(3):
        say("replay", rep)
        out = b.replay().clone()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        # eager work between replays, then replay again
        junk = b.run().clone()
        torch.cuda.synchronize()
        assert torch.equal(junk, eager)
    # new inputs through the same graph
    fields2 = [synth.aperture_field(40 + i, n=1 << k) for i, k in enumerate(ks)]
    b.load(fields2)
    g2 = b.replay().clone()
    e2 = b.run().clone()
    torch.cuda.synchronize()
    assert torch.equal(g2, e2)
    api.check_status()


def test_autotune_keeps_results_bit_identical():
    torch = need_gpu()
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import batch as BT
    from paper_2510_23089_amd import _lib as L
    lib = L.load()
    L.check(lib.tt_autotune_clear(), "clear")
    ks = [4, 6, 5]
    chis = [8, 32, 16]
    b = BT.UnevenBatch(ks, chis, LAM, DX, 50e-6, prec="bf16x3", refine=True)
    b.load([synth.aperture_field(50 + i, n=1 << k) for i, k in enumerate(ks)])
    before = b.run().clone()
    n = b.tune()
    assert n > 0
    table = api.autotune_table()
    # FP32 products have five tile variants, the other forms three
    assert len(table) == n and all(0 <= e[5] < (5 if e[0] == 0 else 3) for e in table)
    after = b.run().clone()
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    # export / import round trip
    L.check(lib.tt_autotune_clear(), "clear")
    assert api.autotune_table() == []
    api.autotune_load(table)
    assert sorted(api.autotune_table()) == sorted(table)
    b.capture()
    assert torch.equal(b.replay().clone(), before)
    api.check_status()


def test_every_contraction_variant_gives_the_same_propagation():
    """An FP32 encode, batched propagation (both axes) and decompression with
    every recorded contraction shape forced to each tile variant in turn (the
    wide FP32 tiles and the k-major operand forms included; the FP64-
    accumulated Gram shapes cycle through their three) reproduces the default
    run's bits: the variants only partition the outputs differently."""
    torch = need_gpu()
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import _lib as L
    lib = L.load()
    n, chi = 9, 48
    zs = (0.5e-3, 2e-3)
    m = 2 * n
    d = torch.from_numpy(synth.aperture_field(71, n=1 << n)).to(torch.complex64).cuda()
    prop = api.FresnelBatch(n, LAM, DX, zs, device="cuda")
    bi = api.MPSBatch(len(zs), m, chi)
    mid = api.MPSBatch(len(zs), m, chi)
    out = api.MPSBatch(len(zs), m, chi)

    def run():
        psi = api.tt_encode(d, chi)
        bi.fill_from(psi)
        prop(bi, chi, tmp=mid, out=out)
        dens = api.tt_to_dense_batched(out)
        torch.cuda.synchronize()
        return dens.clone(), out.bonds.clone()

    L.check(lib.tt_autotune_clear(), "clear")
    try:
        base, bonds = run()
        api.check_status()
        assert api.autotune(run) > 0
        table = api.autotune_table()
        assert any(e[0] == 0 for e in table) and any(e[0] != 0 for e in table)
        for v in range(5):
            say("forced variant", v)
            L.check(lib.tt_autotune_clear(), "clear")
            api.autotune_load([list(e[:5]) + [v if e[0] == 0 else v % 3] for e in table])
            got, gb = run()
            assert torch.equal(gb, bonds), v
            assert torch.equal(got, base), v
        api.check_status()
    finally:
        L.check(lib.tt_autotune_clear(), "clear")


def test_native_group_encode_matches_padded_encode():
    """UnevenBatch encodes each side on its own grid and puts 2(K - k) leading
    |0> sites in front; the result must be the encode of the zero-padded
    image (same bonds everywhere, same fields after propagation), and the
    padding of the decompressed members must stay exactly zero."""
    torch = need_gpu()
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import batch as BT
    ks = [3, 5, 4, 5, 3, 4, 2]
    chis = [4, 16, 8, 6, 8, 16, 4]
    z = 20e-6
    fields = [synth.aperture_field(70 + i, n=1 << k) for i, k in enumerate(ks)]
    b = BT.UnevenBatch(ks, chis, LAM, DX, z)
    b.load(fields)
    got = b.run().clone()
    api.check_status()
    # the padded-image pipeline through the same MPOs
    K = max(ks)
    side = 1 << K
    img = torch.zeros((len(ks), side, side), dtype=torch.complex64, device="cuda")
    for i, f in enumerate(fields):
        n = f.shape[0]
        img[i, :n, :n] = torch.from_numpy(f).to(torch.complex64)
    chi_dev = torch.tensor(chis, dtype=torch.int32, device="cuda")
    psi = api.tt_encode_batched(img, max(chis), chi_dev=chi_dev)
    assert torch.equal(psi.bonds, b.psi.bonds)
    mid = api.mpo_apply_batched(psi, b.wx, max(chis), chi_dev=chi_dev)
    out = api.mpo_apply_batched(mid, b.wy, max(chis), chi_dev=chi_dev)
    ref = api.tt_to_dense_batched(out)
    api.check_status()
    assert torch.equal(out.bonds, b.out.bonds)
    for i, k in enumerate(ks):
        n = 1 << k
        say("member", i, k)
        assert rel(got[i, :n, :n].cpu().numpy(), ref[i, :n, :n].cpu().numpy()) < 1e-5
        if n < side:
            assert got[i, n:, :].abs().max().item() == 0 and got[i, :, n:].abs().max().item() == 0


def test_uneven_batch_full_size_members_vs_oracle():
    """Members at the sizes of the 256-field batch's extremes, through the
    padded pipeline with the oracle's MPOs (z = 2 mm): a 2048^2 field at chi
    128 (22 sites) and a 256^2 field at chi 16 padded into it, each against the
    oracle's TT-SVD, zip-up and sweep on its own grid (FP32 bar 1e-4 against
    the identically truncated result, equal bonds, zero padding outside)."""
    torch = need_gpu()
    from paper_2510_23089_amd import api
    ks = [11, 8]
    chis = [128, 16]
    z = 2e-3
    fields = [synth.aperture_field(40 + i, n=1 << k) for i, k in enumerate(ks)]
    say("full-size uneven members", ks, chis)
    psi, out, dense = _run_batch(api, torch, fields, ks, chis, z)
    K = max(ks)
    for i, (k, chi, f) in enumerate(zip(ks, chis, fields)):
        cores = T.tt_svd(Q.to_quantics(f), 2 * k, chi, tau=1e-13)
        _, _, c = _oracle_padded(k, K, z)
        wx, wy = OM.embed_axis(c, "x"), OM.embed_axis(c, "y")
        r1, _ = Z.mpo_apply(cores, wx, chi, tau=1e-13)
        r2, _ = Z.mpo_apply(r1, wy, chi, tau=1e-13)
        ref = Z.to_dense(r2, k)
        n = 1 << k
        got = dense[i].cpu().numpy()
        err = rel(got[:n, :n], ref)
        say("  member %d (2^%d, chi %d): rel err %.3e" % (i, k, chi, err))
        assert err < 1e-4
        assert [int(x) for x in out.bonds[i].cpu()][2 * (K - k):] == Z.bonds(r2)
        if n < got.shape[0]:
            assert np.abs(got[n:, :]).max() == 0 and np.abs(got[:, n:]).max() == 0


def test_grouped_batch_vs_oracle_padded_batch_and_graph():
    """The unpadded form (one lockstep batch per side, each on its own
    stream): every member equals the oracle's zip-up + sweep on its own grid
    (FP32 bar 1e-4, equal bonds), agrees with the padded batch to FP32
    rounding (the K-split of the Gram products follows the batch width, so
    the sums may associate differently), and graph replays equal eager runs
    bit for bit, with eager work in between."""
    torch = need_gpu()
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import batch as BT
    ks = [3, 5, 4, 5, 3, 4, 5]
    chis = [4, 16, 8, 6, 8, 16, 12]
    z = 20e-6
    fields = [synth.aperture_field(10 + i, n=1 << k) for i, k in enumerate(ks)]
    gb = BT.GroupedBatch(ks, chis, LAM, DX, z)
    gb.load(fields)
    gb.run()
    torch.cuda.synchronize()
    gb.check_status()
    pb = BT.UnevenBatch(ks, chis, LAM, DX, z)
    pb.load(fields)
    pb.run()
    api.check_status()
    from paper_2510_23089_amd import mpo_build as B
    for i, (k, chi, f) in enumerate(zip(ks, chis, fields)):
        cores = T.tt_svd(Q.to_quantics(f), 2 * k, chi, tau=1e-13)
        c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << k, LAM, DX, z), k)
        r1, _ = Z.mpo_apply(cores, OM.embed_axis(c, "x"), chi, tau=1e-13)
        r2, _ = Z.mpo_apply(r1, OM.embed_axis(c, "y"), chi, tau=1e-13)
        got = gb.field(i).cpu().numpy()
        e = rel(got, Z.to_dense(r2, k))
        e_pad = rel(got, pb.field(i).cpu().numpy())
        say("member %d (2^%d, chi %d): vs oracle %.2e, vs padded batch %.2e" % (i, k, chi, e, e_pad))
        assert e < 1e-4
        assert e_pad < 1e-5
        assert [int(x) for x in gb.bonds(i).cpu()] == T.bonds(r2)
    eager = [d.clone() for d in gb.run()]
    torch.cuda.synchronize()
    gb.capture()
    for rep in range(3):
        gb.replay()
        torch.cuda.synchronize()
        for g, d in zip(gb.groups, eager):
            assert torch.equal(g["dense"], d), rep
        junk = gb.run()
        torch.cuda.synchronize()
        for a, d in zip(junk, eager):
            assert torch.equal(a, d)
    gb.check_status()
