"""Batches of fields of uneven size and bond cap in one lockstep pass.

A field of side 2^k inside a batch of side 2^K (k <= K) is stored
zero-padded in the top-left 2^k x 2^k block of the 2^K grid.  In quantics
order (most significant bit first) its first 2(K - k) sites are then the
state |0> with bond 1, and its propagator is the Fresnel MPO of its own
2^k grid (periodic on that grid) on the remaining sites with identity
(pass-through) cores on the padded ones: every member is processed exactly
as it would be alone, while all members advance site by site together.  Per
field bond caps go to the device as one int per field.

Members are encoded on their own grids, one batched encode per distinct
side (the padded image would only feed zeros to the leading Gram products),
and placed behind 2(K - k) leading cores |0> of bond 1 -- the state the
encode of the padded image produces there, up to a phase per core.

The whole pipeline (encode, x then y application, optional refinement, and
decompression) is a fixed sequence of stream-ordered library calls with no
host synchronisation, so it can be captured once in a HIP graph and replayed.
"""
import numpy as np
import torch

from . import api
from . import mpo_build as B


def padded_axis_mpos(k, K, lam, dx, z, rel=1e-12):
    """(x cores, x kinds, y cores, y kinds) of a 2^k field in a 2^K batch."""
    w1 = B.fresnel_axis(k, lam, dx, z, rel)
    pad = [B.identity_core(1)] * (2 * (K - k))
    cx, kx = B.embed(w1, "x")
    cy, ky = B.embed(w1, "y")
    return (pad + cx, [1] * len(pad) + kx, pad + cy, [1] * len(pad) + ky)


class UnevenBatch:
    """Encode + propagate (x then y) + decompress a batch of square fields of
    sides 2^ks[i] with bond caps chis[i], all at distance z."""

    def __init__(self, ks, chis, lam, dx, z, device="cuda", prec="fp32", refine=False, rel=1e-12):
        self.ks = [int(k) for k in ks]
        self.chis = [int(c) for c in chis]
        self.count = len(self.ks)
        self.K = max(self.ks)
        self.m = 2 * self.K
        self.chi = max(self.chis)
        self.prec, self.refine = prec, refine
        self.device = torch.device(device)
        per_k = {}
        for k in sorted(set(self.ks)):
            cx, kx, cy, ky = padded_axis_mpos(k, self.K, lam, dx, z, rel)
            per_k[k] = (api.MPO(cx, kx, dtype=torch.complex64, device="cpu"),
                        api.MPO(cy, ky, dtype=torch.complex64, device="cpu"))
        self.wx = api.MPOBatch([per_k[k][0] for k in self.ks], device=device)
        self.wy = api.MPOBatch([per_k[k][1] for k in self.ks], device=device)
        self.chi_dev = torch.tensor(self.chis, dtype=torch.int32, device=device)
        side = 1 << self.K
        self.psi = api.MPSBatch(self.count, self.m, self.chi, device=device)
        # one group per distinct side: member indices, native images, its encode
        self.groups = []
        for k in sorted(set(self.ks)):
            idx = [i for i, kk in enumerate(self.ks) if kk == k]
            n = 1 << k
            imgs = torch.zeros((len(idx), n, n), dtype=torch.complex64, device=device)
            enc = api.MPSBatch(len(idx), 2 * k, self.chi, device=device)
            chis = torch.tensor([self.chis[i] for i in idx], dtype=torch.int32, device=device)
            self.groups.append((k, idx, torch.tensor(idx, dtype=torch.long, device=device), imgs, enc, chis))
            p = 2 * (self.K - k)
            if p:
                lead = torch.zeros((p, self.chi, 2, self.chi), dtype=torch.complex64, device=device)
                lead[:, 0, 0, 0] = 1.0          # |0>, bond 1 (never rewritten by run())
                self.psi.cores[idx, :p] = lead
        self.mid = api.MPSBatch(self.count, self.m, self.chi, device=device)
        self.out = api.MPSBatch(self.count, self.m, self.chi, device=device)
        self.dense = torch.empty((self.count, side, side), dtype=torch.complex64, device=device)
        self.graph = None

    def load(self, fields):
        """Copy host fields (list of 2^k x 2^k arrays) into the device batch."""
        for k, idx, _, imgs, _, _ in self.groups:
            for j, i in enumerate(idx):
                f = np.asarray(fields[i])
                assert f.shape[0] == 1 << k
                imgs[j].copy_(torch.from_numpy(f).to(torch.complex64))

    def encode(self):
        """Encode every group on its own grid and place it behind its leading sites."""
        for k, _, idx_dev, imgs, enc, chis in self.groups:
            api.tt_encode_batched(imgs, self.chi, out=enc, chi_dev=chis)
            p = 2 * (self.K - k)
            self.psi.cores[:, p:].index_copy_(0, idx_dev, enc.cores)
            self.psi.bonds[:, p:].index_copy_(0, idx_dev, enc.bonds)
            self.psi.norms.index_copy_(0, idx_dev, enc.norms)
        return self.psi

    def run(self):
        """The pipeline on the current stream (capturable)."""
        self.encode()
        api.mpo_apply_batched(self.psi, self.wx, self.chi, out=self.mid, chi_dev=self.chi_dev, prec=self.prec,
                              refine=self.refine)
        api.mpo_apply_batched(self.mid, self.wy, self.chi, out=self.out, chi_dev=self.chi_dev, prec=self.prec,
                              refine=self.refine)
        api.tt_to_dense_batched(self.out, out=self.dense)
        return self.dense

    def tune(self, path=None):
        """Autotune the contraction tiles on this batch's call shapes (before capture)."""
        return api.autotune(self.run, device=self.device, path=path)

    def capture(self):
        """Record run() in a HIP graph (after one eager run that sizes every
        workspace), then replay() re-issues the whole batch in one launch."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        torch.cuda.synchronize(self.device)
        # the graph records raw workspace addresses: hold the buffers it uses
        self._held = list(api._WS_CACHE.values())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.dense

    def field(self, i):
        """Dense result of member i on its own 2^k grid (device view)."""
        n = 1 << self.ks[i]
        return self.dense[i, :n, :n]


class GroupedBatch:
    """The same uneven batch without padding: one lockstep batch per distinct
    side 2^k, on its own 2k sites with the Fresnel MPO of its own grid, each
    group on a stream of its own (forked from the calling stream and joined
    back to it), so the groups' chains run concurrently and a captured graph
    holds them as parallel branches of one launch.  Each group has its own
    workspaces and status words (keys "grp<k>-enc", "grp<k>-apply",
    "grp<k>-dense")."""

    def __init__(self, ks, chis, lam, dx, z, device="cuda", prec="fp32", refine=False, rel=1e-12):
        self.ks = [int(k) for k in ks]
        self.chis = [int(c) for c in chis]
        self.count = len(self.ks)
        self.prec, self.refine = prec, refine
        self.device = torch.device(device)
        self.where = [None] * self.count          # member -> (group, position)
        self.groups = []
        for k in sorted(set(self.ks)):
            idx = [i for i, kk in enumerate(self.ks) if kk == k]
            for j, i in enumerate(idx):
                self.where[i] = (len(self.groups), j)
            n, cnt = 1 << k, len(idx)
            chi = max(self.chis[i] for i in idx)
            w1 = B.fresnel_axis(k, lam, dx, z, rel)
            cx, kx = B.embed(w1, "x")
            cy, ky = B.embed(w1, "y")
            wx = api.MPO(cx, kx, dtype=torch.complex64, device="cpu")
            wy = api.MPO(cy, ky, dtype=torch.complex64, device="cpu")
            g = {
                "k": k, "idx": idx, "chi": chi,
                "chi_dev": torch.tensor([self.chis[i] for i in idx], dtype=torch.int32, device=device),
                "imgs": torch.zeros((cnt, n, n), dtype=torch.complex64, device=device),
                "wx": api.MPOBatch([wx] * cnt, device=device),
                "wy": api.MPOBatch([wy] * cnt, device=device),
                "psi": api.MPSBatch(cnt, 2 * k, chi, device=device),
                "mid": api.MPSBatch(cnt, 2 * k, chi, device=device),
                "out": api.MPSBatch(cnt, 2 * k, chi, device=device),
                "dense": torch.empty((cnt, n, n), dtype=torch.complex64, device=device),
                "stream": torch.cuda.Stream(device=self.device),
                "key": "grp%d" % k,
            }
            self.groups.append(g)
        self.graph = None

    def load(self, fields):
        """Copy host fields (list of 2^k x 2^k arrays) into the device groups."""
        for g in self.groups:
            for j, i in enumerate(g["idx"]):
                f = np.asarray(fields[i])
                assert f.shape[0] == 1 << g["k"]
                g["imgs"][j].copy_(torch.from_numpy(f).to(torch.complex64))

    def run(self):
        """The pipeline, forked over the groups' streams and joined back to
        the current stream (capturable)."""
        cur = torch.cuda.current_stream(self.device)
        for g in self.groups:
            g["stream"].wait_stream(cur)
        for g in self.groups:
            with torch.cuda.stream(g["stream"]):
                key = g["key"]
                api.tt_encode_batched(g["imgs"], g["chi"], out=g["psi"], chi_dev=g["chi_dev"], ws_key=key + "-enc")
                api.mpo_apply_batched(g["psi"], g["wx"], g["chi"], out=g["mid"], chi_dev=g["chi_dev"],
                                      prec=self.prec, refine=self.refine, ws_key=key + "-apply")
                api.mpo_apply_batched(g["mid"], g["wy"], g["chi"], out=g["out"], chi_dev=g["chi_dev"],
                                      prec=self.prec, refine=self.refine, ws_key=key + "-apply")
                api.tt_to_dense_batched(g["out"], out=g["dense"], ws_key=key + "-dense")
        for g in self.groups:
            cur.wait_stream(g["stream"])
        return [g["dense"] for g in self.groups]

    def check_status(self):
        for g in self.groups:
            for part in ("-enc", "-apply", "-dense"):
                api.check_status(key=g["key"] + part)

    def tune(self, path=None):
        """Autotune the contraction tiles on this batch's call shapes (before capture)."""
        return api.autotune(self.run, device=self.device, path=path)

    def capture(self):
        """Record run() in a HIP graph after one eager run that sizes every
        workspace; replay() then re-issues every group's chain in one launch."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        torch.cuda.synchronize(self.device)
        self._held = list(api._WS_CACHE.values())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def field(self, i):
        """Dense result of member i on its own 2^k grid (device view)."""
        gi, j = self.where[i]
        return self.groups[gi]["dense"][j]

    def bonds(self, i):
        gi, j = self.where[i]
        return self.groups[gi]["out"].bonds[j]
