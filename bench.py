"""Benchmark: MPO x MPS Fresnel propagations per second at 2^20 px, chi = 128.

Workload (one step): B (--fields-per-step, default 5) seeded 1024 x 1024
complex64 fields (disk aperture of radius 300 px, 1/f^2-power amplitude
modulation, smoothed random phase; seeds 0..B-1) are encoded into 20-site
quantics MPS (chi 128) by one batched encode; the Fresnel MPO (lambda 500 nm,
pixel 1 um) propagates each to z = 0.5, 2 and 8 mm -- each propagation is a
zip-up + truncation sweep for the x axis then the y axis at chi 128, the 3B
(field, distance) members advancing as one batch -- and every result is
decompressed to the 1024 x 1024 grid.  value = propagations / s over whole
steps (encode and decompression included).  A step is a chain of ~95
dependent truncations, each an FP64 eigensolve of one small matrix per
member, so independent steps also run concurrently: step k on stream k mod
S (S = --inflight, default 2: the main stream and one more), each stream
with its own buffers and library workspaces.  The multi-workgroup reduction
of the 256-wide zip-up Gram matrices needs its 8 workgroups per matrix
resident together, so 3 B x 8 x S must stay within the 256 compute units
(B S <= 10; its waits are bounded, so an oversubscribed schedule reports an
error instead of hanging).  Nothing else runs inside the timed region.  serial_ms_per_step: one field's step (its three distances as
one batch) timed alone on one stream, i.e. the latency of a single field.
Inputs are resident in HBM before the timed region; the host float64 MPO
construction is setup.

The dominant kernel (qtt::tridiag_lds_kernel, the Householder
tridiagonalisation of the FP64 Gram matrices up to 128 and of the trailing
128 x 128 block of wider ones, one workgroup per matrix with the packed
triangle in LDS) is timed in a pass of its own right after the timed region
(same steps, same lanes), with HIP events around each of its launches on
their streams, and reports the algorithmic FP64 work (16/3) n^3 of each
launch from the matrix or block sizes the kernel logs on the device; its
time per step and share of a step come from a serial pass.

parts: a single field's step split into its parts, timed on their own after
the timed region on one stream: the propagations alone (its three distances
from inputs already encoded: a propagation is the x and y applications), the
encode and the decompression.

cpu_baseline: the float64 oracle (numpy/LAPACK) on the host, on a bounded
sample of the same workload: one propagation (x then y) of the first field
at z = 2 mm, median of three runs (its encode reported beside it).

batched (the uneven-batch precision form): 256 fields with side 2^k, k
uniform in {8..11}, and bond caps uniform in {16, 32, 64, 128} (seeded draws),
aperture fields of the same recipe; zero-padded into one 2048^2 batch, encoded,
propagated (x then y, z = 2 mm) and decompressed in one HIP-graph replay,
with split-bfloat16 contractions and the full-precision fitting sweep; beside
it the same with plain bfloat16 contractions and the fitting sweep, the same
batch with plain FP32 contractions and sweep, the same FP32 work without
padding (one lockstep batch per side on its own stream, the four chains as
parallel branches of one graph), and a per-field FP32 baseline (fields
processed one at a time) on a sample of the batch.

grad_step (second headline number, phase retrieval): 32 independent 4096^2
problems (24 sites), a learnable phase mask exp(i phi) (phi: iid N(0,1)
smoothed by a periodic Gaussian of 16 px, std pi/8) encoded at chi 64, the
Fresnel MPO at z = 2 mm (x then y, chi 64), decompression and the summed
squared intensity error against targets made the same way (std pi/2); one
step = forward with saved state + loss + the full adjoint back to the mask
cores, all 32 problems as one batch.

large_field (a field too large to densify): the 16384^2 Gaussian beam (waist
2000 px) times a binary grating (period 64 px), 28 sites, encoded from its two
1-D factors at chi 256, the eight log-spaced distances 0.1 .. 10 mm propagated
as one batch (x then y to chi 256) and 1e5 sampled pixels read per distance.

Prints ONE JSON line (N = 1 only).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LAM, DX = 500e-9, 1e-6
ZS = (0.5e-3, 2e-3, 8e-3)
N_LOG2 = 10
CHI = 128
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector = matrix)
# Memory traffic of the dominant kernel per launch, from two rocprofv3 counter
# passes (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000 after calibration on a plain
# copy); valid only while the kernel's sources (see _kernel_source_hash) are
# the ones the counters were taken on, and for the schedule they were taken in
# (a launch holds one matrix per (field, z) member of a step).
TRAFFIC = {"src_sha256_prefix": "ac66566e2bff046f", "fields_per_step": 5,
           "bytes_per_launch": (369.345 * 2.0 + 618.611) * 1024.0}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=24)
    p.add_argument("--warmup", type=int, default=2, help="warm-up steps per lane")
    p.add_argument("--fields-per-step", type=int, default=5,
                   help="independent 1024^2 fields per step, each propagated to the three distances as one batch")
    p.add_argument("--serial-steps", type=int, default=8)
    p.add_argument("--no-parts", action="store_true")
    p.add_argument("--chi", type=int, default=CHI)
    p.add_argument("--inflight", type=int, default=2,
                   help="independent steps executing concurrently, one stream each: the main stream and "
                        "inflight - 1 more (at most 4: the HIP runtime's default of four hardware queues)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-grad", action="store_true")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--copy-probe", type=int, default=0,
                   help="after the run, copy this many MiB device to device (calibrates HBM byte counters)")
    p.add_argument("--grad-steps", type=int, default=3)
    p.add_argument("--no-large", action="store_true")
    p.add_argument("--large-steps", type=int, default=2)
    return p.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(field, chi):
    """Oracle on host cores: encode + one propagation (x, y) at z = 2 mm."""
    from oracle import fresnel as F
    from oracle import mpo as OM
    from oracle import quantics as Q
    from oracle import ttsvd as T
    from oracle import zipup as Z
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads") or 0) for p in threadpool_info()) or None
    except Exception:
        pass
    c = OM.mpo_from_matrix(F.fresnel_matrix_1d(1 << N_LOG2, LAM, DX, 2e-3), N_LOG2)
    wx, wy = OM.embed_axis(c, "x"), OM.embed_axis(c, "y")
    t_enc, t_props = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        cores = T.tt_svd(Q.to_quantics(field), 2 * N_LOG2, chi)
        t1 = time.perf_counter()
        c1, _ = Z.mpo_apply(cores, wx, chi)
        Z.mpo_apply(c1, wy, chi)
        t2 = time.perf_counter()
        t_enc.append(t1 - t0)
        t_props.append(t2 - t1)
    t_prop = float(np.median(t_props))
    t_e = float(np.median(t_enc))
    return {
        "value": 1.0 / t_prop,
        "unit": "propagations/s",
        "cores": threads or os.cpu_count(),
        "kind": "oracle",
        "sample": "float64 numpy/LAPACK oracle on the host: one propagation (x then y, z=2 mm, chi %d) of "
                  "the first 1024^2 field, median of 3 runs (%.2f s); its encode (median %.2f s) is not in value"
                  % (chi, t_prop, t_e),
        "cpu": _cpu_model(),
    }


def batched_bench(dev, replays=3, sample=16):
    """256 uneven fields in one graph replay; per-field FP32 baseline on a sample."""
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import synth
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import batch as BT
    z = 2e-3
    specs = synth.batch_specs(0, 256, 8, 11, (16, 32, 64, 128))
    ks = [k for k, _, _ in specs]
    chis = [c for _, c, _ in specs]
    with ThreadPoolExecutor(16) as ex:
        fields = list(ex.map(lambda sp: synth.aperture_field(sp[2], n=1 << sp[0]).astype(np.complex64), specs))
    px = sum(4 ** k for k in ks)
    res = {"fields": len(ks), "pixels": px, "z_mm": 2.0, "sides": sorted(set(1 << k for k in ks)),
           "chis": sorted(set(chis))}

    def timed(run, reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            run()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    outs = {}
    for name, prec, refine in (("bf16x3_fit_graph", "bf16x3", True), ("bf16_fit_graph", "bf16", True),
                               ("fp32_graph", "fp32", False), ("fp32_grouped_graph", "fp32", False)):
        cls = BT.GroupedBatch if "grouped" in name else BT.UnevenBatch
        b = cls(ks, chis, LAM, DX, z, device=dev, prec=prec, refine=refine)
        b.load(fields)
        b.capture()
        ms_untuned = timed(b.replay, replays)
        n_tuned = b.tune()
        b.capture()
        ms = timed(b.replay, replays)
        if "grouped" in name:
            b.check_status()
        else:
            api.check_status()
        outs[name] = [b.field(i).clone() for i in range(sample)]
        res[name] = {"ms_per_batch": ms, "fields_per_s": len(ks) / (ms / 1e3),
                     "propagations_per_s": len(ks) / (ms / 1e3), "ms_per_batch_untuned": ms_untuned,
                     "tuned_shapes": n_tuned}
        del b
        api._WS_CACHE.clear()
        torch.cuda.empty_cache()
    # per-field FP32 baseline (one field at a time, each with its own MPO)
    props = {}
    tot = 0.0
    for i in range(sample):
        k, chi = ks[i], chis[i]
        if k not in props:
            props[k] = api.FresnelPropagator(k, LAM, DX, z, device=dev)
        img = torch.from_numpy(fields[i]).to(dev)

        def one():
            psi = api.tt_encode(img, chi)
            out = props[k](psi, chi)
            return api.tt_to_dense(out)
        one()
        tot += timed(one, 1)
        d = one()
        outs.setdefault("per_field", []).append(d.clone())
    api.check_status()
    px_s = sum(4 ** ks[i] for i in range(sample))
    res["per_field_fp32_sample"] = {"fields": sample, "ms_total": tot, "fields_per_s": sample / (tot / 1e3),
                                    "pixel_share_of_batch": px_s / px}
    # accuracy against the exact propagation (float64 FFT on the host; the
    # truncation to chi dominates both forms' error, and the two must agree)
    errs = {"bf16x3_fit_graph": [], "bf16_fit_graph": [], "fp32_graph": [], "fp32_grouped_graph": [],
            "per_field": []}
    for i in range(sample):
        n = 1 << ks[i]
        f = np.fft.fftfreq(n, d=DX)
        t = np.exp(-1j * np.pi * LAM * z * f * f)
        exact = np.fft.ifft2(np.fft.fft2(fields[i].astype(np.complex128)) * (t[:, None] * t[None, :]))
        nrm = np.linalg.norm(exact)
        for key in errs:
            errs[key].append(float(np.linalg.norm(outs[key][i].cpu().numpy() - exact) / nrm))
    res["error_vs_exact"] = {
        "sample": sample,
        "per_field_fp32": errs["per_field"],
        "max_abs_gap_bf16x3_fit_minus_per_field": max(abs(a - b) for a, b in zip(errs["bf16x3_fit_graph"],
                                                                              errs["per_field"])),
        "max_abs_gap_fp32_batched_minus_per_field": max(abs(a - b) for a, b in zip(errs["fp32_graph"],
                                                                                errs["per_field"])),
        "max_abs_gap_fp32_grouped_minus_per_field": max(abs(a - b) for a, b in zip(errs["fp32_grouped_graph"],
                                                                                errs["per_field"])),
        "mean_bf16x3_fit": float(np.mean(errs["bf16x3_fit_graph"])),
        "mean_bf16_fit": float(np.mean(errs["bf16_fit_graph"])),
        "max_abs_gap_bf16_fit_minus_per_field": max(abs(a - b) for a, b in zip(errs["bf16_fit_graph"],
                                                                            errs["per_field"])),
        "mean_per_field_fp32": float(np.mean(errs["per_field"])),
    }
    return res


def grad_step_bench(steps, dev):
    """Phase-retrieval gradient steps: 32 x 4096^2 problems, chi 64, z = 2 mm."""
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import synth
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import autograd as AG
    n, z, chi, nb = 12, 2e-3, 64, 32
    side = 1 << n
    with ThreadPoolExecutor(16) as ex:
        masks = list(ex.map(lambda sd: synth.smoothed_phase(1000 + sd, side, 16.0, np.pi / 8).astype(np.float32),
                            range(nb)))
        tgts = list(ex.map(lambda sd: synth.smoothed_phase(2000 + sd, side, 16.0, np.pi / 2).astype(np.float32),
                           range(nb)))
    prop = api.FresnelPropagator(n, LAM, DX, z, device=dev)
    wx = api.MPOBatch([prop.wx] * nb, device=dev)
    wy = api.MPOBatch([prop.wy] * nb, device=dev)
    ph = torch.from_numpy(np.stack(masks)).to(dev)
    del masks
    mask = api.tt_encode_batched(torch.polar(torch.ones_like(ph), ph), chi)
    ph.copy_(torch.from_numpy(np.stack(tgts)))
    del tgts
    tmps = api.tt_encode_batched(torch.polar(torch.ones_like(ph), ph), chi)
    del ph
    t1 = api.mpo_apply_batched(tmps, wx, chi)
    t2 = api.mpo_apply_batched(t1, wy, chi)
    target = api.tt_to_dense_batched(t2).abs().pow(2).float()
    del t1, t2, tmps
    api.check_status()
    pr = AG.PhaseRetrieval(wx, wy, chi)
    loss, g = pr.loss_and_grad(mask.cores, mask.bonds, target)     # warm-up
    api.check_status()
    # contraction tiles tuned on the gradient step's shapes (setup)
    n_tuned = api.autotune(lambda: pr.loss_and_grad(mask.cores, mask.bonds, target), device=dev)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        loss, g = pr.loss_and_grad(mask.cores, mask.bonds, target)
    ev1.record()
    torch.cuda.synchronize()
    api.check_status()
    ms = ev0.elapsed_time(ev1) / steps
    return {
        "ms": ms,
        "unit": "ms per gradient step (32 problems)",
        "steps": steps,
        "workload": "phase retrieval: 32 x 4096^2 (24 sites), mask chi 64, Fresnel z = 2 mm (x, y) to chi 64, "
                    "decompression, summed squared intensity error; forward with saved state + full adjoint",
        "dtype": "c64 (fp32 MFMA) + f64 eig and eig adjoint",
        "mpo_max_bond": int(max(prop.wx.d_bonds)),
        "autotuned_contraction_shapes": n_tuned,
        "loss": float(loss),
        "grad_norm": float(g.abs().pow(2).sum().sqrt()),
    }


def large_field_bench(steps, dev):
    """16384^2 Gaussian beam x grating (28 sites), never densified: separable
    encode at chi 256, the eight log-spaced distances 0.1 .. 10 mm as one
    batch (x then y, zip-up + sweep to chi 256), 1e5 sampled pixels per
    distance.  Operators built and contraction tiles tuned in the set-up."""
    import torch
    import synth
    from paper_2510_23089_amd import api
    n, chi = 14, 256
    zs = tuple(0.1e-3 * 100.0 ** (j / 7.0) for j in range(8))
    ua, vb = synth.grating_beam_1d(1 << n)
    du = torch.from_numpy(ua).to(torch.complex64).to(dev)
    dv = torch.from_numpy(vb).to(torch.complex64).to(dev)
    rng = np.random.default_rng(7)
    rows = torch.from_numpy(rng.integers(0, 1 << n, 100000)).to(dev)
    cols = torch.from_numpy(rng.integers(0, 1 << n, 100000)).to(dev)
    prop = api.FresnelBatch(n, LAM, DX, zs, device=dev)
    psi = api.MPS(2 * n, chi, device=dev)
    batch = api.MPSBatch(len(zs), 2 * n, chi, device=dev)
    mid = api.MPSBatch(len(zs), 2 * n, chi, device=dev)
    res = api.MPSBatch(len(zs), 2 * n, chi, device=dev)

    def step():
        api.tt_encode_separable(du, dv, chi, out=psi)
        batch.fill_from(psi)
        out = prop(batch, chi, tmp=mid, out=res)
        vals = [api.tt_eval_points(api.MPS.wrap(out.cores[f], out.bonds[f]), rows, cols) for f in range(len(zs))]
        return out, vals

    step()                                                          # set-up: workspaces
    api.check_status()
    n_tuned = api.autotune(step, device=dev)
    step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        out, _vals = step()
    ev1.record()
    torch.cuda.synchronize()
    api.check_status()
    ms = ev0.elapsed_time(ev1) / steps
    return {
        "ms": ms,
        "unit": "ms per batch of 8 propagations (16384^2, chi 256)",
        "propagations_per_s": len(zs) * 1e3 / ms,
        "steps": steps,
        "workload": "16384^2 Gaussian beam (waist 2000 px) x binary grating (period 64 px), 28 sites, never "
                    "densified: separable encode at chi 256, z = 0.1 .. 10 mm (8, log-spaced) as one batch, "
                    "x then y to chi 256, 1e5 sampled pixels per distance",
        "max_bond": int(out.bonds.max()),
        "autotuned_contraction_shapes": n_tuned,
    }


def _kernel_source_hash():
    """sha256 prefix of the sources the dominant kernel is built from: the
    shared helpers (common.h), the eigensolver's helpers and workspace layout
    (eig.hip up to the LDS reduction) and the LDS reduction itself."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2510_23089_amd", "csrc")
    with open(os.path.join(csrc, "common.h"), "rb") as fh:
        common = fh.read()
    with open(os.path.join(csrc, "eig.hip"), "rb") as fh:
        eig = fh.read()
    b = eig.index(b"// (b) 128 < n <= 512: the full matrix is streamed")
    return hashlib.sha256(common + eig[:b]).hexdigest()[:16]


def _traffic(fields_per_step):
    if fields_per_step != TRAFFIC["fields_per_step"]:
        return None
    try:
        h = _kernel_source_hash()
    except (OSError, ValueError):
        return None
    return TRAFFIC["bytes_per_launch"] if h == TRAFFIC["src_sha256_prefix"] else None


FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 (matrix = vector)


def parts_pass(lanes, steps, nz, dev):
    """The step's parts timed on their own after the timed region: the
    propagations alone (x then y for the three distances, from inputs already
    encoded, on the same concurrent lanes), and the encode and the
    decompression of one step, one at a time on one stream."""
    import torch
    main_s = torch.cuda.current_stream(dev)

    def timed(fn):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def props():
        for ln in lanes:
            ln.s.wait_stream(main_s)
        for k in range(steps):
            ln = lanes[k % len(lanes)]
            with torch.cuda.stream(ln.s):
                ln.propagate()
        for ln in lanes:
            main_s.wait_stream(ln.s)

    ln0 = lanes[0]
    ms_prop = timed(props)
    ms_enc = timed(lambda: [ln0.encode() for _ in range(steps)])
    ms_dense = timed(lambda: [ln0.decompress() for _ in range(steps)])
    for ln in lanes:
        ln.check()
    return {"propagation_only": {"propagations_per_s": nz * steps / (ms_prop / 1e3),
                                 "ms_per_step": ms_prop / steps,
                                 "what": "x then y for the %d distances of one field (one batch), inputs already "
                                         "encoded, %d steps on one stream" % (nz, steps)},
            "encode_ms": ms_enc / steps,
            "decompression_ms": ms_dense / steps,
            "serial": "encode (one 1024^2 field, chi 128) and decompression (three 1024^2 fields) of one field, "
                      "one at a time on one stream"}


def contraction_pass(lib, L, run, dev, steps=2):
    """Throughput of the contractions (MFMA) in a separate, untimed pass of
    `steps` serial steps: every product and Gram matrix the library enqueues
    is bracketed by HIP events and its algorithmic flops (8 M N K per complex
    product, 4 n^2 K per Hermitian Gram, from the device-side sizes) logged
    by the library; FP32-MFMA products are priced against the FP32 peak, the
    FP64-accumulating Gram matrices against the FP64 peak."""
    import ctypes
    import torch
    max_l = 600 * steps
    flog = torch.zeros(2 * max_l, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    L.check(lib.tt_prof_begin_flops(ctypes.c_void_p(flog.data_ptr()), max_l), "tt_prof_begin_flops")
    run(steps, 1)
    torch.cuda.synchronize()
    nl, ne, tot = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    L.check(lib.tt_prof_end(ctypes.byref(nl), ctypes.byref(ne), ctypes.byref(tot)), "tt_prof_end")
    n = nl.value
    ms = (ctypes.c_float * max(n, 1))()
    got = lib.tt_prof_times(ms, n)
    if got < 0:
        L.check(got, "tt_prof_times")
    t = np.array(ms[:n], dtype=np.float64) / 1e3
    fl = flog[:2 * n].view(n, 2).cpu().numpy()
    is64 = fl[:, 1] > 0

    def part(mask, col, peak, what):
        f = float(fl[mask, col].sum())
        sec = float(t[mask].sum())
        ach = f / sec / 1e12 if sec > 0 else 0.0
        return {"what": what, "launches_per_step": int(mask.sum()) // steps, "gflop_per_step": f / steps / 1e9,
                "ms_per_step": sec * 1e3 / steps, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak}

    return {"pass": "%d serial steps after the timed region, every contraction bracketed by HIP events" % steps,
            "fp32_products": part(~is64, 0, FP32_PEAK_TFLOPS,
                                  "complex64 products on v_mfma_f32 (zip-up, sweep, encode projections, decompression)"),
            "fp64_gram": part(is64, 1, FP64_PEAK_TFLOPS,
                              "Gram matrices of complex64 operands accumulated on v_mfma_f64 (K-split reductions "
                              "included)")}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build measures one GPU only (DESIGN.md describes how the path would shard). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import ctypes
    import torch
    import synth
    from paper_2510_23089_amd import api
    from paper_2510_23089_amd import _lib as L

    torch.cuda.init()
    dev = torch.device("cuda:0")
    nb = max(a.fields_per_step, 1)
    fields = [synth.aperture_field(seed, n=1 << N_LOG2) for seed in range(nb)]
    d_fields = torch.from_numpy(np.stack(fields)).to(torch.complex64).to(dev)
    nz = len(ZS)
    prop = api.FresnelBatch(N_LOG2, LAM, DX, ZS * nb, device=dev)       # member f * nz + j: field f, ZS[j]
    prop1 = api.FresnelBatch(N_LOG2, LAM, DX, ZS, device=dev)           # one field (serial latency)
    m = 2 * N_LOG2
    chi = a.chi
    main_s = torch.cuda.current_stream(dev)

    class Lane:
        """One step in flight: its own stream (default priority), state
        buffers and library workspaces (keyed per lane).  A step: encode nf
        fields (one batched encode), propagate each to the nz distances (one
        batched zip-up + sweep per axis over nf * nz members), decompress all."""

        def __init__(self, i, nf, pr):
            self.s = main_s if i == 0 else torch.cuda.Stream(device=dev)
            self.nf, self.prop = nf, pr
            self.img = d_fields[:nf]
            self.enc = api.MPSBatch(nf, m, chi, device=dev)
            self.inp = api.MPSBatch(nf * nz, m, chi, device=dev)
            self.mid = api.MPSBatch(nf * nz, m, chi, device=dev)
            self.out = api.MPSBatch(nf * nz, m, chi, device=dev)
            self.dens = torch.empty((nf * nz, 1 << N_LOG2, 1 << N_LOG2), dtype=torch.complex64, device=dev)
            self.key = "lane%d.%d" % (i, nf)

        def encode(self):
            api.tt_encode_batched(self.img, chi, out=self.enc, ws_key=self.key + ".enc")
            # every field's MPS is the input of its nz propagations (device copies)
            sh = self.enc.cores.shape
            self.inp.cores.view(self.nf, nz, *sh[1:]).copy_(self.enc.cores.unsqueeze(1).expand(-1, nz, *sh[1:]))
            self.inp.bonds.view(self.nf, nz, m + 1).copy_(self.enc.bonds.unsqueeze(1).expand(-1, nz, m + 1))

        def propagate(self):
            self.prop(self.inp, chi, tmp=self.mid, out=self.out, ws_key=self.key)

        def decompress(self):
            api.tt_to_dense_batched(self.out, out=self.dens, ws_key=self.key + ".dense")

        def step(self):
            self.encode()
            self.propagate()
            self.decompress()

        def check(self):
            for k in (self.key, self.key + ".enc", self.key + ".dense"):
                api.check_status(k)

    lanes = [Lane(i, nb, prop) for i in range(max(a.inflight, 1))]
    single = Lane(0, 1, prop1)

    def run(steps, inflight, lane_set=None):
        """`steps` steps; step k on lane k mod `inflight` (each lane's steps are
        ordered by its stream, different lanes run concurrently)."""
        ls = (lane_set or lanes)[:inflight]
        for ln in ls:
            ln.s.wait_stream(main_s)
        for k in range(steps):
            ln = ls[k % len(ls)]
            with torch.cuda.stream(ln.s):
                ln.step()
        for ln in ls:
            main_s.wait_stream(ln.s)

    def timed(fn):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run(len(lanes), len(lanes))
    run(1, 1, [single])
    # contraction tiles tuned on the steps' shapes (setup, before any timing;
    # variants differ only in output partitioning, so results are unchanged)
    n_tuned = api.autotune(lambda: (run(1, 1), run(1, 1, [single])), device=dev)
    run(a.warmup * len(lanes), len(lanes))
    for ln in lanes:
        ln.check()
    # ---- headline: nothing but the steps inside the timed region
    t0 = time.perf_counter()
    ms = timed(lambda: run(a.steps, len(lanes))) / a.steps
    wall = time.perf_counter() - t0
    for ln in lanes:
        ln.check()
    # ---- latency of one field's step (one field, its nz distances, one stream);
    # --serial-steps 0 skips it (reported as null)
    serial_ms = None
    if a.serial_steps > 0:
        run(2, 1, [single])
        serial_ms = timed(lambda: run(a.serial_steps, 1, [single])) / a.serial_steps
    # ---- dominant kernel, its launches bracketed by HIP events on their
    # streams, in a pass of its own: the same steps on the same lanes
    lib = L.load()
    psteps = len(lanes) * 2
    max_launch = 200 * psteps * nb
    nlog = torch.zeros(max_launch * nz * 4, dtype=torch.int32, device=dev)
    L.check(lib.tt_prof_begin(2, ctypes.c_void_p(nlog.data_ptr()), nlog.numel(), max_launch), "tt_prof_begin")
    ms_prof = timed(lambda: run(psteps, len(lanes))) / psteps
    launches, entries, kms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    L.check(lib.tt_prof_end(ctypes.byref(launches), ctypes.byref(entries), ctypes.byref(kms)), "tt_prof_end")
    ns = nlog[:entries.value].cpu().numpy().astype(np.float64)
    flops = float(np.sum(16.0 / 3.0 * ns ** 3))
    nl = max(launches.value, 1)
    avg_launch_s = kms.value / 1e3 / nl
    achieved = flops / nl / avg_launch_s / 1e12 if launches.value else 0.0
    # the same kernel's time per step in a serial pass (one stream, no overlap)
    L.check(lib.tt_prof_begin(2, ctypes.c_void_p(nlog.data_ptr()), nlog.numel(), max_launch), "tt_prof_begin")
    run(2, 1)
    torch.cuda.synchronize()
    l2, e2, k2 = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    L.check(lib.tt_prof_end(ctypes.byref(l2), ctypes.byref(e2), ctypes.byref(k2)), "tt_prof_end")
    ms_serial_batch = timed(lambda: run(2, 1)) / 2

    mfma = contraction_pass(lib, L, run, dev)
    gflop = mfma["fp32_products"]["gflop_per_step"] + mfma["fp64_gram"]["gflop_per_step"]
    for ln in lanes:
        ln.check()

    props_per_step = nz * nb
    value = props_per_step / (ms / 1e3)
    res = {
        "metric": "MPO x MPS Fresnel propagations/s at 2^20 px, chi=128",
        "value": value,
        "unit": "propagations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 MFMA) + f64 eig",
        "data": "synthetic",
        "config": {"workload": "%d independent 1024x1024 complex64 aperture fields (seeds 0..%d) per step, each "
                               "propagated to z in {0.5, 2, 8} mm at chi %d: one batched encode, one batched "
                               "zip-up + sweep per axis over the %d (field, z) members, %d decompressions"
                               % (nb, nb - 1, chi, props_per_step, props_per_step),
                   "global_batch": nb, "chi": chi, "sites": m,
                   "steps_in_flight": len(lanes),
                   "schedule": "step k on stream k mod %d (the main stream and %d more, default priority, each "
                               "lane with its own buffers and workspaces)" % (len(lanes), len(lanes) - 1),
                   "autotuned_contraction_shapes": n_tuned},
        "serial_ms_per_step": serial_ms,
        "serial": "one field, its three distances as one batch (encode, x and y application, decompression), "
                  "steps one at a time on one stream: the latency of a single field",
        "roofline": {
            "kernel": "qtt::tridiag_lds_kernel (Householder reduction to tridiagonal form, FP64 Gram "
                      "eigensolver, one workgroup per matrix with its packed lower triangle in LDS: "
                      "matrices up to 128 and the last 128 steps of wider ones)",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": _traffic(a.fields_per_step),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
            "launches": launches.value,
            "avg_launch_ms": avg_launch_s * 1e3,
            "pass": "%d steps on the timed region's lanes right after it, every launch of the kernel bracketed "
                    "by HIP events on its stream (%.2f ms per step with the events)" % (psteps, ms_prof),
            "kernel_ms_per_step_serial": k2.value / 2,
            "serial_ms_per_step": ms_serial_batch,
            "kernel_share_serial": (k2.value / 2) / ms_serial_batch if ms_serial_batch > 0 else None,
            "work_per_launch": "(16/3) n^3 FP64 flops per matrix or trailing block of size n <= 128, "
                               "n logged by the kernel",
            "end_to_end": {
                "gflop_per_step": gflop,
                "what": "algorithmic contraction flops of a step (FP32-MFMA products + FP64-accumulated Gram "
                        "matrices, from the contraction pass) over the headline ms_per_step",
                "achieved_tflops": gflop / ms if ms > 0 else 0.0,
                "frac_of_fp32_peak": gflop / ms / FP32_PEAK_TFLOPS if ms > 0 else 0.0,
            },
        },
        "mfma": mfma,
        "wall_s": wall,
    }
    if a.copy_probe > 0:
        src = torch.ones(a.copy_probe << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_probe_mib"] = a.copy_probe
        del src, dst
    if not a.no_parts:
        res["parts"] = parts_pass([single], a.serial_steps, nz, dev)
    if not a.no_batched:
        res["batched"] = batched_bench(dev)
    if not a.no_grad:
        res["grad_step"] = grad_step_bench(a.grad_steps, dev)
    if not a.no_large:
        res["large_field"] = large_field_bench(a.large_steps, dev)
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(fields[0], chi)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
