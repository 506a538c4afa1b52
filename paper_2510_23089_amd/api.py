"""Python binding of libqtt: device tensors from PyTorch, compute in HIP.

PyTorch provides device memory and the current HIP stream; every step of the
path runs in libqtt's kernels through the C ABI (see include/qtt.h).  Nothing
here computes on the host except argument marshalling and bookkeeping.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L

_WS_CACHE = {}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _device(device):
    """torch.device with its index filled in ("cuda" and "cuda:0" name one
    cache slot, so a status check finds the workspace its call used)."""
    d = torch.device(device) if device is not None else torch.device("cuda")
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def workspace(nbytes, device=None, key="default"):
    """Cached device workspace (zero-initialised on first use: the status word
    must start at 0)."""
    device = _device(device)
    k = (key, str(device))
    buf = _WS_CACHE.get(k)
    if buf is None or buf.numel() < nbytes:
        buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS_CACHE[k] = buf
    return buf


def _prec_code(prec):
    return {"fp32": L.PREC_FP32, "bf16": L.PREC_BF16, "fp64": L.PREC_FP64, "bf16x3": L.PREC_BF16X3}[prec]


def _ctype(prec):
    return torch.complex128 if prec == "fp64" else torch.complex64


class MPS:
    """Device MPS in capacity layout: cores (m, chi_cap, 2, chi_cap), bonds (m+1) int32."""

    def __init__(self, n_sites, chi_cap, dtype=torch.complex64, device="cuda"):
        self.n_sites = int(n_sites)
        self.chi_cap = int(chi_cap)
        self.cores = torch.zeros((n_sites, chi_cap, 2, chi_cap), dtype=dtype, device=device)
        self.bonds = torch.ones(n_sites + 1, dtype=torch.int32, device=device)
        self.norm = torch.zeros(1, dtype=torch.float64, device=device)

    @property
    def dtype(self):
        return self.cores.dtype

    @property
    def prec(self):
        return "fp64" if self.cores.dtype == torch.complex128 else "fp32"

    def cstruct(self):
        s = L.QttMps()
        s.n_sites = self.n_sites
        s.chi_cap = self.chi_cap
        s.dtype = L.QTT_C128 if self.cores.dtype == torch.complex128 else L.QTT_C64
        s.cores = self.cores.data_ptr()
        s.bonds = self.bonds.data_ptr()
        s.norm = self.norm.data_ptr()
        return s

    def host_cores(self):
        """List of numpy cores [r_k, 2, r_(k+1)] (synchronises)."""
        b = self.bonds.cpu().numpy()
        c = self.cores.cpu().numpy()
        return [c[k, :b[k], :, :b[k + 1]].copy() for k in range(self.n_sites)]

    def host_bonds(self):
        return [int(x) for x in self.bonds.cpu().numpy()]

    @classmethod
    def wrap(cls, cores, bonds, norm=None):
        """View existing device tensors (cores (m, cap, 2, cap), bonds (m+1,) int32) as an MPS."""
        obj = cls.__new__(cls)
        obj.n_sites = int(cores.shape[0])
        obj.chi_cap = int(cores.shape[1])
        obj.cores = cores
        obj.bonds = bonds
        obj.norm = norm if norm is not None else torch.zeros(1, dtype=torch.float64, device=cores.device)
        return obj

    @classmethod
    def from_host(cls, cores, chi_cap=None, dtype=torch.complex64, device="cuda"):
        m = len(cores)
        cap = chi_cap or max(max(c.shape[0], c.shape[2]) for c in cores)
        out = cls(m, cap, dtype=dtype, device=device)
        host = np.zeros((m, cap, 2, cap), dtype=np.complex128)
        bonds = [1]
        for k, c in enumerate(cores):
            host[k, :c.shape[0], :, :c.shape[2]] = c
            bonds.append(c.shape[2])
        out.cores.copy_(torch.from_numpy(host).to(dtype))
        out.bonds.copy_(torch.tensor(bonds, dtype=torch.int32))
        return out


class MPO:
    """Device MPO: flat cores, core k at offset k*d_cap*4*d_cap, dense
    [D_k][t][s][D_(k+1)] with actual bonds; bonds and site kinds on the host."""

    def __init__(self, cores, site_kind=None, dtype=torch.complex64, device="cuda", d_cap=None):
        m = len(cores)
        self.n_sites = m
        self.d_bonds = np.array([1] + [int(c.shape[3]) for c in cores], dtype=np.int32)
        assert int(cores[0].shape[0]) == 1 and self.d_bonds[-1] == 1
        self.d_cap = int(d_cap or max(self.d_bonds.max(), max(int(c.shape[0]) for c in cores)))
        stride = self.d_cap * 4 * self.d_cap
        flat = np.zeros(m * stride, dtype=np.complex128)
        for k, c in enumerate(cores):
            v = np.asarray(c, dtype=np.complex128).reshape(-1)
            flat[k * stride:k * stride + v.size] = v
        self.flat = torch.from_numpy(flat).to(dtype).to(device)
        self.site_kind = None if site_kind is None else np.array(site_kind, dtype=np.int32)
        self.host = [np.asarray(c) for c in cores]

    def cstruct(self):
        s = L.QttMpo()
        s.n_sites = self.n_sites
        s.d_cap = self.d_cap
        s.dtype = L.QTT_C128 if self.flat.dtype == torch.complex128 else L.QTT_C64
        s.cores = self.flat.data_ptr()
        s.d_bonds = self.d_bonds.ctypes.data
        s.site_kind = self.site_kind.ctypes.data if self.site_kind is not None else None
        return s


def _opts(chi_max, chi_zip=0, cutoff=0.0, tau=0.0, prec="fp32", refine=False):
    o = L.QttOpts()
    o.chi_max = int(chi_max)
    o.chi_zip = int(chi_zip or 0)
    o.cutoff = float(cutoff)
    o.tau = float(tau)
    o.prec = _prec_code(prec)
    o.refine = 1 if refine else 0
    return o


def _apply_prec(psi, prec):
    """Contraction precision of an application: the state's (fp32 / fp64) or
    "bf16" (complex64 states only)."""
    if prec is None:
        return psi.prec
    if prec in ("bf16", "bf16x3") and psi.prec != "fp32":
        raise ValueError("bfloat16 contractions need complex64 states")
    return prec


def check_status(key="default"):
    lib = L.load()
    ws = workspace(256, key=key)
    L.check(lib.tt_check_status(_ptr(ws), _stream()), "tt_check_status")


# ------------------------------------------------------------------ entry points
def tt_encode(img, chi, cutoff=0.0, tau=0.0, prec="fp32", chi_cap=None, out=None, ws_key="default"):
    """Encode a square 2^n x 2^n device tensor (float32/64, complex64/128).
    ws_key names the cached workspace (and its status word): calls that may
    run concurrently on different streams need different keys."""
    lib = L.load()
    assert img.is_cuda and img.dim() == 2 and img.shape[0] == img.shape[1]
    n = int(img.shape[0]).bit_length() - 1
    if (1 << n) != img.shape[0]:
        raise ValueError("side must be a power of two")
    img = img.contiguous()
    dt = {torch.float32: L.QTT_F32, torch.float64: L.QTT_F64,
          torch.complex64: L.QTT_C64, torch.complex128: L.QTT_C128}[img.dtype]
    m = 2 * n
    if out is None:
        out = MPS(m, chi_cap or chi, dtype=_ctype(prec), device=img.device)
    o = _opts(chi, 0, cutoff, tau, prec)
    nb = lib.tt_workspace_size(L.OP_ENCODE, m, int(chi), 1, o.prec)
    ws = workspace(nb, img.device, key=ws_key)
    s = out.cstruct()
    L.check(lib.tt_encode(_ptr(img), dt, n, ctypes.byref(o), ctypes.byref(s), _ptr(ws), nb, _stream()), "tt_encode")
    return out


def _cap(psi, out, chi, chi_zip):
    return max(psi.chi_cap, out.chi_cap, int(chi_zip or 0), int(chi))


def saved_buffer(psi, mpo, chi, chi_zip=0, out_cap=None):
    """Device buffer for what a forward application keeps for its adjoint."""
    lib = L.load()
    cap = max(psi.chi_cap, int(out_cap or chi), int(chi_zip or 0), int(chi))
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    count = getattr(psi, "count", None)
    if count is None:
        nb = lib.tt_saved_size(psi.n_sites, cap, mpo.d_cap, prec)
    else:
        nb = lib.tt_saved_size_batched(count, psi.n_sites, cap, mpo.d_cap, prec)
    return torch.empty(max(int(nb), 256), dtype=torch.uint8, device=psi.cores.device)


def mpo_apply(psi, mpo, chi, chi_zip=0, cutoff=0.0, tau=0.0, out=None, chi_cap=None, saved=None, prec=None,
              refine=False):
    """out = W psi: zip-up then the truncation sweep (refine=False) or one
    two-site fitting sweep in full precision (refine=True).  prec: None (the
    state's precision) or "bf16" for bfloat16 contraction operands."""
    lib = L.load()
    prec = _apply_prec(psi, prec)
    if out is None:
        out = MPS(psi.n_sites, chi_cap or chi, dtype=psi.dtype, device=psi.cores.device)
    o = _opts(chi, chi_zip, cutoff, tau, prec, refine)
    nb = lib.tt_workspace_size(L.OP_APPLY, psi.n_sites, _cap(psi, out, chi, chi_zip), mpo.d_cap, o.prec)
    ws = workspace(nb, psi.cores.device)
    si, so, w = psi.cstruct(), out.cstruct(), mpo.cstruct()
    sp, sn = (_ptr(saved), saved.numel()) if saved is not None else (None, 0)
    L.check(lib.mpo_apply(ctypes.byref(si), ctypes.byref(w), ctypes.byref(o), ctypes.byref(so), sp, sn,
                          _ptr(ws), nb, _stream()), "mpo_apply")
    return out


def mpo_apply_backward(psi, mpo, chi, saved, out, grad_out, chi_zip=0, cutoff=0.0, tau=0.0, grad_in=None):
    """Vector-Jacobian product of mpo_apply at psi (cotangent grad_out on the
    output cores); returns the gradient on psi's cores as an MPS."""
    lib = L.load()
    if grad_in is None:
        grad_in = MPS(psi.n_sites, psi.chi_cap, dtype=psi.dtype, device=psi.cores.device)
    o = _opts(chi, chi_zip, cutoff, tau, psi.prec)
    nb = lib.tt_workspace_size(L.OP_APPLY_BACKWARD, psi.n_sites, _cap(psi, out, chi, chi_zip), mpo.d_cap, o.prec)
    ws = workspace(nb, psi.cores.device, key="backward")
    si, w, so, sg, sgi = psi.cstruct(), mpo.cstruct(), out.cstruct(), grad_out.cstruct(), grad_in.cstruct()
    L.check(lib.mpo_apply_backward(ctypes.byref(si), ctypes.byref(w), ctypes.byref(o), _ptr(saved), saved.numel(),
                                   ctypes.byref(so), ctypes.byref(sg), ctypes.byref(sgi), _ptr(ws), nb, _stream()),
            "mpo_apply_backward")
    return grad_in


def tt_to_dense_backward(psi, grad_dense, grad=None):
    """Gradient on psi's cores of a real loss given its gradient on the dense field."""
    lib = L.load()
    if grad is None:
        grad = MPS(psi.n_sites, psi.chi_cap, dtype=psi.dtype, device=psi.cores.device)
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    nb = lib.tt_workspace_size(L.OP_TO_DENSE_BACKWARD, psi.n_sites, psi.chi_cap, 1, prec)
    ws = workspace(nb, psi.cores.device, key="dense_bwd")
    s, sg = psi.cstruct(), grad.cstruct()
    gd = grad_dense.to(psi.dtype).contiguous()
    L.check(lib.tt_to_dense_backward(ctypes.byref(s), _ptr(gd), ctypes.byref(sg), _ptr(ws), nb, _stream()),
            "tt_to_dense_backward")
    return grad


def tt_truncate(psi, chi, cutoff=0.0, tau=0.0):
    lib = L.load()
    o = _opts(chi, 0, cutoff, tau, psi.prec)
    nb = lib.tt_workspace_size(L.OP_TRUNCATE, psi.n_sites, psi.chi_cap, 1, o.prec)
    ws = workspace(nb, psi.cores.device)
    s = psi.cstruct()
    L.check(lib.tt_truncate(ctypes.byref(s), ctypes.byref(o), _ptr(ws), nb, _stream()), "tt_truncate")
    return psi


def tt_to_dense(psi, out=None):
    lib = L.load()
    n = psi.n_sites // 2
    if out is None:
        out = torch.empty((1 << n, 1 << n), dtype=psi.dtype, device=psi.cores.device)
    dt = L.QTT_C128 if out.dtype == torch.complex128 else L.QTT_C64
    nb = lib.tt_workspace_size(L.OP_TO_DENSE, psi.n_sites, psi.chi_cap, 1,
                               L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32)
    ws = workspace(nb, psi.cores.device, key="dense")
    s = psi.cstruct()
    L.check(lib.tt_to_dense(ctypes.byref(s), _ptr(out), dt, _ptr(ws), nb, _stream()), "tt_to_dense")
    return out


def tt_encode_separable(vec_a, vec_b, chi_cap, prec="fp32", out=None):
    """Field vec_a[a] * vec_b[b] (two device vectors of length 2^n, n even)
    as a 2n-site MPS without forming the 2-D array."""
    lib = L.load()
    N = int(vec_a.numel())
    n = N.bit_length() - 1
    assert (1 << n) == N and int(vec_b.numel()) == N
    dt = {torch.float32: L.QTT_F32, torch.float64: L.QTT_F64,
          torch.complex64: L.QTT_C64, torch.complex128: L.QTT_C128}[vec_a.dtype]
    vb = vec_b.to(vec_a.dtype).contiguous()
    va = vec_a.contiguous()
    if out is None:
        out = MPS(2 * n, chi_cap, dtype=_ctype(prec), device=vec_a.device)
    nb = lib.tt_encode_separable_workspace_size(n, out.chi_cap, _prec_code(prec))
    ws = workspace(nb, vec_a.device, key="separable")
    s = out.cstruct()
    L.check(lib.tt_encode_separable(_ptr(va), _ptr(vb), dt, n, ctypes.byref(s), _ptr(ws), nb, _stream()),
            "tt_encode_separable")
    return out


def tt_encode_low_rank(vecs_a, vecs_b, chi, term_cap=None, chi_cap=None, tau=0.0, prec="fp32", out=None,
                       ws_key="low_rank"):
    """Field sum_r vecs_a[r][a] * vecs_b[r][b] (two device tensors of shape
    (rank, 2^n), n even) as a 2n-site MPS of bonds <= chi, without forming
    the 2-D array: the terms encoded as separable fields (bond cap term_cap,
    default chi_cap // rank), summed as MPS and TT-rounded."""
    lib = L.load()
    assert vecs_a.dim() == 2 and vecs_a.shape == vecs_b.shape
    rank, N = int(vecs_a.shape[0]), int(vecs_a.shape[1])
    n = N.bit_length() - 1
    assert (1 << n) == N
    dt = {torch.float32: L.QTT_F32, torch.float64: L.QTT_F64,
          torch.complex64: L.QTT_C64, torch.complex128: L.QTT_C128}[vecs_a.dtype]
    va = vecs_a.contiguous()
    vb = vecs_b.to(vecs_a.dtype).contiguous()
    if out is None:
        out = MPS(2 * n, chi_cap or 256, dtype=_ctype(prec), device=vecs_a.device)
    tc = int(term_cap or out.chi_cap // rank)
    o = _opts(chi, 0, 0.0, tau, prec)
    nb = lib.tt_encode_low_rank_workspace_size(n, rank, tc, out.chi_cap, o.prec)
    if nb == 0:
        raise ValueError("rank %d / term_cap %d / chi_cap %d outside the supported range" % (rank, tc, out.chi_cap))
    ws = workspace(nb, vecs_a.device, key=ws_key)
    s = out.cstruct()
    L.check(lib.tt_encode_low_rank(_ptr(va), _ptr(vb), dt, n, rank, tc, ctypes.byref(s), ctypes.byref(o), _ptr(ws), nb,
                                   _stream()), "tt_encode_low_rank")
    return out


def tt_sample(psi, count=None, uniforms=None, seed=0, ws_key="sample"):
    """Perfect samples (rows, cols) of |E|^2 / ||E||^2 from a left-canonical
    MPS (device int32 tensors).  uniforms: device float64 (count, n_sites) in
    [0, 1), the random numbers the sampling draws; by default torch's
    generator seeded with `seed` on the MPS's device."""
    lib = L.load()
    m = psi.n_sites
    dev = psi.cores.device
    if uniforms is None:
        g = torch.Generator(device=dev)
        g.manual_seed(int(seed))
        uniforms = torch.rand((int(count), m), dtype=torch.float64, device=dev, generator=g)
    uniforms = uniforms.to(torch.float64).contiguous()
    count = int(uniforms.shape[0])
    assert uniforms.shape[1] == m
    rows = torch.empty(count, dtype=torch.int32, device=dev)
    cols = torch.empty(count, dtype=torch.int32, device=dev)
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    nb = lib.tt_sample_workspace_size(m, psi.chi_cap, count, prec)
    ws = workspace(nb, dev, key=ws_key)
    s = psi.cstruct()
    L.check(lib.tt_sample(ctypes.byref(s), _ptr(uniforms), count, _ptr(rows), _ptr(cols), _ptr(ws), nb, _stream()),
            "tt_sample")
    return rows, cols


def tt_eval_points(psi, rows, cols):
    """Field values at pixels (rows[p], cols[p]) (device int32 tensors)."""
    lib = L.load()
    count = int(rows.numel())
    r = rows.to(torch.int32).contiguous()
    c = cols.to(torch.int32).contiguous()
    out = torch.empty(count, dtype=psi.dtype, device=psi.cores.device)
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    nb = lib.tt_eval_points_workspace_size(psi.n_sites, psi.chi_cap, count, prec)
    ws = workspace(nb, psi.cores.device, key="points")
    s = psi.cstruct()
    L.check(lib.tt_eval_points(ctypes.byref(s), _ptr(r), _ptr(c), count, _ptr(out), _ptr(ws), nb, _stream()),
            "tt_eval_points")
    return out


def tt_to_dense_block(psi, log2_block, block_row, block_col, out=None):
    """The aligned 2^log2_block square block (block_row, block_col) of the field."""
    lib = L.load()
    side = 1 << log2_block
    if out is None:
        out = torch.empty((side, side), dtype=psi.dtype, device=psi.cores.device)
    dt = L.QTT_C128 if out.dtype == torch.complex128 else L.QTT_C64
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    nb = lib.tt_to_dense_block_workspace_size(psi.n_sites, psi.chi_cap, log2_block, prec)
    ws = workspace(nb, psi.cores.device, key="block")
    s = psi.cstruct()
    L.check(lib.tt_to_dense_block(ctypes.byref(s), log2_block, block_row, block_col, _ptr(out), dt, _ptr(ws), nb,
                                  _stream()), "tt_to_dense_block")
    return out


def tt_to_dense_window(psi, row0, col0, rows, cols, log2_block=0, out=None):
    """An arbitrary rows x cols window at (row0, col0) of the field, assembled
    by the library from the aligned blocks that cover it (nothing outside
    those blocks is formed); log2_block 0 lets the library pick the block."""
    lib = L.load()
    if out is None:
        out = torch.empty((rows, cols), dtype=psi.dtype, device=psi.cores.device)
    dt = L.QTT_C128 if out.dtype == torch.complex128 else L.QTT_C64
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    nb = lib.tt_to_dense_window_workspace_size(psi.n_sites, psi.chi_cap, rows, cols, int(log2_block or 0), prec)
    ws = workspace(max(nb, 256), psi.cores.device, key="window")
    s = psi.cstruct()
    L.check(lib.tt_to_dense_window(ctypes.byref(s), row0, col0, rows, cols, int(log2_block or 0), _ptr(out), dt,
                                   _ptr(ws), max(nb, 256), _stream()), "tt_to_dense_window")
    return out


def tt_hadamard(a, b, chi, conj_a=False, chi_zip=0, cutoff=0.0, tau=0.0, out=None, chi_cap=None):
    """Element-wise product out = a (.) b (conj(a) (.) b if conj_a) of two
    MPS of the same site count, truncated to chi (zip-up cap chi_zip)."""
    lib = L.load()
    if out is None:
        out = MPS(b.n_sites, chi_cap or chi, dtype=b.dtype, device=b.cores.device)
    o = _opts(chi, chi_zip, cutoff, tau, b.prec)
    cap = max(b.chi_cap, out.chi_cap, int(chi_zip or 0), int(chi))
    nb = lib.tt_hadamard_workspace_size(b.n_sites, a.chi_cap, cap, o.prec)
    ws = workspace(nb, b.cores.device, key="hadamard")
    sa, sb, so = a.cstruct(), b.cstruct(), out.cstruct()
    L.check(lib.tt_hadamard(ctypes.byref(sa), 1 if conj_a else 0, ctypes.byref(sb), ctypes.byref(o), ctypes.byref(so),
                            _ptr(ws), nb, _stream()), "tt_hadamard")
    return out


class MPSBatch:
    """count MPS of one shape in one allocation: cores (count, m, chi_cap, 2, chi_cap)."""

    def __init__(self, count, n_sites, chi_cap, dtype=torch.complex64, device="cuda"):
        self.count = int(count)
        self.n_sites = int(n_sites)
        self.chi_cap = int(chi_cap)
        self.cores = torch.zeros((count, n_sites, chi_cap, 2, chi_cap), dtype=dtype, device=device)
        self.bonds = torch.ones((count, n_sites + 1), dtype=torch.int32, device=device)
        self.norms = torch.zeros(count, dtype=torch.float64, device=device)

    @property
    def dtype(self):
        return self.cores.dtype

    @property
    def prec(self):
        return "fp64" if self.cores.dtype == torch.complex128 else "fp32"

    def cstruct(self):
        s = L.QttMpsBatch()
        s.count = self.count
        s.n_sites = self.n_sites
        s.chi_cap = self.chi_cap
        s.dtype = L.QTT_C128 if self.cores.dtype == torch.complex128 else L.QTT_C64
        s.cores = self.cores.data_ptr()
        s.bonds = self.bonds.data_ptr()
        s.norms = self.norms.data_ptr()
        return s

    @classmethod
    def wrap(cls, cores, bonds, norms=None):
        """View existing device tensors (cores (count, m, cap, 2, cap), bonds (count, m+1)) as a batch."""
        obj = cls.__new__(cls)
        obj.count = int(cores.shape[0])
        obj.n_sites = int(cores.shape[1])
        obj.chi_cap = int(cores.shape[2])
        obj.cores = cores
        obj.bonds = bonds
        obj.norms = norms if norms is not None else torch.zeros(obj.count, dtype=torch.float64, device=cores.device)
        return obj

    def fill_from(self, psi, index=None):
        """Copy a single MPS (same n_sites, chi_cap <= ours) into one or all fields (device copy)."""
        idx = range(self.count) if index is None else [index]
        c = psi.chi_cap
        for f in idx:
            self.cores[f, :, :c, :, :c].copy_(psi.cores)
            self.bonds[f].copy_(psi.bonds)
        return self

    def field(self, f):
        """Host cores of field f (synchronises)."""
        b = self.bonds[f].cpu().numpy()
        c = self.cores[f].cpu().numpy()
        return [c[k, :b[k], :, :b[k + 1]].copy() for k in range(self.n_sites)]


class MPOBatch:
    """count MPOs padded to one bond profile (zero padding leaves each operator unchanged)."""

    def __init__(self, mpos, dtype=torch.complex64, device="cuda"):
        m = mpos[0].n_sites if isinstance(mpos[0], MPO) else len(mpos[0])
        hosts = [x.host if isinstance(x, MPO) else x for x in mpos]
        kinds = [x.site_kind if isinstance(x, MPO) else None for x in mpos]
        self.count = len(hosts)
        self.n_sites = m
        prof = np.ones(m + 1, dtype=np.int32)
        for h in hosts:
            prof = np.maximum(prof, [1] + [int(c.shape[3]) for c in h])
        self.d_bonds = prof.astype(np.int32)
        self.d_cap = int(prof.max())
        # a site is a pass-through (kind 1) for the batch when it is one for
        # every member (its padded bond profile then stays equal across it)
        if all(k is not None for k in kinds):
            # identity for the batch when an identity for every member,
            # diagonal when diagonal for every member, else general
            kind = np.zeros(m, dtype=np.int32)
            for j in range(m):
                kj = {int(k[j]) for k in kinds}
                kind[j] = kj.pop() if len(kj) == 1 and kj <= {1, 2} else 0
            ok = all(prof[j] == prof[j + 1] for j in range(m) if kind[j] == 1)
            self.site_kind = kind if ok and kind.any() else None
        else:
            self.site_kind = None
        stride = self.d_cap * 4 * self.d_cap
        flat = np.zeros((self.count, m * stride), dtype=np.complex128)
        for f, h in enumerate(hosts):
            for k, c in enumerate(h):
                w = np.zeros((prof[k], 2, 2, prof[k + 1]), dtype=np.complex128)
                w[:c.shape[0], :, :, :c.shape[3]] = c
                flat[f, k * stride:k * stride + w.size] = w.reshape(-1)
        self.flat = torch.from_numpy(flat).to(dtype).to(device)

    def cstruct(self):
        s = L.QttMpoBatch()
        s.count = self.count
        s.n_sites = self.n_sites
        s.d_cap = self.d_cap
        s.dtype = L.QTT_C128 if self.flat.dtype == torch.complex128 else L.QTT_C64
        s.cores = self.flat.data_ptr()
        s.d_bonds = self.d_bonds.ctypes.data
        s.site_kind = self.site_kind.ctypes.data if self.site_kind is not None else None
        return s


def mpo_apply_batched(psi, mpo, chi, chi_zip=0, cutoff=0.0, tau=0.0, out=None, chi_dev=None, chi_cap=None,
                      saved=None, prec=None, refine=False, ws_key="default"):
    """ws_key names the cached workspace (and its status word), as in tt_encode:
    calls that may run concurrently on different streams need different keys."""
    lib = L.load()
    prec = _apply_prec(psi, prec)
    if out is None:
        out = MPSBatch(psi.count, psi.n_sites, chi_cap or chi, dtype=psi.dtype, device=psi.cores.device)
    o = _opts(chi, chi_zip, cutoff, tau, prec, refine)
    nb = lib.tt_workspace_size_batched(L.OP_APPLY, psi.count, psi.n_sites, _cap(psi, out, chi, chi_zip), mpo.d_cap,
                                       o.prec)
    ws = workspace(nb, psi.cores.device, key=ws_key)
    si, so, w = psi.cstruct(), out.cstruct(), mpo.cstruct()
    sp, sn = (_ptr(saved), saved.numel()) if saved is not None else (None, 0)
    L.check(lib.mpo_apply_batched(ctypes.byref(si), ctypes.byref(w), ctypes.byref(o), _ptr(chi_dev),
                                  ctypes.byref(so), sp, sn, _ptr(ws), nb, _stream()), "mpo_apply_batched")
    return out


def mpo_apply_backward_batched(psi, mpo, chi, saved, out, grad_out, chi_zip=0, cutoff=0.0, tau=0.0, grad_in=None):
    lib = L.load()
    if grad_in is None:
        grad_in = MPSBatch(psi.count, psi.n_sites, psi.chi_cap, dtype=psi.dtype, device=psi.cores.device)
    o = _opts(chi, chi_zip, cutoff, tau, psi.prec)
    nb = lib.tt_workspace_size_batched(L.OP_APPLY_BACKWARD, psi.count, psi.n_sites, _cap(psi, out, chi, chi_zip),
                                       mpo.d_cap, o.prec)
    ws = workspace(nb, psi.cores.device, key="backward")
    si, w, so, sg, sgi = psi.cstruct(), mpo.cstruct(), out.cstruct(), grad_out.cstruct(), grad_in.cstruct()
    L.check(lib.mpo_apply_backward_batched(ctypes.byref(si), ctypes.byref(w), ctypes.byref(o), _ptr(saved),
                                           saved.numel(), ctypes.byref(so), ctypes.byref(sg), ctypes.byref(sgi),
                                           _ptr(ws), nb, _stream()), "mpo_apply_backward_batched")
    return grad_in


def tt_to_dense_backward_batched(psi, grad_dense, grad=None):
    lib = L.load()
    if grad is None:
        grad = MPSBatch(psi.count, psi.n_sites, psi.chi_cap, dtype=psi.dtype, device=psi.cores.device)
    prec = L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32
    nb = lib.tt_workspace_size_batched(L.OP_TO_DENSE_BACKWARD, psi.count, psi.n_sites, psi.chi_cap, 1, prec)
    ws = workspace(nb, psi.cores.device, key="dense_bwd")
    s, sg = psi.cstruct(), grad.cstruct()
    gd = grad_dense.to(psi.dtype).contiguous()
    L.check(lib.tt_to_dense_backward_batched(ctypes.byref(s), _ptr(gd), ctypes.byref(sg), _ptr(ws), nb, _stream()),
            "tt_to_dense_backward_batched")
    return grad


def intensity_loss(field, target, with_grad=True):
    """Per-field loss sum (|E|^2 - I)^2 of (count, N, N) or (N, N) fields and
    its gradient 4 (|E|^2 - I) E; returns (loss float64 tensor (count,), grad or None)."""
    lib = L.load()
    f = field if field.dim() == 3 else field.unsqueeze(0)
    f = f.contiguous()
    count, side = int(f.shape[0]), int(f.shape[1])
    n = side.bit_length() - 1
    real_t = torch.float64 if f.dtype == torch.complex128 else torch.float32
    t = target.to(real_t).reshape(f.shape).contiguous()
    dt = L.QTT_C128 if f.dtype == torch.complex128 else L.QTT_C64
    loss = torch.empty(count, dtype=torch.float64, device=f.device)
    grad = torch.empty_like(f) if with_grad else None
    nb = lib.tt_workspace_size_batched(L.OP_LOSS, count, 2, 1, 1, L.PREC_FP32)
    ws = workspace(nb, f.device, key="loss")
    L.check(lib.tt_intensity_loss(_ptr(f), _ptr(t), dt, n, count, _ptr(loss), _ptr(grad), _ptr(ws), nb, _stream()),
            "tt_intensity_loss")
    if field.dim() == 2 and grad is not None:
        grad = grad[0]
    return loss, grad


def tt_encode_batched(imgs, chi, cutoff=0.0, tau=0.0, prec="fp32", chi_cap=None, out=None, chi_dev=None,
                      ws_key="encode"):
    """imgs: device tensor (count, N, N).  ws_key: the cached workspace, as in tt_encode."""
    lib = L.load()
    count = int(imgs.shape[0])
    n = int(imgs.shape[1]).bit_length() - 1
    imgs = imgs.contiguous()
    dt = {torch.float32: L.QTT_F32, torch.float64: L.QTT_F64,
          torch.complex64: L.QTT_C64, torch.complex128: L.QTT_C128}[imgs.dtype]
    if out is None:
        out = MPSBatch(count, 2 * n, chi_cap or chi, dtype=_ctype(prec), device=imgs.device)
    o = _opts(chi, 0, cutoff, tau, prec)
    nb = lib.tt_workspace_size_batched(L.OP_ENCODE, count, 2 * n, int(chi), 1, o.prec)
    ws = workspace(nb, imgs.device, key=ws_key)
    s = out.cstruct()
    L.check(lib.tt_encode_batched(_ptr(imgs), dt, n, ctypes.byref(o), _ptr(chi_dev), ctypes.byref(s), _ptr(ws), nb,
                                  _stream()), "tt_encode_batched")
    return out


def tt_to_dense_batched(psi, out=None, ws_key="dense"):
    """ws_key: the cached workspace, as in tt_encode."""
    lib = L.load()
    n = psi.n_sites // 2
    if out is None:
        out = torch.empty((psi.count, 1 << n, 1 << n), dtype=psi.dtype, device=psi.cores.device)
    dt = L.QTT_C128 if out.dtype == torch.complex128 else L.QTT_C64
    nb = lib.tt_workspace_size_batched(L.OP_TO_DENSE, psi.count, psi.n_sites, psi.chi_cap, 1,
                                       L.PREC_FP64 if psi.prec == "fp64" else L.PREC_FP32)
    ws = workspace(nb, psi.cores.device, key=ws_key)
    s = psi.cstruct()
    L.check(lib.tt_to_dense_batched(ctypes.byref(s), _ptr(out), dt, _ptr(ws), nb, _stream()), "tt_to_dense_batched")
    return out


class FresnelBatch:
    """x- and y-axis Fresnel MPOs for several distances z, batched (one field per z)."""

    def __init__(self, n, lam, dx, zs, dtype=torch.complex64, device="cuda", rel=1e-12):
        uniq = {}
        for z in zs:
            if z not in uniq:
                uniq[z] = FresnelPropagator(n, lam, dx, z, dtype=dtype, device=device, rel=rel)
        props = [uniq[z] for z in zs]
        self.wx = MPOBatch([p.wx for p in props], dtype=dtype, device=device)
        self.wy = MPOBatch([p.wy for p in props], dtype=dtype, device=device)
        self.count = len(zs)

    def __call__(self, psi, chi, chi_zip=0, cutoff=0.0, tau=0.0, tmp=None, out=None, chi_dev=None, prec=None,
                 refine=False, ws_key="default"):
        mid = mpo_apply_batched(psi, self.wx, chi, chi_zip, cutoff, tau, out=tmp, chi_dev=chi_dev, prec=prec,
                                refine=refine, ws_key=ws_key)
        return mpo_apply_batched(mid, self.wy, chi, chi_zip, cutoff, tau, out=out, chi_dev=chi_dev, prec=prec,
                                 refine=refine, ws_key=ws_key)


class FresnelPropagator:
    """Both axis MPOs of the Fresnel propagator for an N x N grid (Sec. 6.1)."""

    def __init__(self, n, lam, dx, z, dtype=torch.complex64, device="cuda", rel=1e-12):
        from . import mpo_build as B
        w1 = B.fresnel_axis(n, lam, dx, z, rel)
        cx, kx = B.embed(w1, "x")
        cy, ky = B.embed(w1, "y")
        dcap = max(B.bonds(w1))
        self.wx = MPO(cx, kx, dtype=dtype, device=device, d_cap=dcap)
        self.wy = MPO(cy, ky, dtype=dtype, device=device, d_cap=dcap)
        self.axis_cores = w1

    def __call__(self, psi, chi, chi_zip=0, cutoff=0.0, tau=0.0, tmp=None, out=None, prec=None, refine=False):
        mid = mpo_apply(psi, self.wx, chi, chi_zip, cutoff, tau, out=tmp, prec=prec, refine=refine)
        return mpo_apply(mid, self.wy, chi, chi_zip, cutoff, tau, out=out, prec=prec, refine=refine)


_QFT_CACHE = {}


def _qft_pair(n, rel=1e-12):
    """(QFT_br, QFT_br^H) per-axis MPOs, left-canonical, cached per n."""
    from . import mpo_build as B
    if n not in _QFT_CACHE:
        q = B.round_left(B.qft_br(n), rel)
        _QFT_CACHE[n] = (q, B.round_left(B.dagger(q), rel))
    return _QFT_CACHE[n]


class FresnelThreeStage:
    """The per-axis propagator applied as its three factors (Sec. 6.1, Fig. of
    the MPO product): QFT_br, the diagonal transfer function, QFT_br^H, each
    an MPO application (zip-up + sweep to chi) of its own, x axis then y axis.
    route: the diagonal's construction ("svd", "pauli" or, for the lattice
    dispersion, "bessel"); its sites run the diagonal contraction."""

    def __init__(self, n, lam, dx, z, route="svd", dispersion="parabolic", dtype=torch.complex64, device="cuda",
                 rel=1e-12):
        from . import mpo_build as B
        q, iq = _qft_pair(n, rel)
        d = B.diag_fresnel(n, lam, dx, z, route, dispersion, rel=rel)
        self.axis = {"qft": q, "diag": d, "iqft": iq}
        self.stages = {}
        for ax in ("x", "y"):
            seq = []
            for name, cores, diag in (("qft", q, False), ("diag", d, True), ("iqft", iq, False)):
                c, kind = B.embed(cores, ax, diag=diag)
                seq.append(MPO(c, kind, dtype=dtype, device=device, d_cap=max(B.bonds(cores))))
            self.stages[ax] = seq

    def __call__(self, psi, chi, chi_zip=0, cutoff=0.0, tau=0.0):
        out = psi
        for ax in ("x", "y"):
            for w in self.stages[ax]:
                out = mpo_apply(out, w, chi, chi_zip, cutoff, tau)
        return out


def qft2(psi, chi, inverse=False, chi_zip=0, cutoff=0.0, tau=0.0):
    """2-D unitary DFT of the field (x then y; with bit-reversed frequency
    registers, as the QFT MPO of Sec. 5 produces them), or its inverse
    (bit-reversed registers in, natural order out)."""
    from . import mpo_build as B
    n = psi.n_sites // 2
    q, iq = _qft_pair(n)
    w1 = iq if inverse else q
    key = (n, inverse, str(psi.cores.device), psi.dtype)
    mp = _QFT_MPO.get(key)
    if mp is None:
        mp = [MPO(*B.embed(w1, ax), dtype=psi.dtype, device=psi.cores.device, d_cap=max(B.bonds(w1)))
              for ax in ("x", "y")]
        _QFT_MPO[key] = mp
    out = mpo_apply(psi, mp[0], chi, chi_zip, cutoff, tau)
    return mpo_apply(out, mp[1], chi, chi_zip, cutoff, tau)


_QFT_MPO = {}


def psf(pupil, chi, chi_field=None, chi_zip=0):
    """Point spread function of a pupil field (Sec. 5): the focal-plane field
    phi = QFT(pupil) (x then y, bit-reversed frequency registers, truncated
    to chi_field), then PSF = conj(phi) (.) phi, truncated to chi.  Returns
    (phi, psf) as MPS."""
    phi = qft2(pupil, chi_field or chi, chi_zip=chi_zip)
    return phi, tt_hadamard(phi, phi, chi, conj_a=True, chi_zip=chi_zip)


def image_formation(obj, psf_mps, chi, chi_zip=0):
    """Image of a scene through an optical system of point spread function
    psf (both on the natural N x N grid, Sec. 5, equation of the convolution):
    IQFT(QFT(psf) (.) QFT(obj)), every step truncated to chi; with unitary
    transforms this is the circular convolution psf * obj divided by N."""
    a = qft2(psf_mps, chi, chi_zip=chi_zip)
    b = qft2(obj, chi, chi_zip=chi_zip)
    return qft2(tt_hadamard(a, b, chi, chi_zip=chi_zip), chi, inverse=True, chi_zip=chi_zip)


class AngularSpectrum:
    """The non-paraxial angular-spectrum propagator (Sec. 6.1): QFT on both
    axes, the 2-D transfer function as one diagonal MPO over all 2n sites
    (it does not separate), inverse QFT on both axes; five MPO applications
    (zip-up + sweep to chi each)."""

    def __init__(self, n, lam, dx, z, dtype=torch.complex64, device="cuda", rel=1e-12):
        from . import mpo_build as B
        q, iq = _qft_pair(n, rel)
        d2 = B.angular_spectrum_diag(n, lam, dx, z, rel)
        self.diag_cores = d2
        dq = max(B.bonds(q))
        self.qx = MPO(*B.embed(q, "x"), dtype=dtype, device=device, d_cap=dq)
        self.qy = MPO(*B.embed(q, "y"), dtype=dtype, device=device, d_cap=dq)
        self.iqx = MPO(*B.embed(iq, "x"), dtype=dtype, device=device, d_cap=dq)
        self.iqy = MPO(*B.embed(iq, "y"), dtype=dtype, device=device, d_cap=dq)
        self.d = MPO(d2, [2] * len(d2), dtype=dtype, device=device)

    def __call__(self, psi, chi, chi_zip=0, cutoff=0.0, tau=0.0):
        out = psi
        for w in (self.qx, self.qy, self.d, self.iqy, self.iqx):
            out = mpo_apply(out, w, chi, chi_zip, cutoff, tau)
        return out


# ------------------------------------------------------------------ autotuner
def autotune(run, device=None, path=None):
    """Record the contraction shapes of run() (called once), time every tile
    variant for each on this device and keep the fastest.  Optionally save the
    table as JSON to `path`.  Returns the number of shapes tuned."""
    import json
    lib = L.load()
    L.check(lib.tt_autotune_record(1), "tt_autotune_record")
    try:
        run()
        torch.cuda.synchronize(device)
    finally:
        L.check(lib.tt_autotune_record(0), "tt_autotune_record")
    nb = int(lib.tt_autotune_workspace_size())
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device or "cuda")
    n = ctypes.c_int(0)
    L.check(lib.tt_autotune_run(_ptr(ws), ws.numel(), _stream(), ctypes.byref(n)), "tt_autotune_run")
    if path is not None:
        with open(path, "w") as fh:
            json.dump(autotune_table(), fh)
    return n.value


def autotune_table():
    """The current tuning table as a list of [types, m, n, depth, pattern, variant]."""
    lib = L.load()
    cnt = lib.tt_autotune_export(None, 0)
    buf = (ctypes.c_int32 * (6 * max(cnt, 1)))()
    cnt = lib.tt_autotune_export(ctypes.cast(buf, ctypes.c_void_p), cnt)
    return [list(buf[6 * i:6 * i + 6]) for i in range(cnt)]


def autotune_load(table_or_path):
    """Load a table saved by autotune(path=...) (or the list itself)."""
    import json
    lib = L.load()
    table = table_or_path
    if isinstance(table_or_path, str):
        with open(table_or_path) as fh:
            table = json.load(fh)
    flat = [int(x) for e in table for x in e]
    buf = (ctypes.c_int32 * max(len(flat), 1))(*flat)
    L.check(lib.tt_autotune_import(ctypes.cast(buf, ctypes.c_void_p), len(table)), "tt_autotune_import")
