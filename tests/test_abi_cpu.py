"""Host-side checks of the C ABI library: it loads, exports every symbol the
public header declares, and rejects bad arguments before touching the GPU
(no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_23089_amd", "libqtt.so")
HDR = os.path.join(ROOT, "include", "qtt.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built (run __graft_entry__.build())")
    from paper_2510_23089_amd import _lib
    return _lib.load(LIB)


def test_header_declares_the_core_calls():
    names = _declared()
    for n in ("tt_encode", "mpo_apply", "tt_truncate", "tt_to_dense", "mpo_apply_backward"):
        assert n in names


def test_every_declared_symbol_exported(lib):
    from paper_2510_23089_amd import _lib
    for n in _declared():
        assert hasattr(lib, n), "missing export %s" % n
    assert sorted(_lib.EXPORTS) == sorted(_declared())


def test_version_and_sizes(lib):
    from paper_2510_23089_amd import _lib as L
    assert b"gfx950" in lib.tt_version()
    assert lib.tt_workspace_size(L.OP_APPLY, 20, 128, 32, L.PREC_FP32) > 0
    assert lib.tt_workspace_size(L.OP_ENCODE, 20, 128, 1, L.PREC_FP32) > 0
    assert lib.tt_workspace_size(L.OP_TO_DENSE, 20, 128, 1, L.PREC_FP32) > 0
    assert lib.tt_workspace_size(L.OP_APPLY, 3, 128, 32, L.PREC_FP32) == 0        # odd site count
    assert lib.tt_workspace_size(L.OP_APPLY, 20, 1000, 32, L.PREC_FP32) == 0      # capacity too large
    # FP64 needs more than FP32
    assert lib.tt_workspace_size(L.OP_APPLY, 12, 32, 8, L.PREC_FP64) > lib.tt_workspace_size(L.OP_APPLY, 12, 32, 8, L.PREC_FP32)


def test_argument_errors_before_enqueue(lib):
    """Invalid arguments are rejected on the host with negative codes; the
    pointers here are never dereferenced on a device."""
    from paper_2510_23089_amd import _lib as L
    fake = ctypes.c_void_p(0x1000)
    s = L.QttMps(12, 32, L.QTT_C64, 0x1000, 0x2000, 0)
    o = L.QttOpts(64, 0, 0.0, 0.0, L.PREC_FP32)           # chi_max > chi_cap
    rc = lib.tt_encode(fake, L.QTT_F32, 6, ctypes.byref(o), ctypes.byref(s), fake, 1 << 30, None)
    assert rc == -5 and b"chi_max" in lib.tt_last_error()
    o = L.QttOpts(16, 0, 0.0, 0.0, L.PREC_FP32)
    rc = lib.tt_encode(fake, L.QTT_F32, 5, ctypes.byref(o), ctypes.byref(s), fake, 1 << 30, None)
    assert rc == -2                                         # 12 sites vs log2_side 5
    rc = lib.tt_encode(fake, L.QTT_F32, 6, ctypes.byref(o), ctypes.byref(s), fake, 16, None)
    assert rc == -4                                         # workspace too small
    rc = lib.tt_encode(None, L.QTT_F32, 6, ctypes.byref(o), ctypes.byref(s), fake, 1 << 30, None)
    assert rc == -1
    rc = lib.tt_encode(fake, 99, 6, ctypes.byref(o), ctypes.byref(s), fake, 1 << 30, None)
    assert rc == -3
    s64 = L.QttMps(12, 32, L.QTT_C64, 0x1000, 0x2000, 0)
    o64 = L.QttOpts(16, 0, 0.0, 0.0, L.PREC_FP64)          # precision/dtype mismatch
    rc = lib.tt_encode(fake, L.QTT_F32, 6, ctypes.byref(o64), ctypes.byref(s64), fake, 1 << 30, None)
    assert rc == -3
    # mpo_apply: MPO site count mismatch, aliasing, MPO boundary bonds
    bonds = (ctypes.c_int32 * 13)(*([1] + [2] * 11 + [1]))
    w = L.QttMpo(10, 2, L.QTT_C64, 0x3000, ctypes.cast(bonds, ctypes.c_void_p), None)
    out = L.QttMps(12, 32, L.QTT_C64, 0x5000, 0x6000, 0)
    rc = lib.mpo_apply(ctypes.byref(s), ctypes.byref(w), ctypes.byref(o), ctypes.byref(out), None, 0, fake, 1 << 30, None)
    assert rc == -2
    rc = lib.mpo_apply(ctypes.byref(s), ctypes.byref(w), ctypes.byref(o), ctypes.byref(s), None, 0, fake, 1 << 30, None)
    assert rc == -1
    bad = (ctypes.c_int32 * 13)(*([2] + [2] * 11 + [1]))
    w = L.QttMpo(12, 2, L.QTT_C64, 0x3000, ctypes.cast(bad, ctypes.c_void_p), None)
    rc = lib.mpo_apply(ctypes.byref(s), ctypes.byref(w), ctypes.byref(o), ctypes.byref(out), None, 0, fake, 1 << 30, None)
    assert rc == -2
    # tt_heev / tt_cgemm shape checks
    assert lib.tt_heev(fake, 1000, 1, 4, 0.0, 0.0, fake, fake, fake, fake, 1 << 30, None) == -2
    assert lib.tt_cgemm(0, 4, 4, fake, 4, 0, fake, 4, 0, fake, 4, L.PREC_FP32, None) == -2


def test_adjoint_argument_errors(lib):
    """The adjoint entry points validate on the host like the forward ones."""
    from paper_2510_23089_amd import _lib as L
    fake = ctypes.c_void_p(0x1000)
    assert lib.tt_saved_size(12, 32, 8, L.PREC_FP32) > 0
    assert lib.tt_saved_size_batched(4, 12, 32, 8, L.PREC_FP32) > 3 * lib.tt_saved_size(12, 32, 8, L.PREC_FP32)
    assert lib.tt_workspace_size(L.OP_APPLY_BACKWARD, 12, 32, 8, L.PREC_FP32) > 0
    assert lib.tt_workspace_size(L.OP_TO_DENSE_BACKWARD, 12, 32, 1, L.PREC_FP32) > 0
    assert lib.tt_workspace_size_batched(L.OP_LOSS, 3, 2, 1, 1, L.PREC_FP32) > 256
    s = L.QttMps(12, 32, L.QTT_C64, 0x1000, 0x2000, 0)
    out = L.QttMps(12, 32, L.QTT_C64, 0x5000, 0x6000, 0)
    go = L.QttMps(12, 32, L.QTT_C64, 0x7000, 0x6000, 0)
    gi = L.QttMps(12, 32, L.QTT_C64, 0x9000, 0x2000, 0)
    o = L.QttOpts(16, 0, 0.0, 0.0, L.PREC_FP32)
    bonds = (ctypes.c_int32 * 13)(*([1] + [2] * 11 + [1]))
    w = L.QttMpo(12, 2, L.QTT_C64, 0x3000, ctypes.cast(bonds, ctypes.c_void_p), None)
    args = (ctypes.byref(s), ctypes.byref(w), ctypes.byref(o))
    # no saved buffer
    rc = lib.mpo_apply_backward(*args, None, 0, ctypes.byref(out), ctypes.byref(go), ctypes.byref(gi), fake, 1 << 30,
                                None)
    assert rc == -1
    # saved buffer too small
    rc = lib.mpo_apply_backward(*args, fake, 16, ctypes.byref(out), ctypes.byref(go), ctypes.byref(gi), fake, 1 << 30,
                                None)
    assert rc == -4 and b"saved" in lib.tt_last_error()
    # grad_in aliasing the input
    rc = lib.mpo_apply_backward(*args, fake, 1 << 40, ctypes.byref(out), ctypes.byref(go), ctypes.byref(s), fake,
                                1 << 30, None)
    assert rc == -1
    # grad_out of a different capacity than out
    go2 = L.QttMps(12, 16, L.QTT_C64, 0x7000, 0x6000, 0)
    rc = lib.mpo_apply_backward(*args, fake, 1 << 40, ctypes.byref(out), ctypes.byref(go2), ctypes.byref(gi), fake,
                                1 << 30, None)
    assert rc == -2
    # forward with a too-small saved buffer
    rc = lib.mpo_apply(ctypes.byref(s), ctypes.byref(w), ctypes.byref(o), ctypes.byref(out), fake, 16, fake, 1 << 30,
                       None)
    assert rc == -4
    # decompression adjoint: dtype mismatch, aliasing
    g64 = L.QttMps(12, 32, L.QTT_C128, 0x9000, 0x2000, 0)
    assert lib.tt_to_dense_backward(ctypes.byref(s), fake, ctypes.byref(g64), fake, 1 << 30, None) == -2
    assert lib.tt_to_dense_backward(ctypes.byref(s), fake, ctypes.byref(s), fake, 1 << 30, None) == -1
    # loss: bad dtype, bad side, small workspace
    assert lib.tt_intensity_loss(fake, fake, L.QTT_F32, 4, 1, fake, None, fake, 1 << 20, None) == -3
    assert lib.tt_intensity_loss(fake, fake, L.QTT_C64, 0, 1, fake, None, fake, 1 << 20, None) == -2
    assert lib.tt_intensity_loss(fake, fake, L.QTT_C64, 4, 1, fake, None, fake, 8, None) == -4


def test_autotune_table_host_side(lib):
    """The tuning table is host state: import/export/clear need no device."""
    import ctypes as C
    assert lib.tt_autotune_clear() == 0
    assert lib.tt_autotune_export(None, 0) == 0
    good = (C.c_int32 * 12)(0, 64, 32, 8, 1, 2, 2, 128, 64, 16, 3, 0)
    assert lib.tt_autotune_import(C.cast(good, C.c_void_p), 2) == 0
    assert lib.tt_autotune_export(None, 0) == 2
    out = (C.c_int32 * 12)()
    assert lib.tt_autotune_export(C.cast(out, C.c_void_p), 2) == 2
    assert sorted([tuple(out[0:6]), tuple(out[6:12])]) == sorted([tuple(good[0:6]), tuple(good[6:12])])
    bad = (C.c_int32 * 6)(0, 64, 32, 8, 1, 7)          # variant out of range
    assert lib.tt_autotune_import(C.cast(bad, C.c_void_p), 1) == -1
    wide = (C.c_int32 * 12)(0, 300, 260, 1, 1, 4, 1, 300, 260, 1, 1, 4)   # wide tile: FP32 only
    assert lib.tt_autotune_import(C.cast(wide, C.c_void_p), 2) == -1
    assert lib.tt_autotune_export(None, 0) == 3
    assert lib.tt_autotune_clear() == 0
    assert lib.tt_autotune_export(None, 0) == 0
    assert lib.tt_autotune_record(0) == 0
    assert lib.tt_autotune_workspace_size() >= 256
