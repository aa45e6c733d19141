"""The C ABI: the library loads on a machine without a GPU and exports every
function declared in include/hqr.h; argument checks reject bad input without
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hqr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hqr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hqr_factor", "hqr_elimlist", "hqr_workspace_size", "hqr_status"):
        assert must in names


def test_every_declared_symbol_is_exported(hqr_lib):
    for name in declared_functions():
        assert hasattr(hqr_lib, name), name
        assert ctypes.cast(getattr(hqr_lib, name), ctypes.c_void_p).value


def test_binding_covers_the_header(hqr_lib):
    from paper_1110_1553_amd import _lib

    assert sorted(_lib.EXPORTS) == declared_functions()


def test_argument_checks_do_not_touch_the_device(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    p = h.make_params(nb=64, a=100)
    # M < N, lda < M, bad tile size, bad inner blocking: rejected before any HIP call
    assert hqr_lib.hqr_factor(ctypes.c_void_p(16), 100, 200, 100, ctypes.byref(p), None, ctypes.c_void_p(16), 1 << 30, None, None) == -2
    assert hqr_lib.hqr_factor(ctypes.c_void_p(16), 200, 100, 100, ctypes.byref(p), None, ctypes.c_void_p(16), 1 << 30, None, None) == -4
    bad = h.make_params(nb=96)
    assert hqr_lib.hqr_factor(ctypes.c_void_p(16), 256, 128, 256, ctypes.byref(bad), None, ctypes.c_void_p(16), 1 << 30, None, None) == -5
    bad = h.make_params(nb=64, ib=32)
    assert hqr_lib.hqr_factor(ctypes.c_void_p(16), 256, 128, 256, ctypes.byref(bad), None, ctypes.c_void_p(16), 1 << 30, None, None) == -5
    # workspace too small
    need = h.workspace_size(256, 128, p)
    assert hqr_lib.hqr_factor(ctypes.c_void_p(16), 256, 128, 256, ctypes.byref(p), None, ctypes.c_void_p(16), need - 1, None, None) == -8
    with pytest.raises(h.HQRError):
        h.workspace_size(10, 20, p)
    assert _lib.load().hqr_strerror(2).decode().startswith("a task waited")


def test_workspace_holds_padded_tile_copy(hqr_lib):
    import paper_1110_1553_amd as h

    p = h.make_params(nb=64)
    aligned = h.workspace_size(512, 256, p)
    ragged = h.workspace_size(500, 250, p)
    # same 8 x 4 tile grid; the workspace holds the zero-padded tiles
    assert ragged == aligned
    assert aligned >= 512 * 256 * 8 + 2 * 8 * 4 * 64 * 16 * 8
    assert h.workspace_size(513, 256, p) >= aligned + 4 * 64 * 64 * 8


def test_apply_and_lstsq_argument_checks(hqr_lib):
    import paper_1110_1553_amd as h

    p = h.make_params(nb=64)
    vp = ctypes.c_void_p
    need = h.workspace_size(256, 128, p)
    bneed = h.apply_workspace_size(256, 3, p)
    assert bneed >= 256 * 64 * 8
    args = lambda M, N, ldb, nrhs, wb, bb: (M, N, ctypes.byref(p), None, vp(16), wb, vp(16), ldb, nrhs, vp(16), bb, None)
    for fn in (hqr_lib.hqr_apply_qt, hqr_lib.hqr_apply_q):
        assert fn(*args(100, 200, 100, 1, need, bneed)) == -2       # M < N
        assert fn(*args(256, 128, 200, 1, need, bneed)) == -9       # ldb < M
        assert fn(*args(256, 128, 256, 0, need, bneed)) == -10      # nrhs < 1
        assert fn(*args(256, 128, 256, 3, need - 1, bneed)) == -7   # factorization workspace too small
        assert fn(*args(256, 128, 256, 3, need, bneed - 1)) == -12  # apply workspace too small
    lneed = h.lstsq_workspace_size(256, 128, 3, p)
    assert lneed >= need + 256 * 64 * 8
    L = hqr_lib.hqr_lstsq
    assert L(vp(16), 256, 128, 256, vp(16), 200, 1, ctypes.byref(p), None, vp(16), lneed, None, None) == -6
    assert L(vp(16), 256, 128, 256, vp(16), 256, 3, ctypes.byref(p), None, vp(16), lneed - 1, None, None) == -11
    assert L(vp(16), 256, 128, 256, vp(16), 256, 0, ctypes.byref(p), None, vp(16), lneed, None, None) == -7
    with pytest.raises(h.HQRError):
        h.apply_workspace_size(256, 0, p)


def test_f32_ir_and_solve_argument_checks(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    p = h.make_params(nb=64)
    vp = ctypes.c_void_p
    # FP32 workspaces hold float tiles and T: smaller than the FP64 ones, larger than the float tiles alone
    w64, w32 = h.workspace_size(512, 256, p), _lib.workspace_size_f32(512, 256, p)
    assert 512 * 256 * 4 < w32 < w64
    F = hqr_lib.hqr_factor_f32
    assert F(vp(16), 100, 200, 100, ctypes.byref(p), None, vp(16), 1 << 30, None, None) == -2
    assert F(vp(16), 200, 100, 150, ctypes.byref(p), None, vp(16), 1 << 30, None, None) == -4
    assert F(vp(16), 512, 256, 512, ctypes.byref(p), None, vp(16), w32 - 1, None, None) == -8
    # refinement
    need = _lib.lstsq_ir_workspace_size(512, 256, p)
    assert need > w32
    info = _lib.IrInfo()
    IR = hqr_lib.hqr_lstsq_ir
    args = lambda M, N, lda, it, tol, wb: (vp(16), M, N, lda, vp(16), vp(16), None, ctypes.byref(p), None, it, tol,  # noqa: E731
                                           vp(16), wb, None, ctypes.byref(info))
    assert IR(*args(100, 200, 100, 30, 1e-12, need)) == -2
    assert IR(*args(512, 256, 500, 30, 1e-12, need)) == -4
    assert IR(*args(512, 256, 512, 0, 1e-12, need)) == -10
    assert IR(*args(512, 256, 512, 30, -1.0, need)) == -11
    assert IR(*args(512, 256, 512, 30, float("nan"), need)) == -11
    assert IR(*args(512, 256, 512, 30, 1e-12, need - 1)) == -13
    # least squares with a finished factorization: same checks as the apply entry points
    bneed = h.apply_workspace_size(256, 3, p)
    S = hqr_lib.hqr_solve
    assert S(256, 128, ctypes.byref(p), None, vp(16), w64, vp(16), 200, 3, vp(16), bneed, None) == -9
    assert S(256, 128, ctypes.byref(p), None, vp(16), w64, vp(16), 256, 0, vp(16), bneed, None) == -10
    assert S(256, 128, ctypes.byref(p), None, vp(16), h.workspace_size(256, 128, p), vp(16), 256, 3, vp(16),
             bneed - 1, None) == -12
    # exporting a batch problem's factors
    b = _lib.Batch([300, 200], [100, 200], [1, 0], p)
    E = hqr_lib.hqr_batch_export_factors
    assert E(b.handle, 2, vp(16), vp(16), 1 << 30, None) == -2
    assert E(b.handle, 0, vp(16), vp(16), h.workspace_size(300, 100, p) - 1, None) == -5
    # publishing a batch status into host memory
    P = hqr_lib.hqr_batch_publish_status
    assert P(None, vp(16), vp(16), None) == -1
    assert P(b.handle, None, vp(16), None) == -2
    assert P(b.handle, vp(16), None, None) == -3
    # exporting every problem's factors in one launch (b was never bound)
    X = hqr_lib.hqr_batch_export_all
    assert X(None, vp(16), vp(16), vp(16), None) == -1
    assert X(b.handle, vp(16), vp(16), vp(16), None) == -2
    b.close()


def test_precision_field_and_handle_argument_checks(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import _lib

    vp = ctypes.c_void_p
    # the double entry points take FP64 only; an unknown precision is a bad parameter set
    p32 = h.make_params(nb=64, precision="fp32")
    need = h.workspace_size(256, 128, h.make_params(nb=64))
    assert hqr_lib.hqr_factor(vp(16), 256, 128, 256, ctypes.byref(p32), None, vp(16), need, None, None) == -5
    bad = h.make_params(nb=64, precision=7)
    assert hqr_lib.hqr_factor(vp(16), 256, 128, 256, ctypes.byref(bad), None, vp(16), need, None, None) == -5
    with pytest.raises(h.HQRError):
        h.workspace_size(256, 128, bad)
    lneed = h.lstsq_workspace_size(256, 128, 1, h.make_params(nb=64))
    assert hqr_lib.hqr_lstsq(vp(16), 256, 128, 256, vp(16), 256, 1, ctypes.byref(p32), None, vp(16), lneed, None,
                             None) == -8
    # the tree does not depend on the precision
    assert (h.elimlist(8, 4, p32) == h.elimlist(8, 4, h.make_params(nb=64))).all()
    # handle entry points: a NULL handle and argument checks before any device work
    for name in ("hqr_factors_apply_qt", "hqr_factors_apply_q", "hqr_factors_solve"):
        fn = getattr(hqr_lib, name)
        assert fn(None, None, vp(16), 256, 1, vp(16), 1 << 20, None) == -1
    n = ctypes.c_size_t()
    assert hqr_lib.hqr_factors_apply_workspace_size(None, 1, ctypes.byref(n)) == -1
    assert hqr_lib.hqr_factors_query(None, None, None, None, None, None) == -1
    hqr_lib.hqr_factors_destroy(None)
    assert _lib.load().hqr_strerror(_lib.ERR_FACTORS).decode().startswith("the workspace does not hold")


def test_factorization_offsets_do_not_depend_on_right_hand_sides(hqr_lib):
    # a least-squares workspace holds the T factors and tiles where the apply entry points look for
    # them: its extra bytes (the right-hand-side tile columns and their counters) come after the
    # factorization's regions, so the factorization workspace is a prefix of it in size
    import paper_1110_1553_amd as h

    for (M, N, nb) in ((2100, 513, 64), (2100, 513, 256), (32768, 2048, 256), (1000, 300, 128)):
        p = h.make_params(nb=nb)
        w0 = h.workspace_size(M, N, p)
        for nrhs in (1, 3, 70, 300):
            assert h.lstsq_workspace_size(M, N, nrhs, p) > w0
