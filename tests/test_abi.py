"""C-ABI contract checks that need no GPU: the library loads, exports every
function the header declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mps_abi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


@pytest.fixture(scope="module")
def L():
    from paper_2505_06119_amd import mps
    if not os.path.exists(mps.LIB_PATH):
        from paper_2505_06119_amd import build
        build.build()
    return mps.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("mps_apply_gate", "mps_apply_layer", "qrcp_truncate", "mps_amplitude", "mps_update_bond",
                 "mps_create", "mps_destroy", "mps_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_work_size_queries(L):
    from paper_2505_06119_amd import mps
    assert mps.qrcp_work_bytes(64, 64, 32, mps.MPS_FP64) > 64 * 64 * 16
    assert mps.qrcp_work_bytes(64, 64, 32, mps.MPS_MIXED) > 64 * 64 * 8
    assert mps.qrcp_work_bytes(-1, 4, 4, mps.MPS_FP64) == -1
    assert mps.qrcp_work_bytes(4, 4, 4, 7) == -1
    assert mps.qrcp_work_bytes(4, 4, 4, mps.MPS_FP64, 5) == -1
    assert mps.qrcp_work_bytes(64, 64, 32, mps.MPS_FP64, mps.MPS_PIVOT_LEARNED) > \
        mps.qrcp_work_bytes(64, 64, 32, mps.MPS_FP64)
    assert mps.mps_update_work_bytes(8, 8, 8, 8, mps.MPS_FP64) > 0
    assert mps.mps_update_work_bytes(0, 8, 8, 8, mps.MPS_FP64) == -1
    cfg = mps.Config(12, 32, mps.MPS_FP64, 0, 1.01, 64, 0, 0, None, 0, 0)
    assert L.mps_arena_bytes(ctypes.byref(cfg)) > 0
    bad = mps.Config(1, 32, mps.MPS_FP64, 0, 1.01, 64, 0, 0, None, 0, 0)
    assert L.mps_arena_bytes(ctypes.byref(bad)) == -1


def test_einval_on_host(L):
    from paper_2505_06119_amd import mps
    z = ctypes.c_void_p(0)
    Q, LRN = mps.MPS_PIVOT_QRCP, mps.MPS_PIVOT_LEARNED

    def q(m, n, k, prec, mode, lc, A, lda, ldq, ldr, work, wb):
        return L.qrcp_truncate(m, n, k, prec, mode, lc, A, lda, A, ldq, A, ldr, A, A, None, None, None, None,
                               work, wb, z)

    st = q(0, 4, 4, mps.MPS_FP64, Q, None, z, 4, 4, 4, z, 0)
    assert st == 1 and "m, n, k_max" in mps.last_error()
    assert q(4, 4, 4, 9, Q, None, z, 4, 4, 4, z, 0) == 1
    st = q(4, 4, 4, mps.MPS_FP64, 7, None, z, 4, 4, 4, z, 0)
    assert st == 1 and "pivot mode" in mps.last_error()
    st = q(4, 4, 4, mps.MPS_FP64, LRN, None, z, 4, 4, 4, z, 0)
    assert st == 1 and "learned" in mps.last_error()
    st = q(4, 4, 4, mps.MPS_FP64, Q, None, z, 4, 4, 4, z, 0)
    assert st == 1 and "null" in mps.last_error()
    p = ctypes.c_void_p(256)       # never dereferenced: leading dimensions are checked first
    st = q(8, 4, 4, mps.MPS_FP64, Q, None, p, 4, 8, 4, p, 1 << 20)
    assert st == 1 and "leading dimension" in mps.last_error()
    assert q(8, 4, 4, mps.MPS_FP64, Q, None, p, 8, 8, 4, p, 16) == 2        # workspace too small
    lc = mps.LearnedCfg(256, 16, 0, 1, 1.01)
    need_q = L.qrcp_work_bytes(8, 4, 4, mps.MPS_FP64, Q)
    st = q(8, 4, 4, mps.MPS_FP64, LRN, ctypes.byref(lc), p, 8, 8, 4, p, need_q)
    assert st == 2 and "need" in mps.last_error()                        # learned needs more
    g = (ctypes.c_double * 32)()
    st = L.mps_update_bond(0, 4, 4, 4, 0, 0, p, p, g, p, p, 1, None, None, p, 1 << 30, z)
    assert st == 1
    st = L.mps_update_bond(4, 4, 4, 4, 0, 1, p, p, g, p, p, 1, None, None, p, 1 << 30, z)
    assert st == 1 and "learned" in mps.last_error()
    bad_cfg = mps.LearnedCfg(256, 0, 0, 1, 1.01)             # sketch_rows = 0
    st = L.mps_update_bond(4, 4, 4, 4, 0, 1, p, p, g, p, p, 1, ctypes.byref(bad_cfg), None, p, 1 << 30, z)
    assert st == 1
    assert L.pivnet_work_bytes(8, 8, 0, 0) == -1
    assert L.pivnet_forward(None, None, 4, None, z) == 1
    assert L.pivnet_adam(p, p, p, p, 0, ctypes.c_float(1e-3), z) == 1
    g[3] = float("nan")
    st = L.mps_update_bond(4, 4, 4, 4, 0, 0, p, p, g, p, p, 1, None, None, p, 1 << 30, z)
    assert st == 4
    h = ctypes.c_void_p()
    bad = mps.Config(1, 8, 0, 0, 1.01, 64, 0, 0, None, 0, 0)
    assert L.mps_create(ctypes.byref(bad), p, 1 << 30, z, ctypes.byref(h)) == 1
    good = mps.Config(4, 8, 0, 0, 1.01, 64, 0, 0, None, 0, 0)
    assert L.mps_create(ctypes.byref(good), p, 16, z, ctypes.byref(h)) == 2
    bad_net = mps.Config(4, 8, 0, mps.MPS_PIVOT_LEARNED, 1.01, 0, 0, 0, p, 0, 0)    # sketch_rows = 0
    assert L.mps_create(ctypes.byref(bad_net), p, 1 << 30, z, ctypes.byref(h)) == 1
    assert "learned" in mps.last_error()
    assert L.mps_apply_gate(None, 0, g, None) == 1
    assert L.mps_destroy(None) == 1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2505_06119_amd import mps
    monkeypatch.setattr(mps, "_lib", None)
    monkeypatch.setattr(mps, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        mps.lib()


def test_small_bond_limit_validation(L):
    from paper_2505_06119_amd import mps
    for v in (-1, 65, 1 << 20):
        assert L.mps_set_small_bond_limit(v) == 1, v
        assert "mps_set_small_bond_limit" in mps.last_error()
    for v in (0, 1, 16, 64):
        assert L.mps_set_small_bond_limit(v) == 0, v


def test_set_truncation_null_context(L):
    from paper_2505_06119_amd import mps
    for mode in (0, 1, 2):
        assert L.mps_set_truncation(None, mode) == 1, mode
        assert "mps_set_truncation" in mps.last_error()


def test_tuning_validation(L):
    from paper_2505_06119_amd import mps
    for pw, win in ((12, -1), (32, 48), (32, -2), (0, 513), (128, 0)):
        assert L.mps_set_tuning(pw, win) == 1, (pw, win)
        assert "mps_set_tuning" in mps.last_error()
    for pw, win in ((16, 64), (64, 512), (0, 0), (32, 256)):
        assert L.mps_set_tuning(pw, win) == 0, (pw, win)
    assert L.mps_set_tuning(0, -1) == 0
