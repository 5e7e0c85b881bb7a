"""ctypes binding of libmpsgpu.so (declared in include/mps_abi.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors, the context arena, the
workspace) and the stream (``torch.cuda.current_stream()``).

Layouts on the device
* a matrix is column-major: a torch tensor ``M`` of shape (rows, cols) with
  strides (1, rows) -- see :func:`colmajor`;
* a site tensor A[l, s, r] lives at l + chi_l*(s + 2r): a contiguous torch
  tensor of shape (chi_r, 2, chi_l) -- see :func:`site_to_device`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpsgpu.so")

MPS_FP64, MPS_MIXED = 0, 1
MPS_PIVOT_QRCP, MPS_PIVOT_LEARNED = 0, 1
MPS_TRUNC_QRCP, MPS_TRUNC_SVD = 0, 1
STATUS = {0: "MPS_OK", 1: "MPS_EINVAL", 2: "MPS_ENOMEM", 3: "MPS_EDEVICE", 4: "MPS_ENUMERIC", 5: "MPS_ESTATE"}


class MpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class UpdateInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("trunc_err_sq", ctypes.c_double), ("norm_sq", ctypes.c_double),
                ("retained", ctypes.c_double), ("fallback", ctypes.c_int32), ("panels", ctypes.c_int32),
                ("refreshes", ctypes.c_int32), ("window_misses", ctypes.c_int32),
                ("learned_err_sq", ctypes.c_double),
                ("qrcp_err_sq", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


PIVNET_PARAMS = 97
PIVNET_FEATURES = 4


class LearnedCfg(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("sketch_rows", ctypes.c_int32), ("verify", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("fallback_ratio", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class TuneEntry(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int64), ("panel_width", ctypes.c_int32), ("qr_window", ctypes.c_int32),
                ("ms", ctypes.c_double), ("ms_default", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Config(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("chi_max", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("pivot", ctypes.c_int32), ("fallback_ratio", ctypes.c_double), ("sketch_rows", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("seed", ctypes.c_uint64), ("mlp_weights", ctypes.c_void_p),
                ("learned_verify", ctypes.c_int32), ("pad2", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmpsgpu.so; raises when it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_06119_amd.build.build()")
    # the library and torch share one HIP runtime in the process: let torch
    # bring it up first (on a host without a GPU this only reports False)
    _torch().cuda.is_available()
    L = ctypes.CDLL(LIB_PATH)
    p, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    pd, pi64 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    L.mps_last_error.restype = ctypes.c_char_p
    L.mps_last_error.argtypes = []
    L.qrcp_work_bytes.restype = i64
    L.qrcp_work_bytes.argtypes = [i64, i64, i64, i32, i32]
    L.qrcp_truncate.restype = i32
    L.qrcp_truncate.argtypes = [i64, i64, i64, i32, i32, ctypes.POINTER(LearnedCfg), p, i64, p, i64, p, i64, p,
                                p, pi64, pd, pd, ctypes.POINTER(UpdateInfo), p, i64, p]
    L.qrcp_noalloc_scratch_bytes.restype = i64
    L.qrcp_noalloc_scratch_bytes.argtypes = []
    L.qrcp_truncate_noalloc.restype = i32
    L.qrcp_truncate_noalloc.argtypes = [i64, i64, i64, i32, i32, ctypes.POINTER(LearnedCfg), p, i64, p, i64, p,
                                        i64, p, p, pi64, pd, pd, ctypes.POINTER(UpdateInfo), p]
    L.mps_update_work_bytes.restype = i64
    L.mps_update_work_bytes.argtypes = [i64, i64, i64, i64, i32, i32]
    L.mps_update_bond.restype = i32
    L.mps_update_bond.argtypes = [i64, i64, i64, i64, i32, i32, p, p, pd, p, p, ctypes.c_int,
                                  ctypes.POINTER(LearnedCfg), ctypes.POINTER(UpdateInfo), p, i64, p]
    L.mps_move_work_bytes.restype = i64
    L.mps_move_work_bytes.argtypes = [i64, i64, i64, i32, i32]
    L.mps_move_centre.restype = i32
    L.mps_move_centre.argtypes = [i64, i64, i64, i32, i32, p, p, p, p, pi64, p, i64, p]
    L.mps_theta.restype = i32
    L.mps_theta.argtypes = [i64, i64, i64, i32, p, p, pd, p, i64, p, i64, p]
    L.pivnet_work_bytes.restype = i64
    L.pivnet_work_bytes.argtypes = [i64, i64, i32, i32]
    L.pivnet_features.restype = i32
    L.pivnet_features.argtypes = [i64, i64, i32, p, i64, i32, ctypes.c_uint64, p, p, i64, p]
    L.pivnet_forward.restype = i32
    L.pivnet_forward.argtypes = [p, p, i64, p, p]
    L.pivnet_grad.restype = i32
    L.pivnet_grad.argtypes = [p, p, p, i64, p, p, i64, p]
    L.pivnet_adam.restype = i32
    L.pivnet_adam.argtypes = [p, p, p, p, i32, ctypes.c_float, p]
    L.pivnet_rank.restype = i32
    L.pivnet_rank.argtypes = [p, i64, p, p]
    L.mps_set_pivot_network.restype = i32
    L.mps_set_pivot_network.argtypes = [p, ctypes.POINTER(LearnedCfg)]
    L.mps_set_tuning.restype = i32
    L.mps_set_tuning.argtypes = [i32, i32]
    L.mps_set_panel_mode.restype = i32
    L.mps_set_panel_mode.argtypes = [i32]
    L.mps_autotune_work_bytes.restype = i64
    L.mps_autotune_work_bytes.argtypes = [i32, i32]
    L.mps_autotune.restype = i32
    L.mps_autotune.argtypes = [i32, i32, p, i64, p, ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32)]
    L.mps_clear_autotune.restype = i32
    L.mps_clear_autotune.argtypes = []
    L.mps_set_small_bond_limit.restype = i32
    L.mps_set_small_bond_limit.argtypes = [i32]
    L.mps_set_truncation.restype = i32
    L.mps_set_truncation.argtypes = [ctypes.c_void_p, i32]
    L.mps_profile.restype = i32
    L.mps_profile.argtypes = [ctypes.c_int]
    L.mps_profile_read.restype = i32
    L.mps_profile_read.argtypes = [p, i32]
    L.mps_arena_bytes.restype = i64
    L.mps_arena_bytes.argtypes = [ctypes.POINTER(Config)]
    L.mps_create.restype = i32
    L.mps_create.argtypes = [ctypes.POINTER(Config), p, i64, p, ctypes.POINTER(p)]
    L.mps_destroy.restype = i32
    L.mps_destroy.argtypes = [p]
    L.mps_apply_gate.restype = i32
    L.mps_apply_gate.argtypes = [p, i32, pd, ctypes.POINTER(UpdateInfo)]
    L.mps_apply_layer.restype = i32
    L.mps_apply_layer.argtypes = [p, i64, ctypes.POINTER(ctypes.c_int32), pd, ctypes.POINTER(UpdateInfo)]
    L.mps_amplitude.restype = i32
    L.mps_amplitude.argtypes = [p, ctypes.POINTER(ctypes.c_uint8), pd]
    L.mps_log_norm_fidelity.restype = i32
    L.mps_log_norm_fidelity.argtypes = [p, pd]
    L.mps_bond_dims.restype = i32
    L.mps_bond_dims.argtypes = [p, pi64]
    L.mps_centre.restype = i32
    L.mps_centre.argtypes = [p, ctypes.POINTER(ctypes.c_int32)]
    L.mps_get_site.restype = i32
    L.mps_get_site.argtypes = [p, i32, p, i64]
    L.mps_apply_mpo.restype = i32
    L.mps_apply_mpo.argtypes = [p, i32, i32, ctypes.POINTER(ctypes.c_int32), pd, pd]
    L.mps_load_state.restype = i32
    L.mps_load_state.argtypes = [p, pi64, pd]
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise MpsError(status, lib().mps_last_error().decode())


def last_error() -> str:
    return lib().mps_last_error().decode()


# --- device helpers ----------------------------------------------------------------

def _torch():
    import torch
    return torch


def cdtype(prec: int):
    torch = _torch()
    return torch.complex128 if prec == MPS_FP64 else torch.complex64


def np_cdtype(prec: int):
    return np.complex128 if prec == MPS_FP64 else np.complex64


def stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def colmajor(a: np.ndarray, prec: int, device="cuda"):
    """Upload a (rows, cols) matrix as a column-major device tensor."""
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a).T.astype(np_cdtype(prec))))
    return t.to(device).t()


def empty_colmajor(rows: int, cols: int, prec: int, device="cuda"):
    torch = _torch()
    return torch.empty((cols, rows), dtype=cdtype(prec), device=device).t()


def site_to_device(a: np.ndarray, prec: int, device="cuda"):
    """Site [l, s, r] (numpy) -> contiguous device tensor of shape (chi_r, 2, chi_l)."""
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).transpose(2, 1, 0).astype(np_cdtype(prec)))).to(device)


def site_from_device(t, chi_l: int, chi_r: int) -> np.ndarray:
    """Inverse of site_to_device; returns complex128 [l, s, r]."""
    arr = t.reshape(-1)[: chi_l * 2 * chi_r].reshape(chi_r, 2, chi_l).cpu().numpy()
    return np.ascontiguousarray(arr.transpose(2, 1, 0)).astype(np.complex128)


def gate_buffer(g: np.ndarray):
    g = np.ascontiguousarray(np.asarray(g, dtype=np.complex128).reshape(4, 4))
    buf = np.ascontiguousarray(g.view(np.float64).reshape(-1))
    return buf, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# --- stateless calls -------------------------------------------------------------------

def set_tuning(panel_width: int = 0, qr_window: int = -1):
    """Process-wide pivoted-QR tuning (mps_set_tuning): panel width (0 = automatic)
    and candidate-window width (-1 = automatic, 0 = off)."""
    _check(lib().mps_set_tuning(panel_width, qr_window))


def set_panel_mode(mode: int) -> None:
    """Process-wide (mps_set_panel_mode): 0 = one launch per pivot step,
    1 = a panel's pivots from its window's Gram matrix."""
    _check(lib().mps_set_panel_mode(mode))


def autotune(chi_max: int, prec: int, stream=None) -> list:
    """Tune the pivoted-QR tiles per bond bucket up to chi_max (mps_autotune);
    returns the table as a list of dicts.  Process-wide from then on."""
    torch = _torch()
    wb = int(lib().mps_autotune_work_bytes(chi_max, prec))
    if wb < 0:
        raise MpsError(1, f"mps_autotune_work_bytes({chi_max}, {prec}) rejected its arguments")
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    table = (TuneEntry * 8)()
    n = ctypes.c_int32(0)
    _check(lib().mps_autotune(chi_max, prec, _ptr(work), wb, stream if stream is not None else stream_ptr(),
                              table, 8, ctypes.byref(n)))
    return [table[i].as_dict() for i in range(n.value)]


def clear_autotune():
    _check(lib().mps_clear_autotune())


def set_small_bond_limit(max_dim: int = 64):
    """Process-wide limit of the one-launch small-bond chains
    (mps_set_small_bond_limit; 0 = off)."""
    _check(lib().mps_set_small_bond_limit(max_dim))


def qrcp_work_bytes(m: int, n: int, k_max: int, prec: int, mode: int = MPS_PIVOT_QRCP) -> int:
    return int(lib().qrcp_work_bytes(m, n, k_max, prec, mode))


def qrcp_truncate(A, k_max: int, prec: int, work=None, stream=None, learned=None) -> dict:
    """Pivoted QR of the column-major device matrix A (m x n), k = min(k_max, m, n).

    learned: a LearnedCfg (see learned_cfg) to factorise with the proposed
    column order (MPS_PIVOT_LEARNED); "piv" is then the proposed order when
    the proposal was accepted (info["fallback"] == 0)."""
    torch = _torch()
    mode = MPS_PIVOT_QRCP if learned is None else MPS_PIVOT_LEARNED
    m, n = A.shape
    k = max(0, min(k_max, m, n))
    lda = A.stride(1) if n > 1 else max(m, 1)
    if A.stride(0) != 1:
        raise ValueError("A must be column-major (stride (1, lda))")
    Q = empty_colmajor(m, k, prec)
    R = empty_colmajor(k, n, prec)
    piv = torch.empty(n, dtype=torch.int32, device=A.device)
    diag = torch.empty(max(k, 1), dtype=torch.float64, device=A.device)
    wb = qrcp_work_bytes(m, n, k_max, prec, mode)
    if work is None:
        work = torch.empty(max(wb, 1), dtype=torch.uint8, device=A.device)
    kout = ctypes.c_int64(0)
    err = ctypes.c_double(0)
    afro = ctypes.c_double(0)
    info = UpdateInfo()
    _check(lib().qrcp_truncate(m, n, k_max, prec, mode, ctypes.byref(learned) if learned is not None else None,
                               _ptr(A), lda, _ptr(Q), m, _ptr(R), max(k, 1), _ptr(piv), _ptr(diag),
                               ctypes.byref(kout), ctypes.byref(err), ctypes.byref(afro), ctypes.byref(info),
                               _ptr(work), work.numel(), stream if stream is not None else stream_ptr()))
    return {"Q": Q, "RPt": R, "piv": piv, "diagR": diag[:k], "k": int(kout.value), "err": float(err.value),
            "a_fro": float(afro.value), "info": info.as_dict()}


def qrcp_truncate_noalloc(A, k_max: int, prec: int, stream=None, learned=None) -> dict:
    """qrcp_truncate_noalloc: the same factorisation with the library's static
    device scratch instead of a workspace (the outputs are still allocated
    here, by torch)."""
    torch = _torch()
    mode = MPS_PIVOT_QRCP if learned is None else MPS_PIVOT_LEARNED
    m, n = A.shape
    k = max(0, min(k_max, m, n))
    lda = A.stride(1) if n > 1 else max(m, 1)
    if A.stride(0) != 1:
        raise ValueError("A must be column-major (stride (1, lda))")
    Q = empty_colmajor(m, k, prec)
    R = empty_colmajor(k, n, prec)
    piv = torch.empty(n, dtype=torch.int32, device=A.device)
    diag = torch.empty(max(k, 1), dtype=torch.float64, device=A.device)
    kout = ctypes.c_int64(0)
    err = ctypes.c_double(0)
    afro = ctypes.c_double(0)
    info = UpdateInfo()
    _check(lib().qrcp_truncate_noalloc(m, n, k_max, prec, mode,
                                       ctypes.byref(learned) if learned is not None else None, _ptr(A), lda, _ptr(Q),
                                       m, _ptr(R), max(k, 1), _ptr(piv), _ptr(diag), ctypes.byref(kout),
                                       ctypes.byref(err), ctypes.byref(afro), ctypes.byref(info),
                                       stream if stream is not None else stream_ptr()))
    return {"Q": Q, "RPt": R, "piv": piv, "diagR": diag[:k], "k": int(kout.value), "err": float(err.value),
            "a_fro": float(afro.value), "info": info.as_dict()}


def mps_update_work_bytes(chi_l, chi_m, chi_r, chi_cap, prec, pivot=MPS_PIVOT_QRCP) -> int:
    return int(lib().mps_update_work_bytes(chi_l, chi_m, chi_r, chi_cap, prec, pivot))


def learned_cfg(params, sketch_rows=64, verify=False, seed=1234, fallback_ratio=1.01) -> LearnedCfg:
    """mps_learned_cfg for a device float32 parameter tensor of PIVNET_PARAMS entries.
    verify: False (certificate), True (verification against plain pivoted QR)
    or "trust" (the proposal is kept unchecked)."""
    v = 2 if verify == "trust" else (1 if verify else 0)
    return LearnedCfg(params.data_ptr(), int(sketch_rows), v, int(seed), float(fallback_ratio))


def mps_update_bond(A, B, g, chi_l, chi_m, chi_r, chi_cap, prec, renormalize=True, A_out=None, B_out=None,
                    work=None, pivot=MPS_PIVOT_QRCP, stream=None, info=None, learned=None) -> dict:
    """Two-site update on device sites A (chi_l x 2 x chi_m) and B (chi_m x 2 x chi_r).

    learned: a LearnedCfg (see learned_cfg) to use the learned pivot order."""
    if learned is not None:
        pivot = MPS_PIVOT_LEARNED
    torch = _torch()
    k = min(chi_cap, 2 * chi_l, 2 * chi_r)
    if A_out is None:
        A_out = torch.empty((k, 2, chi_l), dtype=cdtype(prec), device=A.device)
    if B_out is None:
        B_out = torch.empty((chi_r, 2, k), dtype=cdtype(prec), device=A.device)
    if work is None:
        wb = mps_update_work_bytes(chi_l, chi_m, chi_r, chi_cap, prec, pivot)
        work = torch.empty(max(wb, 1), dtype=torch.uint8, device=A.device)
    gbuf, gp = gate_buffer(g)
    if info is None:
        info = UpdateInfo()
    _check(lib().mps_update_bond(chi_l, chi_m, chi_r, chi_cap, prec, pivot, _ptr(A), _ptr(B), gp, _ptr(A_out),
                                 _ptr(B_out), 1 if renormalize else 0,
                                 ctypes.byref(learned) if learned is not None else None, ctypes.byref(info),
                                 _ptr(work), work.numel(), stream if stream is not None else stream_ptr()))
    del gbuf
    return {"A": A_out, "B": B_out, "info": info.as_dict(), "k": int(info.k)}


def mps_move_centre(A, B, chi_l, chi_c, chi_r, prec, direction, A_out=None, B_out=None, work=None,
                    stream=None) -> dict:
    """One centre move (mps_move_centre) on device sites A (chi_l x 2 x chi_c)
    and B (chi_c x 2 x chi_r); direction +1 (QR of A) or -1 (LQ of B)."""
    torch = _torch()
    cd = cdtype(prec)
    k = min(2 * chi_l, chi_c) if direction > 0 else min(chi_c, 2 * chi_r)
    if A_out is None:
        A_out = torch.empty((k, 2, chi_l), dtype=cd, device=A.device)      # chi_l x 2 x k
    if B_out is None:
        B_out = torch.empty((chi_r, 2, k), dtype=cd, device=A.device)
    if work is None:
        work = torch.empty(max(1, int(lib().mps_move_work_bytes(chi_l, chi_c, chi_r, prec, direction))),
                           dtype=torch.uint8, device=A.device)
    kout = ctypes.c_int64(0)
    _check(lib().mps_move_centre(chi_l, chi_c, chi_r, prec, direction, _ptr(A), _ptr(B), _ptr(A_out), _ptr(B_out),
                                 ctypes.byref(kout), _ptr(work), work.numel(),
                                 stream if stream is not None else stream_ptr()))
    return {"A": A_out, "B": B_out, "k": int(kout.value)}


def mps_theta(A, B, g, chi_l, chi_m, chi_r, prec, work=None, stream=None):
    """theta = G (A B) as a column-major (2 chi_l) x (2 chi_r) device matrix."""
    torch = _torch()
    theta = empty_colmajor(2 * chi_l, 2 * chi_r, prec)
    if work is None:
        work = torch.empty(max(mps_update_work_bytes(chi_l, chi_m, chi_r, 1, prec), 1), dtype=torch.uint8,
                           device=A.device)
    gbuf, gp = gate_buffer(g)
    _check(lib().mps_theta(chi_l, chi_m, chi_r, prec, _ptr(A), _ptr(B), gp, _ptr(theta), 2 * chi_l, _ptr(work),
                           work.numel(), stream if stream is not None else stream_ptr()))
    del gbuf
    return theta


# --- pivot-proposal network ------------------------------------------------------------

def pivnet_features(theta, prec, sketch_rows=64, seed=1234, work=None, stream=None):
    """Sketch features (n x 4 float32) of a column-major device matrix."""
    torch = _torch()
    m, n = theta.shape
    ld = theta.stride(1) if n > 1 else max(m, 1)
    phi = torch.empty((n, PIVNET_FEATURES), dtype=torch.float32, device=theta.device)
    if work is None:
        work = torch.empty(int(lib().pivnet_work_bytes(m, n, sketch_rows, prec)), dtype=torch.uint8,
                           device=theta.device)
    _check(lib().pivnet_features(m, n, prec, _ptr(theta), ld, sketch_rows, seed, _ptr(phi), _ptr(work),
                                 work.numel(), stream if stream is not None else stream_ptr()))
    return phi


def pivnet_forward(params, phi, stream=None):
    torch = _torch()
    n = phi.shape[0]
    scores = torch.empty(n, dtype=torch.float32, device=phi.device)
    _check(lib().pivnet_forward(_ptr(params), _ptr(phi), n, _ptr(scores),
                                stream if stream is not None else stream_ptr()))
    return scores


def pivnet_grad(params, phi, labels, stream=None):
    """(gradient of the mean logistic loss, loss) on the device."""
    torch = _torch()
    n = phi.shape[0]
    grad = torch.empty(PIVNET_PARAMS + 1, dtype=torch.float32, device=phi.device)
    work = torch.empty(4 * (PIVNET_PARAMS + 1) * ((n + 255) // 256), dtype=torch.uint8, device=phi.device)
    _check(lib().pivnet_grad(_ptr(params), _ptr(phi), _ptr(labels), n, _ptr(grad), _ptr(work), work.numel(),
                             stream if stream is not None else stream_ptr()))
    return grad


def pivnet_adam(params, grad, m1, m2, t, lr, stream=None):
    _check(lib().pivnet_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(t), float(lr),
                             stream if stream is not None else stream_ptr()))


def pivnet_rank(scores, stream=None):
    torch = _torch()
    n = scores.shape[0]
    order = torch.empty(n, dtype=torch.int32, device=scores.device)
    _check(lib().pivnet_rank(_ptr(scores), n, _ptr(order), stream if stream is not None else stream_ptr()))
    return order


# --- stateful MPS ------------------------------------------------------------------------

class MPS:
    """An MPS held by the library (mps_create ... mps_destroy)."""

    def __init__(self, n_sites: int, chi_max: int, prec: int = MPS_FP64, pivot: int = MPS_PIVOT_QRCP,
                 device="cuda", learned: LearnedCfg | None = None):
        """learned: optional LearnedCfg whose network and acceptance rule are set
        at creation (mps_config.mlp_weights); otherwise set_pivot_network."""
        torch = _torch()
        if learned is not None:
            self.cfg = Config(n_sites, chi_max, prec, MPS_PIVOT_LEARNED, learned.fallback_ratio, learned.sketch_rows,
                              0, learned.seed, learned.params, learned.verify, 0)
            self._lcfg = learned
        else:
            self.cfg = Config(n_sites, chi_max, prec, pivot, 1.01, 64, 0, 0, None, 0, 0)
        nbytes = int(lib().mps_arena_bytes(ctypes.byref(self.cfg)))
        if nbytes < 0:
            raise MpsError(1, "invalid configuration")
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        _check(lib().mps_create(ctypes.byref(self.cfg), _ptr(self.arena), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))
        self.n = n_sites
        self.prec = prec

    def close(self):
        if self._h:
            lib().mps_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_truncation(self, mode: int):
        """MPS_TRUNC_QRCP or MPS_TRUNC_SVD for the later updates (mps_set_truncation)."""
        _check(lib().mps_set_truncation(self._h, mode))

    def set_pivot_network(self, cfg: LearnedCfg):
        self._lcfg = cfg
        _check(lib().mps_set_pivot_network(self._h, ctypes.byref(cfg)))

    def apply_gate(self, i: int, g) -> dict:
        info = UpdateInfo()
        gbuf, gp = gate_buffer(g)
        _check(lib().mps_apply_gate(self._h, i, gp, ctypes.byref(info)))
        del gbuf
        return info.as_dict()

    def apply_layer(self, layer) -> list:
        n = len(layer)
        idx = (ctypes.c_int32 * max(n, 1))(*[int(i) for i, _ in layer])
        gs = np.ascontiguousarray(np.stack([np.asarray(g, dtype=np.complex128).reshape(4, 4) for _, g in layer])
                                  if n else np.zeros((1, 4, 4), np.complex128))
        gflat = np.ascontiguousarray(gs.view(np.float64).reshape(-1))
        infos = (UpdateInfo * max(n, 1))()
        _check(lib().mps_apply_layer(self._h, n, idx, gflat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     infos))
        return [infos[t].as_dict() for t in range(n)]

    def apply_layers(self, layers):
        out = []
        for layer in layers:
            out += self.apply_layer(sorted(layer, key=lambda ig: ig[0]))
        return out

    def apply_mpo(self, first: int, ws) -> float:
        """MPO on sites first .. first + len(ws) - 1 (mps_apply_mpo): ws[t] is
        W_t[a, s', s, b] with shape (m_t, 2, 2, m_{t+1}), m_0 = m_len = 1.
        Returns the log of the norm fidelity this application retained."""
        ws = [np.asarray(w, dtype=np.complex128) for w in ws]
        md = [ws[0].shape[0]] + [w.shape[3] for w in ws]
        for t, w in enumerate(ws):
            if w.ndim != 4 or w.shape[1:3] != (2, 2) or w.shape[0] != md[t]:
                raise ValueError(f"MPO site {t} has shape {w.shape}")
        # a + m_t (s' + 2 (s + 2 b)): a fastest, i.e. Fortran order of [a, s', s, b]
        flat = np.concatenate([w.reshape(-1, order="F") for w in ws])
        buf = np.ascontiguousarray(flat.view(np.float64))
        mdims = (ctypes.c_int32 * len(md))(*md)
        out = ctypes.c_double(0)
        _check(lib().mps_apply_mpo(self._h, int(first), len(ws), mdims,
                                   buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(out)))
        return float(out.value)

    def load_state(self, sites):
        """Replace the state by the sites [l, s, r] (mps_load_state): right-
        canonical, centre 0, normalised, norm fidelity 1."""
        sites = [np.asarray(a, dtype=np.complex128) for a in sites]
        if len(sites) != self.n:
            raise ValueError("one site per qubit")
        dims = [sites[0].shape[0]] + [a.shape[2] for a in sites]
        # entry (l, s, r) at l + chi_l (s + 2 r): Fortran order of [l, s, r]
        flat = np.concatenate([a.reshape(-1, order="F") for a in sites])
        buf = np.ascontiguousarray(flat.view(np.float64))
        d = (ctypes.c_int64 * len(dims))(*dims)
        _check(lib().mps_load_state(self._h, d, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def amplitude(self, bits) -> complex:
        b = (ctypes.c_uint8 * self.n)(*[int(x) for x in bits])
        out = (ctypes.c_double * 2)()
        _check(lib().mps_amplitude(self._h, b, out))
        return complex(out[0], out[1])

    def log_norm_fidelity(self) -> float:
        v = ctypes.c_double(0)
        _check(lib().mps_log_norm_fidelity(self._h, ctypes.byref(v)))
        return float(v.value)

    def bond_dims(self) -> list:
        dims = (ctypes.c_int64 * (self.n + 1))()
        _check(lib().mps_bond_dims(self._h, dims))
        return [int(x) for x in dims]

    def centre(self) -> int:
        v = ctypes.c_int32(0)
        _check(lib().mps_centre(self._h, ctypes.byref(v)))
        return int(v.value)

    def site(self, j: int) -> np.ndarray:
        """Site j as a complex128 numpy array [l, s, r] (normalised state)."""
        torch = _torch()
        dims = self.bond_dims()
        chl, chr_ = dims[j], dims[j + 1]
        t = torch.empty((chr_, 2, chl), dtype=cdtype(self.prec), device=self.arena.device)
        _check(lib().mps_get_site(self._h, j, _ptr(t), t.numel() * t.element_size()))
        return site_from_device(t, chl, chr_)

    def sites(self) -> list:
        return [self.site(j) for j in range(self.n)]
