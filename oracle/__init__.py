"""Plain FP64 CPU oracle for the two-site MPS gate update -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2505_06119_amd``) and never imports it; inputs come from the seeded
generators in ``paper_2505_06119_amd.synth`` and are passed in as arrays.

Pieces and the passages they follow (arXiv 2505.06119):

* ``theta``             -- Sec. III-B.1 bond contraction and Sec. III-C.2
  tensor application: the two sites are contracted over their shared bond and
  the gate over the two physical indices.
* ``qrcp``              -- Table III, QR with pivoting M = Q R P^T; the greedy
  definition with exact residual norms, in plain C (``qrcp_oracle.c``), with
  the relative margin between the two largest residual norms at every step.
* ``known_order_qr``, ``certificate``, ``learned_update`` -- the learned pivot
  proposal's factorisation and acceptance (an addition of this library, not of
  the paper): Householder QR with a given column order, the truncation error
  of the column set it selects, and the two acceptance rules with the plain
  pivoted-QR fallback.
* ``two_site_update``   -- Sec. III-C.2: contract, truncated pivoted-QR
  decomposition, split back into two sites; with ``truncation="svd"`` the
  truncated decomposition is the SVD of Table III (M = U S V^dagger), the
  Schmidt decomposition of Sec. II-B, keeping the k largest singular values.
* ``MPS``               -- Sec. III-C.1 canonicalisation (QR / LQ moves of the
  orthogonality centre) and Sec. III-C.2 application of two-site gates; the
  state is kept unnormalised so that ``norm_fidelity`` is the paper's
  norm fidelity <Psi_T|Psi_T> (Sec. III-E) by its definition.
* ``MPS.apply_mpo``     -- Sec. III-C.3 MPO application by zip-up, each
  site's contraction truncated by pivoted QR (Table III); ``mpo_operator``
  and ``apply_mpo_dense`` give the dense operator for pins.
* ``amplitude``         -- Eq. (2): product of the site matrices selected by
  the bits.
* ``overlap``           -- Sec. III-E overlap fidelity, by transfer matrices.
* ``statevector`` / ``brute_force`` / ``brute_force_ops`` -- Sec. II-A
  statevector and gates (on neighbouring chain sites, or on any pair of
  logical qubits), for exact comparison on small registers.

Where the paper is silent the oracle takes these readings: site 0 is the most
significant qubit; the gate's row index is 2a'+b' with a on the lower site;
theta's column index is 2r + b' (the right site's physical index runs
fastest), and equal residual norms go to the smallest such column, where
"equal" means equal after rounding the FP64 squared norms to 40 significant
bits; the truncation rank
is k = min(chi_cap, m, n) with no tolerance cut-off; the orthogonality centre
is moved to site i (or i+1 when it lies right of i) before each update and the
split leaves Q on the left site.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "qrcp_oracle.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.orc_qrcp.restype = ctypes.c_int
        lib.orc_qrcp.argtypes = [i64, i64, i64, ctypes.c_int, p, i64, p, i64, p, i64,
                                 p, p, p, p, p]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


# --- factorisation -------------------------------------------------------------

def qrcp(a: np.ndarray, kmax: int, pivoting: bool = True) -> dict:
    """Greedy column-pivoted Householder QR of ``a`` stopped after k steps.

    Returns a dict with Q (m x k), R (k x n, pivoted column order), piv (n),
    diagR (k), err (||R22||_F), k, and gaps (k): the relative margin
    (nu_1 - nu_2) / nu_1 between the two largest squared residual norms at each
    pivoting step (1 without pivoting).  See ``qrcp_oracle.c``."""
    lib = _load()
    a = np.asfortranarray(a, dtype=np.complex128)
    m, n = a.shape
    k = max(0, min(int(kmax), m, n))
    q = np.zeros((m, k), dtype=np.complex128, order="F")
    r = np.zeros((k, n), dtype=np.complex128, order="F")
    piv = np.zeros(n, dtype=np.int32)
    diag = np.zeros(max(k, 1), dtype=np.float64)
    err = np.zeros(1, dtype=np.float64)
    kout = np.zeros(1, dtype=np.int64)
    gaps = np.ones(max(k, 1), dtype=np.float64)
    rc = lib.orc_qrcp(m, n, int(kmax), 1 if pivoting else 0,
                      a.ctypes.data, max(m, 1), q.ctypes.data, max(m, 1),
                      r.ctypes.data, max(k, 1), piv.ctypes.data, diag.ctypes.data,
                      err.ctypes.data, kout.ctypes.data, gaps.ctypes.data)
    if rc != 0:
        raise ValueError("orc_qrcp rejected its arguments")
    return {"Q": q, "R": r, "piv": piv.astype(np.int64), "diagR": diag[:k],
            "err": float(err[0]), "k": int(kout[0]), "gaps": gaps[:k]}


def r_unpivot(r: np.ndarray, piv: np.ndarray) -> np.ndarray:
    """R P^T: column j of R goes back to original column piv[j]."""
    out = np.empty_like(r)
    out[:, piv] = r
    return out


# --- learned pivot proposal: factorisation with a given order, acceptance ----

def known_order_qr(a: np.ndarray, order, kmax: int) -> dict:
    """Householder QR of ``a`` with its columns taken in the given order (no
    pivot search), stopped after k = min(kmax, m, n) steps.

    ``order`` lists every column once; its first k entries form the selected
    set S.  Returns the same fields as ``qrcp`` (piv = order) plus err =
    ||R22||_F, which equals ||(I - Pi_S) a||_F, the distance of ``a`` from
    the span of its columns S."""
    order = np.asarray(order, dtype=np.int64)
    n = a.shape[1]
    if sorted(order.tolist()) != list(range(n)):
        raise ValueError("order must be a permutation of the columns")
    f = qrcp(np.asarray(a, dtype=np.complex128)[:, order], kmax, pivoting=False)
    f["piv"] = order.copy()
    return f


def residual_norms(a: np.ndarray, q: np.ndarray, cols) -> np.ndarray:
    """Euclidean norms of the columns ``cols`` of (I - Q Q^H) a."""
    x = np.asarray(a, dtype=np.complex128)[:, np.asarray(cols, dtype=np.int64)]
    return np.linalg.norm(x - q @ (q.conj().T @ x), axis=0)


def certificate(a: np.ndarray, f: dict) -> bool:
    """Acceptance without a reference factorisation: every unselected column's
    residual norm is at most the smallest |R_jj| of the selected ones, the
    inequality plain pivoted QR satisfies by construction."""
    k = f["k"]
    rest = f["piv"][k:]
    if k == 0 or len(rest) == 0:
        return True
    return float(np.max(residual_norms(a, f["Q"], rest))) <= float(np.min(np.abs(f["diagR"])))


def learned_update(a: np.ndarray, order, kmax: int, ratio: float = 1.01, verify: bool = True) -> dict:
    """The learned path's decision for one matrix: factorise with the proposed
    order, then keep that factorisation if it passes, else fall back to plain
    pivoted QR.  verify=True keeps it when its error is at most ``ratio``
    times plain pivoted QR's; verify=False applies ``certificate``.  Returns
    the kept factorisation with ``accepted``, ``err_s`` (the proposal's error)
    and ``err_q`` (plain pivoted QR's, when it ran)."""
    fs = known_order_qr(a, order, kmax)
    fq = qrcp(a, kmax) if verify else None
    if verify:
        accepted = fs["err"] <= ratio * fq["err"]
    else:
        accepted = certificate(a, fs)
    if not accepted and fq is None:
        fq = qrcp(a, kmax)
    out = dict(fs if accepted else fq)
    out.update(accepted=bool(accepted), err_s=fs["err"], err_q=None if fq is None else fq["err"])
    return out


# --- two-site update -----------------------------------------------------------

def theta(a: np.ndarray, b: np.ndarray, g: np.ndarray) -> np.ndarray:
    """theta[(l,a'),(b',r)] = sum_{a,b} G[a'b',ab] sum_m A[l,a,m] B[m,b,r].

    Returned as a (2*chi_l) x (2*chi_r) matrix with row index 2*l + a' and
    column index 2*r + b'.  The column index is what "smallest original
    column" refers to when pivoted QR breaks a tie."""
    chi_l, chi_r = a.shape[0], b.shape[2]
    t0 = np.tensordot(a, b, axes=(2, 0))                 # [l, a, b, r]
    g4 = np.asarray(g, dtype=np.complex128).reshape(2, 2, 2, 2)
    t = np.einsum("xyab,labr->lxry", g4, t0)
    return t.reshape(2 * chi_l, 2 * chi_r)


def split_right(rp: np.ndarray, chi_r: int) -> np.ndarray:
    """The right site [k, b, r] from a k x (2 chi_r) factor with column 2r + b."""
    k = rp.shape[0]
    return np.ascontiguousarray(rp.reshape(k, chi_r, 2).transpose(0, 2, 1))


def svd_truncate(th: np.ndarray, kmax: int) -> dict:
    """Truncated SVD (Table III, M = U S V^dagger): the k = min(kmax, m, n)
    largest singular values.  Left factor U_k (orthonormal columns), right
    factor S_k V_k^dagger, err = (sum of the discarded s_i^2)^(1/2)."""
    m, n = th.shape
    k = min(int(kmax), m, n)
    u, sv, vh = np.linalg.svd(th, full_matrices=False)
    return {"U": u[:, :k], "SVh": sv[:k, None] * vh[:k], "s": sv, "k": k,
            "err": float(np.sqrt(np.sum(sv[k:] ** 2)))}


def two_site_update(a: np.ndarray, b: np.ndarray, g: np.ndarray, chi_cap: int, truncation: str = "qrcp") -> dict:
    """Contract, factorise by truncated pivoted QR, split (Sec. III-C.2).

    The new left site is Q_k reshaped (chi_l, 2, k); the new right site is
    R_k P^T reshaped (k, 2, chi_r).  With truncation="svd" they are U_k and
    S_k V_k^dagger.  Nothing is renormalised."""
    chi_l, chi_r = a.shape[0], b.shape[2]
    th = theta(a, b, g)
    if truncation == "svd":
        f = svd_truncate(th, chi_cap)
        k = f["k"]
        return {"A": np.ascontiguousarray(f["U"].reshape(chi_l, 2, k)),
                "B": split_right(f["SVh"], chi_r), "k": k, "err": f["err"],
                "norm2": float(np.vdot(th, th).real), "theta": th, "s": f["s"]}
    if truncation != "qrcp":
        raise ValueError(f"unknown truncation {truncation!r}")
    f = qrcp(th, chi_cap, pivoting=True)
    k = f["k"]
    a2 = f["Q"].reshape(chi_l, 2, k)
    rp = r_unpivot(f["R"], f["piv"])
    return {"A": np.ascontiguousarray(a2), "B": split_right(rp, chi_r), "k": k,
            "err": f["err"], "norm2": float(np.vdot(th, th).real), "theta": th,
            "piv": f["piv"], "diagR": f["diagR"], "gaps": f["gaps"]}


class MPS:
    """Matrix product state with sites [l, s, r] (Eq. (2)), kept unnormalised."""

    def __init__(self, sites, chi_cap: int, centre: int = 0, truncation: str = "qrcp"):
        self.sites = [np.array(s, dtype=np.complex128) for s in sites]
        self.chi_cap = int(chi_cap)
        self.centre = int(centre)
        self.truncation = truncation
        self.history = []

    @property
    def n(self) -> int:
        return len(self.sites)

    def _move_right(self):
        c = self.centre
        a = self.sites[c]
        chi_l, _, chi_r = a.shape
        f = qrcp(a.reshape(2 * chi_l, chi_r), min(2 * chi_l, chi_r), pivoting=False)
        k = f["k"]
        self.sites[c] = f["Q"].reshape(chi_l, 2, k)
        self.sites[c + 1] = np.tensordot(f["R"], self.sites[c + 1], axes=(1, 0))
        self.centre = c + 1

    def _move_left(self):
        c = self.centre
        a = self.sites[c]
        chi_l, _, chi_r = a.shape
        # LQ of the chi_l x (2 chi_r) matrix as the QR of its conjugate transpose
        f = qrcp(a.reshape(chi_l, 2 * chi_r).conj().T, min(chi_l, 2 * chi_r), pivoting=False)
        k = f["k"]
        self.sites[c] = np.ascontiguousarray(f["Q"].conj().T).reshape(k, 2, chi_r)
        lmat = f["R"].conj().T                                   # chi_l x k
        self.sites[c - 1] = np.tensordot(self.sites[c - 1], lmat, axes=(2, 0))
        self.centre = c - 1

    def move_centre(self, target: int):
        while self.centre < target:
            self._move_right()
        while self.centre > target:
            self._move_left()

    def apply_gate(self, i: int, g: np.ndarray, chi_cap: int | None = None) -> dict:
        self.move_centre(i if self.centre <= i else i + 1)
        cap = self.chi_cap if chi_cap is None else int(chi_cap)
        u = two_site_update(self.sites[i], self.sites[i + 1], g, cap, self.truncation)
        self.sites[i], self.sites[i + 1] = u["A"], u["B"]
        self.centre = i + 1
        rec = {"i": i, "k": u["k"], "err": u["err"], "norm2": u["norm2"]}
        self.history.append(rec)
        return rec

    def apply_layers(self, layers):
        for layer in layers:
            for i, g in layer:
                self.apply_gate(i, g)

    def apply_mpo(self, first: int, ws, chi_cap: int | None = None) -> dict:
        """Zip-up application of an MPO (Sec. III-C.3) with site tensors
        ws[t][a, s', s, b] on sites first .. first + len(ws) - 1.

        With the centre at ``first``, a matrix C[l', (a, l)] is carried right:
        T[l', s', r, b] = sum C[l', a, l] A[l, s, r] W[a, s', s, b]; T as a
        (2 chi') x (m_b chi_r) matrix (row 2 l' + s', column b chi_r + r) is
        truncated by pivoted QR; Q is the new site and R P^T the next C.  At
        the last site T is the new site and the centre.  Nothing is
        renormalised, so the state's norm afterwards carries the truncation
        (the norm fidelity of a unitary MPO applied to a normalised state)."""
        self.move_centre(first)
        cap = self.chi_cap if chi_cap is None else int(chi_cap)
        c = None
        steps = []
        for t, w in enumerate(ws):
            i = first + t
            a = self.sites[i]
            chi_l, _, chi_r = a.shape
            w = np.asarray(w, dtype=np.complex128)
            ma, mb = w.shape[0], w.shape[3]
            if c is None:
                x = a[None]                                                   # [a, l', s, r], C = 1
            else:
                x = np.einsum("pal,lsr->apsr", c.reshape(c.shape[0], ma, chi_l), a)
            tt = np.einsum("apsr,atsb->ptrb", x, w)                           # [l', s', r, b]
            chip = tt.shape[0]
            if t == len(ws) - 1:
                self.sites[i] = np.ascontiguousarray(tt[:, :, :, 0])
                self.centre = i
                break
            m = tt.transpose(0, 1, 3, 2).reshape(2 * chip, mb * chi_r)
            f = qrcp(m, min(cap, 2 * chip, mb * chi_r), pivoting=True)
            k = f["k"]
            self.sites[i] = f["Q"].reshape(chip, 2, k)
            c = r_unpivot(f["R"], f["piv"])                                   # k x (m_b chi_r), columns (b, r)
            steps.append({"i": i, "k": k, "err": f["err"], "norm2": float(np.vdot(m, m).real)})
        rec = {"first": first, "steps": steps}
        self.history.append(rec)
        return rec

    def bond_dims(self):
        return [s.shape[2] for s in self.sites[:-1]]


# --- read-out ------------------------------------------------------------------

def amplitude(sites, bits) -> complex:
    """<x|Psi> = A_0[:, x_0, :] A_1[:, x_1, :] ... (Eq. (2)); site 0 is the MSB."""
    v = np.ones((1,), dtype=np.complex128)
    for s, x in zip(sites, bits):
        v = v @ s[:, int(x), :]
    return complex(v[0])


def overlap(phi_sites, psi_sites) -> complex:
    """<Phi|Psi> by left transfer matrices."""
    e = np.ones((1, 1), dtype=np.complex128)
    for p, q in zip(phi_sites, psi_sites):
        t = np.tensordot(e, q, axes=(1, 0))                     # [l', s, r]
        e = np.tensordot(p.conj(), t, axes=([0, 1], [0, 1]))    # [r', r]
    return complex(e[0, 0])


def norm_fidelity(sites) -> float:
    """Norm fidelity <Psi_T|Psi_T> (Sec. III-E) of an unnormalised state."""
    return overlap(sites, sites).real


def overlap_fidelity(exact_sv: np.ndarray, sites) -> float:
    """|<Psi_E|Psi_T>|^2 / <Psi_T|Psi_T> for a normalised exact statevector."""
    sv = statevector(sites)
    return float(abs(np.vdot(exact_sv, sv)) ** 2 / np.vdot(sv, sv).real)


def statevector(sites) -> np.ndarray:
    """Dense 2^n statevector of an MPS (site 0 = most significant bit)."""
    t = sites[0]
    for s in sites[1:]:
        t = np.tensordot(t, s, axes=(t.ndim - 1, 0))
    return t.reshape(-1)


def brute_force_ops(n: int, ops) -> np.ndarray:
    """Apply a circuit on logical qubits to |0...0> (Sec. II-A): ops are
    ("1q", q, U 2x2) or ("2q", a, b, U 4x4) with row index 2 a' + b'; qubit 0
    is the most significant bit."""
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for op in ops:
        if op[0] == "1q":
            _, q, u = op
            psi = np.moveaxis(np.tensordot(np.asarray(u, dtype=np.complex128), psi, axes=([1], [q])), 0, q)
        else:
            _, a, b, u = op
            g4 = np.asarray(u, dtype=np.complex128).reshape(2, 2, 2, 2)
            psi = np.moveaxis(np.tensordot(g4, psi, axes=([2, 3], [a, b])), [0, 1], [a, b])
    return psi.reshape(-1)


def mpo_operator(ws) -> np.ndarray:
    """The dense operator of an MPO on L sites: O[(s'_0..s'_{L-1}), (s_0..s_{L-1})]
    = sum over the bonds of prod_t W_t[a_t, s'_t, s_t, a_{t+1}] (site 0 the
    most significant bit), 2^L x 2^L."""
    o = np.ones((1, 1, 1), dtype=np.complex128)                 # [out, in, bond]
    for w in ws:
        w = np.asarray(w, dtype=np.complex128)
        t = np.einsum("xya,atsb->xtysb", o, w)                   # [out, s', in, s, b]
        o = t.reshape(o.shape[0] * 2, o.shape[1] * 2, w.shape[3])
    return o[:, :, 0]


def apply_mpo_dense(psi: np.ndarray, n: int, first: int, ws) -> np.ndarray:
    """The MPO applied to a dense statevector on qubits first .. first+L-1."""
    L = len(ws)
    op = mpo_operator(ws).reshape((2,) * (2 * L))
    t = np.tensordot(op, psi.reshape((2,) * n), axes=(list(range(L, 2 * L)), list(range(first, first + L))))
    return np.moveaxis(t, list(range(L)), list(range(first, first + L))).reshape(-1)


def brute_force(n: int, layers, bits=None) -> np.ndarray:
    """Apply the circuit to a dense statevector (Sec. II-A)."""
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[tuple(int(b) for b in (bits if bits is not None else [0] * n))] = 1.0
    for layer in layers:
        for i, g in layer:
            g4 = np.asarray(g, dtype=np.complex128).reshape(2, 2, 2, 2)
            psi = np.tensordot(g4, psi, axes=([2, 3], [i, i + 1]))
            psi = np.moveaxis(psi, [0, 1], [i, i + 1])
    return psi.reshape(-1)
