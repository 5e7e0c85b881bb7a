"""The two identities the Gram-matrix window panels (panel mode 1) rest on,
checked in plain numpy against the oracle's pivoted QR and LAPACK's zgeqrf
(no GPU, nothing shared with the HIP path):

1. Greedy column pivoting is decided by inner products alone: pivoted
   Cholesky of G = A^H A (largest remaining diagonal, ties to the smaller
   column) picks the oracle's pivots, and its rows are the oracle's R up to a
   sign per row (Table III, QR with pivoting).
2. For Q with orthonormal columns, the LU factorisation without pivoting of
   Q diag(s) - [I; 0], with s_j = -sign(Re w_j) chosen when column j is
   reached (w_j the Schur-complement diagonal), gives the Householder
   reflectors Y (unit lower) and T = -U Y_1^-H of the QR of the same columns
   with the xLARFG sign convention: Y, tau = diag(T) and R = diag(s) R_chol
   equal zgeqrf's."""
import numpy as np
import pytest
import scipy.linalg as sl
from scipy.linalg import lapack

import oracle
from paper_2505_06119_amd import synth


def _pivoted_cholesky(g, b):
    n = g.shape[0]
    d = np.real(np.diag(g)).copy()
    r = np.zeros((b, n), dtype=complex)
    live = np.ones(n, bool)
    piv = []
    for t in range(b):
        cand = np.flatnonzero(live)
        p = cand[np.argmax(d[cand])]
        piv.append(p)
        live[p] = False
        r[t, p] = np.sqrt(d[p])
        for c in np.flatnonzero(live):
            r[t, c] = (g[p, c] - np.vdot(r[:t, p], r[:t, c])) / r[t, p]
            d[c] -= abs(r[t, c]) ** 2
    return np.array(piv), r


def _reconstruct(q):
    """LU of Q diag(s) - [I; 0] with the signs chosen column by column."""
    m, b = q.shape
    w = q.copy()
    y = np.zeros((m, b), dtype=complex)
    u = np.zeros((b, b), dtype=complex)
    s = np.zeros(b)
    for j in range(b):
        s[j] = -1.0 if w[j, j].real >= 0 else 1.0
        u[j, j] = s[j] * w[j, j] - 1.0
        y[j, j] = 1.0
        y[j + 1:, j] = s[j] * w[j + 1:, j] / u[j, j]
        for k in range(j + 1, b):
            u[j, k] = w[j, k]
            w[j + 1:, k] -= y[j + 1:, j] * w[j, k]
    for k in range(b):
        u[:k, k] *= s[k]
    t = -u @ np.linalg.inv(y[:b, :b].conj().T)
    return y, t, s


@pytest.mark.parametrize("m,n,b,seed", [(64, 48, 16, 1), (300, 200, 32, 2), (500, 256, 32, 3)])
def test_pivoted_cholesky_of_the_gram_matrix_is_greedy_qrcp(m, n, b, seed):
    a = synth.cgauss(synth.rng(seed), (m, n)) * np.exp(-np.arange(n) / n)[None, :]
    piv, r = _pivoted_cholesky(a.conj().T @ a, b)
    o = oracle.qrcp(a, b)
    assert list(piv) == list(o["piv"][:b])
    # rows agree up to a sign each (R_oracle = diag(sign) R_chol, with the
    # oracle's diagonal real)
    ro = oracle.r_unpivot(o["R"], o["piv"])
    sgn = np.sign(o["diagR"])
    np.testing.assert_allclose(sgn[:, None] * r, ro, atol=1e-12 * np.abs(ro).max())


@pytest.mark.parametrize("m,b,seed", [(64, 16, 4), (400, 32, 5), (1000, 32, 6)])
def test_householder_reconstruction_is_zgeqrf(m, b, seed):
    a = synth.cgauss(synth.rng(seed), (m, b))
    qr, tau, _, info = lapack.zgeqrf(np.asfortranarray(a))
    assert info == 0
    v = np.tril(qr[:, :b], -1) + np.eye(m, b)
    r_lapack = np.triu(qr[:b, :b])
    # an orthonormal Q with a positive-diagonal R (CholeskyQR2 gives this one)
    r1 = np.linalg.cholesky(a.conj().T @ a).conj().T
    q1 = sl.solve_triangular(r1, a.T, trans="T", lower=False).T
    r2 = np.linalg.cholesky(q1.conj().T @ q1).conj().T
    q = sl.solve_triangular(r2, q1.T, trans="T", lower=False).T
    r_chol = r2 @ r1
    y, t, s = _reconstruct(q)
    np.testing.assert_allclose(y, v, atol=1e-12)
    np.testing.assert_allclose(np.diag(t), tau[:b], atol=1e-12)
    np.testing.assert_allclose(s[:, None] * r_chol, r_lapack, atol=1e-11 * np.abs(r_lapack).max())
    # the compact WY form reproduces the signed Q
    np.testing.assert_allclose(np.eye(m)[:, :b] - y @ t @ y[:b].conj().T, q * s[None, :], atol=1e-12)
