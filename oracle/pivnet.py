"""FP64 reference of the learned pivot proposal -- TEST INFRASTRUCTURE ONLY.

The proposal replaces the per-column pivot search of pivoted QR by a column
order predicted from a Gaussian sketch of theta (an addition of this library; the
paper uses plain pivoted QR).  This module computes, plainly and in FP64:

* ``omega``     the sketch matrix: the SplitMix64 output function (Steele, Lea
  and Flood, OOPSLA 2014) of seed + (counter+1)*0x9E3779B97F4A7C15 gives two
  uniforms u1, u2 in (0, 1] per entry (counters 2q and 2q+1 for entry q of the
  column-major ell x m matrix); the entry is sqrt(-ln u1) exp(2 pi i u2), a
  complex Gaussian with E|w|^2 = 1 (Box-Muller).
* ``features``  per column c of theta, with y_c = (Omega theta)[:, c],
  s_c = |y_c|^2, mean/max over columns and y_top the column of largest s:
  (s_c/mean, ln(s_c/mean + 1e-30), s_c/max, |<y_top, y_c>|^2/(s_top s_c)).
* ``forward``   score = w2 . tanh(W1 phi + b1) + b2 (4 -> 16 -> 1).
* ``loss_grad`` mean logistic loss sum_c [softplus(s_c) - y_c s_c]/n and its
  gradient by the chain rule, written out by hand.
* ``adam_step`` one step of the Adam optimiser that trains the network.

The gradient is pinned against central finite differences in the tests, and
the Adam step against its closed forms (the first step, and every step under
a constant gradient, moves each parameter by lr * sign(g) up to eps).
Parameter layout (97 values): W1[h*4 + f] (64), b1 (16), w2 (16), b2 (1).
"""
from __future__ import annotations

import numpy as np

F, H = 4, 16
P = H * F + H + H + 1
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _u01(x: np.ndarray) -> np.ndarray:
    return ((x >> np.uint64(11)).astype(np.float64) + 1.0) / 9007199254740992.0


def omega(ell: int, m: int, seed: int) -> np.ndarray:
    q = np.arange(ell * m, dtype=np.uint64)            # column-major index r + ell*i
    u1 = _u01(splitmix64(seed, np.uint64(2) * q))
    u2 = _u01(splitmix64(seed, np.uint64(2) * q + np.uint64(1)))
    w = np.sqrt(-np.log(u1)) * np.exp(2j * np.pi * u2)
    return w.reshape(m, ell).T                          # [r, i]


def features(theta: np.ndarray, ell: int, seed: int) -> np.ndarray:
    y = omega(ell, theta.shape[0], seed) @ theta
    s = np.sum(np.abs(y) ** 2, axis=0)
    mean = s.mean() if s.mean() > 0 else 1.0
    mx = s.max() if s.max() > 0 else 1.0
    top = int(np.argmax(s))                              # first index among equal maxima
    dot = y[:, top].conj() @ y
    phi = np.empty((theta.shape[1], F))
    phi[:, 0] = s / mean
    phi[:, 1] = np.log(s / mean + 1e-30)
    phi[:, 2] = s / mx
    phi[:, 3] = np.abs(dot) ** 2 / (s[top] * s + 1e-300)
    return phi


def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    w1 = p[:H * F].reshape(H, F)
    b1 = p[H * F:H * F + H]
    w2 = p[H * F + H:H * F + 2 * H]
    b2 = p[H * F + 2 * H]
    return w1, b1, w2, b2


def forward(p: np.ndarray, phi: np.ndarray) -> np.ndarray:
    w1, b1, w2, b2 = unpack(p)
    a = np.tanh(phi @ w1.T + b1)
    return a @ w2 + b2


def loss(p: np.ndarray, phi: np.ndarray, labels: np.ndarray) -> float:
    s = forward(p, phi)
    y = labels.astype(np.float64)
    return float(np.mean(np.logaddexp(0.0, s) - y * s))


def loss_grad(p: np.ndarray, phi: np.ndarray, labels: np.ndarray):
    """(gradient, loss) of the mean logistic loss, by the chain rule."""
    w1, b1, w2, b2 = unpack(p)
    n = phi.shape[0]
    z = phi @ w1.T + b1                 # n x H
    a = np.tanh(z)
    s = a @ w2 + b2                     # n
    y = labels.astype(np.float64)
    ds = (1.0 / (1.0 + np.exp(-s)) - y) / n
    g_w2 = a.T @ ds
    g_b2 = ds.sum()
    dz = (ds[:, None] * w2[None, :]) * (1.0 - a ** 2)
    g_w1 = dz.T @ phi
    g_b1 = dz.sum(axis=0)
    g = np.concatenate([g_w1.reshape(-1), g_b1, g_w2, [g_b2]])
    return g, float(np.mean(np.logaddexp(0.0, s) - y * s))


def adam_step(p: np.ndarray, g: np.ndarray, m1: np.ndarray, m2: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) in FP64: first and
    second moment estimates, their bias corrections by 1 - beta^t, and the
    update p - lr * m_hat / (sqrt(v_hat) + eps).  Returns new (p, m1, m2)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m1 = beta1 * np.asarray(m1, dtype=np.float64) + (1.0 - beta1) * g
    m2 = beta2 * np.asarray(m2, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m1 / (1.0 - beta1 ** t)
    v_hat = m2 / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m1, m2
