"""Pins of the learned-proposal oracle (no GPU): the generator against its
published outputs and distribution, the features against their invariants,
and the hand-derived gradient against central finite differences."""
import os

import numpy as np

from oracle import pivnet
from paper_2505_06119_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.startswith("0x")]
    got = pivnet.splitmix64(0, np.arange(len(vals), dtype=np.uint64))
    assert [int(x) for x in got] == vals


def test_omega_is_standard_complex_gaussian():
    w = pivnet.omega(64, 4096, seed=7).reshape(-1)
    n = w.size
    assert abs(np.mean(np.abs(w) ** 2) - 1.0) < 5 / np.sqrt(n)
    assert abs(np.mean(w)) < 5 / np.sqrt(n)
    assert abs(np.mean(w * w)) < 5 / np.sqrt(n)            # circular: E[w^2] = 0
    assert abs(np.mean(w.real ** 2) - 0.5) < 5 / np.sqrt(n)
    assert not np.allclose(pivnet.omega(4, 8, 1), pivnet.omega(4, 8, 2))


def test_feature_invariants():
    r = synth.rng(3)
    theta = synth.cgauss(r, (48, 40))
    phi = pivnet.features(theta, 16, seed=5)
    np.testing.assert_allclose(phi, pivnet.features(3.7j * theta, 16, seed=5), rtol=1e-12, atol=1e-12)
    assert abs(phi[:, 0].mean() - 1.0) < 1e-12
    assert abs(phi[:, 2].max() - 1.0) < 1e-15
    top = int(np.argmax(phi[:, 2]))
    assert abs(phi[top, 3] - 1.0) < 1e-12
    assert np.all(phi[:, 3] <= 1.0 + 1e-12)
    np.testing.assert_allclose(phi[:, 1], np.log(phi[:, 0]), rtol=1e-12)


def test_gradient_matches_finite_differences():
    r = synth.rng(11)
    p = r.standard_normal(pivnet.P) * 0.5
    phi = r.standard_normal((37, pivnet.F))
    lab = r.integers(0, 2, 37).astype(np.uint8)
    g, loss = pivnet.loss_grad(p, phi, lab)
    assert abs(loss - pivnet.loss(p, phi, lab)) < 1e-14
    h = 1e-6
    fd = np.empty_like(g)
    for q in range(pivnet.P):
        e = np.zeros(pivnet.P)
        e[q] = h
        fd[q] = (pivnet.loss(p + e, phi, lab) - pivnet.loss(p - e, phi, lab)) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_forward_special_cases():
    phi = synth.rng(12).standard_normal((9, pivnet.F))
    p = np.zeros(pivnet.P)
    p[-1] = 0.25                                             # only the output bias
    np.testing.assert_allclose(pivnet.forward(p, phi), 0.25)
    p = np.zeros(pivnet.P)
    p[0] = 1.0                                               # W1[0, 0]
    p[pivnet.H * pivnet.F + pivnet.H] = 2.0                 # w2[0]
    np.testing.assert_allclose(pivnet.forward(p, phi), 2.0 * np.tanh(phi[:, 0]), rtol=1e-15)


def test_adam_first_step_moves_by_lr_sign():
    """Adam's first step (bias-corrected moments m_hat = g, v_hat = g^2) moves
    every parameter by lr * sign(g), up to eps / |g|."""
    r = synth.rng(13)
    p0 = r.standard_normal(pivnet.P)
    g = r.standard_normal(pivnet.P) * 10.0 ** r.uniform(-3, 2, pivnet.P)
    lr = 3e-3
    p1, m1, m2 = pivnet.adam_step(p0, g, np.zeros(pivnet.P), np.zeros(pivnet.P), 1, lr)
    step = p0 - p1
    np.testing.assert_allclose(step, lr * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.all(np.abs(step - lr * np.sign(g)) <= lr * 1e-8 / np.abs(g) + 1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(m2, 1e-3 * g * g, rtol=1e-12)


def test_adam_constant_gradient_steps_are_lr_sign():
    """Under a constant gradient both bias-corrected moments equal g and g^2 at
    every step, so every step moves by lr * sign(g) (up to eps)."""
    r = synth.rng(14)
    g = r.standard_normal(pivnet.P)
    p = r.standard_normal(pivnet.P)
    m1 = np.zeros(pivnet.P)
    m2 = np.zeros(pivnet.P)
    lr = 1e-2
    for t in range(1, 40):
        p_new, m1, m2 = pivnet.adam_step(p, g, m1, m2, t, lr)
        assert np.all(np.abs((p - p_new) - lr * np.sign(g)) <= lr * 1e-8 / np.abs(g) + 1e-13)
        p = p_new


def test_adam_minimises_a_quadratic():
    """On f(p) = |p - c|^2 / 2 (gradient p - c) Adam approaches the minimiser."""
    r = synth.rng(15)
    c = r.standard_normal(8)
    p = np.zeros(8)
    m1 = np.zeros(8)
    m2 = np.zeros(8)
    for t in range(1, 3001):
        p, m1, m2 = pivnet.adam_step(p, p - c, m1, m2, t, 1e-2)
    assert np.max(np.abs(p - c)) < 1e-3
