"""Pins of the oracle's SVD truncation (Table III, M = U S V^dagger; Sec. II-B
Schmidt decomposition) against facts fixed outside it (no GPU): exact
statevectors without truncation, the discarded spectrum computed from the
eigenvalues of theta^H theta, the Eckart-Young optimality of the truncated
SVD against pivoted QR and other rank-k approximations, and the orthogonal
projection of a single truncation at the orthogonality centre."""
import numpy as np
import pytest

import oracle
from paper_2505_06119_amd import synth


def test_svd_exact_matches_statevector():
    """10-qubit brickwork, depth 8, chi cap 32 = 2^(n/2): nothing is discarded."""
    n = 10
    layers = synth.brickwork(synth.rng(300), n, 8)
    m = oracle.MPS(synth.product_state_sites(n), chi_cap=32, truncation="svd")
    m.apply_layers(layers)
    np.testing.assert_allclose(oracle.statevector(m.sites), oracle.brute_force(n, layers), atol=1e-12)
    assert max(h["err"] for h in m.history) < 1e-12
    assert abs(oracle.norm_fidelity(m.sites) - 1.0) < 1e-12


@pytest.mark.parametrize("m_,n_,k,seed", [(40, 30, 12, 1), (24, 64, 10, 2), (32, 32, 31, 3)])
def test_svd_error_is_discarded_spectrum(m_, n_, k, seed):
    """||theta - U_k (S V^dagger)_k||_F = (sum of the n - k smallest eigenvalues
    of theta^H theta)^(1/2); the factors have rank k and U_k is orthonormal."""
    r = synth.rng(seed)
    th = synth.cgauss(r, (m_, n_))
    f = oracle.svd_truncate(th, k)
    approx = f["U"] @ f["SVh"]
    lam = np.sort(np.linalg.eigvalsh(th.conj().T @ th))[::-1]
    lam = np.clip(lam, 0.0, None)
    disc = np.sqrt(lam[k:].sum())
    assert abs(np.linalg.norm(th - approx) - disc) <= 1e-10 * np.linalg.norm(th)
    assert abs(f["err"] - disc) <= 1e-10 * np.linalg.norm(th)
    np.testing.assert_allclose(f["U"].conj().T @ f["U"], np.eye(f["k"]), atol=1e-12)
    assert np.linalg.matrix_rank(approx, tol=1e-10 * np.linalg.norm(th)) == f["k"]


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_svd_no_worse_than_qrcp_and_random_projections(seed):
    """Eckart-Young: the truncated SVD's error is at most pivoted QR's and at
    most that of projecting theta onto any other k-dimensional column space."""
    r = synth.rng(seed)
    sig = synth.exp_spectrum(48, 12.0)
    a, b = synth.canonical_pair(r, 24, 48, 24, sig)
    th = oracle.theta(a, b, synth.haar_unitary(r, 4))
    k = 20
    e_svd = oracle.svd_truncate(th, k)["err"]
    e_qr = oracle.qrcp(th, k)["err"]
    assert e_svd <= e_qr * (1 + 1e-12)
    for _ in range(20):
        basis, _ = np.linalg.qr(synth.cgauss(r, (th.shape[0], k)))
        e_rand = np.linalg.norm(th - basis @ (basis.conj().T @ th))
        assert e_svd <= e_rand * (1 + 1e-12)


def test_svd_single_truncation_overlap_equals_norm_fidelity():
    """One SVD truncation at the orthogonality centre is an orthogonal
    projection: overlap fidelity equals norm fidelity, 1 - eps^2."""
    n = 8
    layers = synth.brickwork(synth.rng(302), n, 6)
    m = oracle.MPS(synth.product_state_sites(n), chi_cap=16, truncation="svd")
    m.apply_layers(layers)
    g = synth.haar_unitary(synth.rng(303), 4)
    exact = oracle.brute_force(n, layers + [[(3, g)]])
    rec = m.apply_gate(3, g, chi_cap=5)
    assert rec["err"] > 1e-3
    fbar = oracle.norm_fidelity(m.sites)
    assert abs(fbar - oracle.overlap_fidelity(exact, m.sites)) < 1e-12
    assert abs(fbar - (1.0 - rec["err"] ** 2)) < 1e-12


def test_svd_and_qrcp_agree_without_truncation():
    """Without truncation both decompositions represent the same state."""
    n = 8
    layers = synth.brickwork(synth.rng(304), n, 6)
    a = oracle.MPS(synth.product_state_sites(n), chi_cap=16, truncation="svd")
    b = oracle.MPS(synth.product_state_sites(n), chi_cap=16)
    a.apply_layers(layers)
    b.apply_layers(layers)
    np.testing.assert_allclose(oracle.statevector(a.sites), oracle.statevector(b.sites), atol=1e-12)


def test_unknown_truncation_rejected():
    r = synth.rng(7)
    a, b = synth.canonical_pair(r, 2, 4, 2, synth.exp_spectrum(4, 2.0))
    with pytest.raises(ValueError):
        oracle.two_site_update(a, b, np.eye(4), 4, truncation="polar")
