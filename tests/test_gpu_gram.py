"""GPU parity of the Gram-matrix window panels (mps_set_panel_mode(1): a
panel's pivots from pivoted Cholesky of the window's Gram matrix, its
reflectors from CholeskyQR2 and a Householder reconstruction) against the
FP64 oracle, at sizes where the pivoted QR runs window panels (more than 256
columns left, at most 8192 rows).

Tolerances as for the per-step panels: 1e-10 relative in FP64, 1e-4 in mixed
mode; pivots must equal the oracle's on well-separated inputs, and in FP64 on
Gaussian ones."""
import numpy as np
import pytest

import oracle
from paper_2505_06119_amd import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-4}


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_06119_amd import mps
    mps.set_panel_mode(1)
    yield mps
    mps.set_panel_mode(0)


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


def _run(M, a, k, prec):
    out = M.qrcp_truncate(M.colmajor(a, prec), k, prec)
    return {"Q": _host(out["Q"]), "RPt": _host(out["RPt"]), "piv": out["piv"].cpu().numpy().astype(np.int64),
            "diagR": out["diagR"].cpu().numpy(), "k": out["k"], "err": out["err"], "info": out.get("info", {})}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,n,seed", [(1000, 700, 3), (3000, 1500, 8), (600, 520, 4)])
def test_gram_panels_well_separated_exact(M, prec, m, n, seed):
    print(f"case gram well_separated m={m} n={n} prec={prec}", flush=True)
    a, p = synth.well_separated(synth.rng(seed), m, n)
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    g = _run(M, a, n, prec)
    o = oracle.qrcp(a, n)
    assert list(o["piv"]) == list(p)
    assert list(g["piv"]) == list(p)
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    np.testing.assert_allclose(g["diagR"], o["diagR"], rtol=tol, atol=tol * scale)
    assert np.linalg.norm(g["RPt"] - oracle.r_unpivot(o["R"], o["piv"])) <= tol * scale
    assert np.linalg.norm(g["Q"] - o["Q"]) <= tol * np.sqrt(n)
    assert np.linalg.norm(a - g["Q"] @ g["RPt"]) <= tol * scale


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,n,k,seed", [(600, 520, 260, 5), (2048, 1024, 512, 7), (700, 1200, 500, 9)])
def test_gram_panels_truncated_gaussian(M, prec, m, n, k, seed):
    print(f"case gram truncated m={m} n={n} k={k} prec={prec}", flush=True)
    a = synth.cgauss(synth.rng(seed), (m, n))
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    g = _run(M, a, k, prec)
    o = oracle.qrcp(a, k)
    assert g["k"] == o["k"]
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    if prec == 0:
        assert list(g["piv"][:k]) == list(o["piv"][:k])
        np.testing.assert_allclose(g["diagR"], o["diagR"], rtol=tol, atol=tol * scale)
        assert np.linalg.norm(g["Q"] - o["Q"]) <= tol * np.sqrt(k)
    approx_g = g["Q"] @ g["RPt"]
    approx_o = o["Q"] @ oracle.r_unpivot(o["R"], o["piv"])
    assert np.linalg.norm(approx_g - approx_o) <= tol * scale
    assert abs(g["err"] - o["err"]) <= tol * scale
    q = g["Q"]
    np.testing.assert_allclose(q.conj().T @ q, np.eye(g["k"]), atol=tol)


@pytest.mark.parametrize("prec", [0, 1])
def test_gram_panels_agree_with_per_step_panels(M, prec):
    """The same Gaussian matrix with both panel modes: identical pivots (the
    inputs' margins are far above either path's rounding) and factors within
    the bar."""
    print(f"case gram vs steps prec={prec}", flush=True)
    a = synth.cgauss(synth.rng(11), (1500, 900))
    k = 600
    g1 = _run(M, a, k, prec)
    M.set_panel_mode(0)
    try:
        g0 = _run(M, a, k, prec)
    finally:
        M.set_panel_mode(1)
    assert list(g1["piv"][:k]) == list(g0["piv"][:k])
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    assert np.linalg.norm(g1["Q"] @ g1["RPt"] - g0["Q"] @ g0["RPt"]) <= tol * scale
    assert abs(g1["err"] - g0["err"]) <= tol * scale


@pytest.mark.parametrize("prec", [0, 1])
def test_gram_panels_rank_deficient(M, prec):
    """Rank 40 with k = 100: once the rank is exhausted a pivot's Gram norm has
    cancelled, the Gram panel ends and the per-step kernels take over; the
    factorisation still reproduces the matrix and Q stays orthonormal."""
    print(f"case gram rank deficient prec={prec}", flush=True)
    r = synth.rng(12)
    a = synth.cgauss(r, (700, 40)) @ synth.cgauss(r, (40, 600))
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    g = _run(M, a, 100, prec)
    tol = TOL[prec]
    q = g["Q"]
    np.testing.assert_allclose(q.conj().T @ q, np.eye(100), atol=tol)
    assert np.linalg.norm(a - q @ g["RPt"]) <= tol * np.linalg.norm(a)
    assert g["err"] <= tol * np.linalg.norm(a)
    o = oracle.qrcp(a, 40)
    if prec == 0:
        assert list(g["piv"][:40]) == list(o["piv"][:40])


@pytest.mark.parametrize("prec", [0, 1])
def test_gram_panels_two_site_update_matches_oracle(M, prec):
    """A whole two-site update (theta 1024 x 1024, chi 512 -> 512) with Gram
    panels against the oracle's update: eps^2 against the norm, and theta_T
    in FP64."""
    print(f"case gram update prec={prec}", flush=True)
    chi = 512
    r = synth.rng(13)
    a, b = synth.canonical_pair(r, chi, chi, chi, synth.exp_spectrum(chi, 150.0 * chi / 1024.0))
    g = synth.haar_unitary(r, 4)
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
        b = b.astype(np.complex64).astype(np.complex128)
    out = M.mps_update_bond(M.site_to_device(a, prec), M.site_to_device(b, prec), g, chi, chi, chi, chi, prec,
                            renormalize=False)
    ref = oracle.two_site_update(a, b, g, chi)
    tol = TOL[prec]
    info = out["info"]
    assert out["k"] == ref["k"]
    assert abs(info["trunc_err_sq"] - ref["err"] ** 2) <= tol * info["norm_sq"]
    if prec == 0:   # mixed storage may part from the oracle's pivots at near ties
        a2 = M.site_from_device(out["A"], chi, ref["k"])
        b2 = M.site_from_device(out["B"], ref["k"], chi)
        tt = np.einsum("lak,kbr->labr", a2, b2)
        tr = np.einsum("lak,kbr->labr", ref["A"], ref["B"])
        assert np.max(np.abs(tt - tr)) <= tol * np.max(np.abs(tr))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,n,k,seed", [(300, 257, 257, 21), (513, 300, 200, 22), (290, 600, 280, 23),
                                         (257, 290, 257, 24), (1025, 333, 333, 25)])
def test_gram_panels_ragged_shapes(M, prec, m, n, k, seed):
    """Ragged sizes: a window with one or a few outside columns, row counts
    that are not multiples of the tiles, wide matrices, full factorisations."""
    print(f"case gram ragged m={m} n={n} k={k} prec={prec}", flush=True)
    a = synth.cgauss(synth.rng(seed), (m, n))
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    g = _run(M, a, k, prec)
    o = oracle.qrcp(a, k)
    assert g["k"] == o["k"] == min(k, m, n)
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    if prec == 0:
        assert list(g["piv"][:g["k"]]) == list(o["piv"][:o["k"]])
    approx_o = o["Q"] @ oracle.r_unpivot(o["R"], o["piv"])
    assert np.linalg.norm(g["Q"] @ g["RPt"] - approx_o) <= tol * scale
    assert abs(g["err"] - o["err"]) <= tol * scale
    np.testing.assert_allclose(g["Q"].conj().T @ g["Q"], np.eye(g["k"]), atol=tol)
