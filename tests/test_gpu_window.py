"""Candidate-window panels of the pivoted QR against the FP64 oracle and
against the same library with windows switched off.

A window panel factorises inside the W columns of largest residual norm and
keeps its steps only as far as a greedy replay against every other column
confirms them (window.hpp), so the pivots must be those of the full search.
Narrow windows force replays that cut panels short (window_misses > 0); the
results must not change.  Tolerances as in test_gpu_qrcp."""
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
    yield mps
    mps.set_tuning(0, -1)


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


def _qrcp(M, a, k, prec):
    out = M.qrcp_truncate(M.colmajor(a, prec), k, prec)
    return {"Q": _host(out["Q"]), "RPt": _host(out["RPt"]), "piv": out["piv"].cpu().numpy().astype(np.int64),
            "diagR": out["diagR"].cpu().numpy(), "k": out["k"], "err": out["err"]}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("pw,win", [(32, 256), (16, 64), (64, 128), (32, 64)])
def test_window_pivots_exact_well_separated(M, prec, pw, win):
    m, n, k = 1100, 900, 600
    print(f"case window well_separated m={m} n={n} k={k} pw={pw} win={win} prec={prec}", flush=True)
    a, p = synth.well_separated(synth.rng(21), m, n)
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    M.set_tuning(pw, win)
    g = _qrcp(M, a, k, prec)
    M.set_tuning(0, -1)
    assert list(g["piv"][:k]) == list(p[:k])
    o = oracle.qrcp(a, k)
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    np.testing.assert_allclose(g["diagR"], o["diagR"], rtol=tol, atol=tol * scale)
    assert abs(g["err"] - o["err"]) <= tol * scale
    assert np.linalg.norm(g["Q"] @ g["RPt"] - o["Q"] @ oracle.r_unpivot(o["R"], o["piv"])) <= tol * scale


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("win", [64, 128, 0])
def test_window_matches_full_search(M, prec, win):
    # a truncated two-site problem: theta 512 x 512 from a chi = 256 canonical pair, k = 256
    chi = 256
    print(f"case window update chi={chi} win={win} prec={prec}", flush=True)
    r = synth.rng(22)
    a, b = synth.canonical_pair(r, chi, chi, chi, synth.exp_spectrum(chi, 150.0 * chi / 1024.0))
    g = synth.haar_unitary(r, 4)
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
        b = b.astype(np.complex64).astype(np.complex128)
    th = oracle.theta(a, b, g)
    M.set_tuning(32, win)
    gw = _qrcp(M, th, chi, prec)
    out = M.mps_update_bond(M.site_to_device(a, prec), M.site_to_device(b, prec), g, chi, chi, chi, chi, prec,
                            renormalize=False)
    M.set_tuning(32, 0)
    gf = _qrcp(M, th, chi, prec)
    M.set_tuning(0, -1)
    info = out["info"]
    if win == 64:
        assert info["window_misses"] > 0      # the replay did cut panels short
    if win == 0:
        assert info["window_misses"] == 0
    o = oracle.qrcp(th, chi)
    tol = TOL[prec]
    scale = np.linalg.norm(th)
    if prec == 0:
        assert list(gw["piv"][:chi]) == list(o["piv"][:chi])
        assert list(gf["piv"][:chi]) == list(o["piv"][:chi])
    approx_o = o["Q"] @ oracle.r_unpivot(o["R"], o["piv"])
    for res in (gw, gf):
        assert np.linalg.norm(res["Q"] @ res["RPt"] - approx_o) <= tol * scale
        assert abs(res["err"] - o["err"]) <= tol * scale
    assert abs(info["trunc_err_sq"] - o["err"] ** 2) <= tol * scale ** 2


@pytest.mark.parametrize("prec", [0, 1])
def test_window_tall_delayed_steps(M, prec):
    # more than 8192 rows: the window panels run the delayed-update steps
    m, n, k = 8400, 600, 300
    print(f"case window tall m={m} n={n} k={k} prec={prec}", flush=True)
    a, p = synth.well_separated(synth.rng(23), m, n)
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    g = _qrcp(M, a, k, prec)
    assert list(g["piv"][:k]) == list(p[:k])
    o = oracle.qrcp(a, k)
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    np.testing.assert_allclose(g["diagR"], o["diagR"], rtol=tol, atol=tol * scale)
    assert abs(g["err"] - o["err"]) <= tol * scale
    approx_o = o["Q"] @ oracle.r_unpivot(o["R"], o["piv"])
    assert np.linalg.norm(g["Q"] @ g["RPt"] - approx_o) <= tol * scale


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_table_and_invariance(M, prec):
    """mps_autotune returns one valid entry per bucket up to chi_max, and the
    tuned tiles change no result: pivots, R_jj and the truncated product equal
    those of the default tiles."""
    print(f"case autotune prec={prec}", flush=True)
    chi = 200
    r = synth.rng(70)
    a, b = synth.canonical_pair(r, chi, chi, chi, synth.exp_spectrum(chi, 150.0 * chi / 1024.0))
    th = oracle.theta(a, b, synth.haar_unitary(r, 4))
    if prec == 1:
        th = th.astype(np.complex64).astype(np.complex128)
    ref = _qrcp(M, th, chi, prec)
    table = M.autotune(512, prec)
    try:
        assert [e["n_max"] for e in table][:2] == [362, 724] and len(table) == 3
        for e in table:
            assert e["panel_width"] in (16, 32, 64)
            assert e["qr_window"] == 0 or 64 <= e["qr_window"] <= 512
            assert 0 < e["ms"] <= e["ms_default"] * (1 + 1e-9)
        got = _qrcp(M, th, chi, prec)
    finally:
        M.clear_autotune()
    tol = TOL[prec]
    scale = np.linalg.norm(th)
    if prec == 0:   # complex64 norms can order near-ties differently under other tiles
        assert list(got["piv"][:chi]) == list(ref["piv"][:chi])
        np.testing.assert_allclose(got["diagR"], ref["diagR"], rtol=tol, atol=tol * scale)
    assert abs(got["err"] - ref["err"]) <= tol * scale
    assert np.linalg.norm(got["Q"] @ got["RPt"] - ref["Q"] @ ref["RPt"]) <= tol * scale


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("rank", [40, 64, 75])
def test_window_rank_deficient_refreshes(M, prec, rank):
    """Window panels past the rank: the replay flags the norms that fall under
    the recomputation threshold, the panel's outside update and norm commit
    (enqueued before the host reads the replay) leave the norms to a refresh,
    and the factorisation still reproduces the matrix with pivots equal to the
    oracle's up to the rank (FP64)."""
    print(f"case window rank deficient rank={rank} prec={prec}", flush=True)
    r = synth.rng(80 + rank)
    a = synth.cgauss(r, (700, rank)) @ synth.cgauss(r, (rank, 600))
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    k = 120
    out = M.qrcp_truncate(M.colmajor(a, prec), k, prec)
    q, rpt = _host(out["Q"]), _host(out["RPt"])
    info = out["info"]
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    assert info["refreshes"] > 0
    np.testing.assert_allclose(q.conj().T @ q, np.eye(k), atol=tol)
    assert np.linalg.norm(a - q @ rpt) <= tol * scale
    d = out["diagR"].cpu().numpy()
    assert np.all(np.abs(d[rank:]) <= tol * abs(d[0]))
    if prec == 0:
        o = oracle.qrcp(a, rank)
        assert list(out["piv"].cpu().numpy()[:rank]) == list(o["piv"][:rank])
