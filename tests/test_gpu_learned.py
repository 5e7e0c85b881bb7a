"""GPU parity of the learned pivot proposal (sketch features, network forward
and gradient, ranking) against the FP64 oracle, and behaviour of the learned
update: verification against plain pivoted QR, fallback, certificate mode, and
what training gains over the untrained network."""
import numpy as np
import pytest

import oracle
from oracle import pivnet as opn
from paper_2505_06119_amd import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-4}


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_06119_amd import mps
    return mps


def _to_oracle_theta(theta_gpu, chi_l, chi_r):
    """GPU theta rows l + chi_l*a, cols b + 2r -> oracle rows 2l + a, cols 2r + b."""
    t = theta_gpu.reshape(2, chi_l, chi_r, 2)          # [a, l, r, b]
    return t.transpose(1, 0, 2, 3).reshape(2 * chi_l, 2 * chi_r)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("chl,chm,chr_", [(4, 8, 4), (24, 40, 20), (33, 17, 50)])
def test_theta_matches_oracle(M, prec, chl, chm, chr_):
    print(f"case theta chi=({chl},{chm},{chr_}) prec={prec}", flush=True)
    r = synth.rng(chl + chm)
    a = synth.cgauss(r, (chl, 2, chm))
    b = synth.cgauss(r, (chm, 2, chr_))
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
        b = b.astype(np.complex64).astype(np.complex128)
    g = synth.haar_unitary(r, 4)
    th = M.mps_theta(M.site_to_device(a, prec), M.site_to_device(b, prec), g, chl, chm, chr_, prec)
    got = _to_oracle_theta(th.cpu().numpy().astype(np.complex128), chl, chr_)
    ref = oracle.theta(a, b, g)
    # one contraction and one gate: well inside the 1e-10 / 1e-4 bar
    tol = 1e-11 if prec == 0 else 2e-5
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", [0, 1])
def test_features_match_oracle(M, prec):
    print(f"case features prec={prec}", flush=True)
    theta = synth.cgauss(synth.rng(21), (96, 70))
    if prec == 1:
        theta = theta.astype(np.complex64).astype(np.complex128)
    phi = M.pivnet_features(M.colmajor(theta, prec), prec, sketch_rows=16, seed=99).cpu().numpy()
    ref = opn.features(theta, 16, 99)
    tol = 1e-5 if prec == 0 else 1e-4
    np.testing.assert_allclose(phi[:, [0, 2, 3]], ref[:, [0, 2, 3]], rtol=tol, atol=tol)
    np.testing.assert_allclose(phi[:, 1], ref[:, 1], rtol=tol, atol=tol)


def test_forward_and_gradient_match_oracle(M):
    import torch
    r = synth.rng(22)
    p = (r.standard_normal(opn.P) * 0.5).astype(np.float32)
    phi = r.standard_normal((1000, opn.F)).astype(np.float32)
    lab = r.integers(0, 2, 1000).astype(np.uint8)
    pd = torch.from_numpy(p).cuda()
    phid = torch.from_numpy(phi).cuda()
    labd = torch.from_numpy(lab).cuda()
    s = M.pivnet_forward(pd, phid).cpu().numpy()
    sref = opn.forward(p.astype(np.float64), phi.astype(np.float64))
    np.testing.assert_allclose(s, sref, rtol=1e-5, atol=1e-5)
    g = M.pivnet_grad(pd, phid, labd).cpu().numpy()
    gref, lref = opn.loss_grad(p.astype(np.float64), phi.astype(np.float64), lab)
    assert np.max(np.abs(g[:opn.P] - gref)) <= 1e-5 * max(1.0, np.max(np.abs(gref)))
    assert abs(g[opn.P] - lref) <= 1e-5 * max(1.0, abs(lref))


def test_adam_matches_oracle(M):
    """Five Adam steps of k_pn_adam (float32) against the FP64 oracle step."""
    import torch
    r = synth.rng(24)
    p = (r.standard_normal(opn.P) * 0.5).astype(np.float32)
    pd = torch.from_numpy(p.copy()).cuda()
    m1 = torch.zeros(opn.P, dtype=torch.float32, device="cuda")
    m2 = torch.zeros(opn.P, dtype=torch.float32, device="cuda")
    po, m1o, m2o = p.astype(np.float64), np.zeros(opn.P), np.zeros(opn.P)
    for t in range(1, 6):
        g = (r.standard_normal(opn.P) * 10.0 ** r.uniform(-2, 1, opn.P)).astype(np.float32)
        M.pivnet_adam(pd, torch.from_numpy(g).cuda(), m1, m2, t, 2e-3)
        po, m1o, m2o = opn.adam_step(po, g.astype(np.float64), m1o, m2o, t, 2e-3)
    torch.cuda.synchronize()
    # float32 parameters of size ~1 moved by ~1e-2: a few float32 ulps of p.
    # The kernel's float32 constants carry their own rounding: 1 - 0.999f is
    # 1e-3 (1 - 1.29e-5), so the second moment is off by 1.3e-5 relative.
    np.testing.assert_allclose(pd.cpu().numpy(), po, rtol=0, atol=4e-7)
    np.testing.assert_allclose(m1.cpu().numpy(), m1o, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(m2.cpu().numpy(), m2o, rtol=3e-5, atol=1e-9)


def test_rank_puts_nan_scores_last(M):
    """A NaN score ranks as -infinity (ties by column), so the order is still a
    permutation and no slot is left unwritten."""
    import torch
    s = np.array([0.5, np.nan, 2.0, np.nan, -1.0, 2.0], dtype=np.float32)
    order = M.pivnet_rank(torch.from_numpy(s).cuda()).cpu().numpy()
    assert list(order) == [2, 5, 0, 4, 1, 3]


def _proposed_order(M, theta_dev, prec, params, sketch_rows, seed):
    phi = M.pivnet_features(theta_dev, prec, sketch_rows=sketch_rows, seed=seed)
    return M.pivnet_rank(M.pivnet_forward(params, phi)).cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,n,k,seed", [(96, 80, 40, 50), (300, 260, 130, 51), (130, 300, 100, 52),
                                         (8400, 600, 300, 55), (2048, 1400, 700, 56)])
def test_known_order_qr_matches_oracle(M, prec, m, n, k, seed):
    """Learned mode of qrcp_truncate with an always-accepting rule: piv is the
    proposed order (the same order the proposal pieces give), and Q, R P^T,
    R_jj and eps_S equal the oracle's QR of A with that order; eps_S equals the
    projection residual of the selected columns (least squares)."""
    import torch
    print(f"case known-order qr m={m} n={n} k={k} prec={prec}", flush=True)
    r = synth.rng(seed)
    a = synth.cgauss(r, (m, n)) * np.exp(-np.arange(n) / (n / 3.0))[None, :]
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    params = torch.from_numpy((synth.rng(seed + 100).standard_normal(opn.P) * 0.5).astype(np.float32)).cuda()
    A = M.colmajor(a, prec)
    lc = M.learned_cfg(params, sketch_rows=32, verify=True, seed=seed, fallback_ratio=1e9)
    out = M.qrcp_truncate(A, k, prec, learned=lc)
    info = out["info"]
    assert info["fallback"] == 0
    piv = out["piv"].cpu().numpy().astype(np.int64)
    assert list(piv) == list(_proposed_order(M, A, prec, params, 32, seed))
    o = oracle.known_order_qr(a, piv, k)
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    q = out["Q"].cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(q - o["Q"])) <= tol
    rp_o = oracle.r_unpivot(o["R"], o["piv"])
    assert np.max(np.abs(out["RPt"].cpu().numpy().astype(np.complex128) - rp_o)) <= tol * scale
    np.testing.assert_allclose(out["diagR"].cpu().numpy(), o["diagR"], rtol=tol, atol=tol * scale)
    assert abs(out["err"] - o["err"]) <= tol * scale
    basis = a[:, piv[:k]]
    coef, *_ = np.linalg.lstsq(basis, a, rcond=None)
    assert abs(out["err"] - np.linalg.norm(a - basis @ coef)) <= tol * scale
    assert abs(info["learned_err_sq"] - o["err"] ** 2) <= tol * scale ** 2
    # the verification's plain pivoted QR error is the oracle's
    assert abs(np.sqrt(info["qrcp_err_sq"]) - oracle.qrcp(a, k)["err"]) <= tol * scale


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("verify", [True, False])
def test_learned_decision_matches_oracle(M, prec, verify):
    """The acceptance decision and the kept factorisation equal the oracle's
    learned_update on the same proposed order: with an untrained network the
    proposal is rejected by both rules, and the result is plain pivoted QR."""
    import torch
    print(f"case learned decision verify={verify} prec={prec}", flush=True)
    r = synth.rng(53)
    m, n, k = 160, 140, 60
    u = synth.haar_isometry(r, m, 70)
    w = synth.haar_isometry(r, n, 70)
    a = (u * synth.exp_spectrum(70, 12.0)) @ w.conj().T
    if prec == 1:
        a = a.astype(np.complex64).astype(np.complex128)
    params = torch.from_numpy((synth.rng(54).standard_normal(opn.P) * 0.5).astype(np.float32)).cuda()
    A = M.colmajor(a, prec)
    order = _proposed_order(M, A, prec, params, 32, 7)
    ref = oracle.learned_update(a, order, k, ratio=1.01, verify=verify)
    lc = M.learned_cfg(params, sketch_rows=32, verify=verify, seed=7, fallback_ratio=1.01)
    out = M.qrcp_truncate(A, k, prec, learned=lc)
    info = out["info"]
    assert not ref["accepted"]
    assert info["fallback"] == 1
    tol = TOL[prec]
    scale = np.linalg.norm(a)
    assert abs(np.sqrt(info["learned_err_sq"]) - ref["err_s"]) <= tol * scale
    assert abs(out["err"] - ref["err"]) <= tol * scale
    if prec == 0:
        assert list(out["piv"].cpu().numpy()[:k]) == list(ref["piv"][:k])


def test_rank_is_stable_descending_argsort(M):
    import torch
    r = synth.rng(23)
    s = np.round(r.standard_normal(3000), 1).astype(np.float32)      # many exact ties
    order = M.pivnet_rank(torch.from_numpy(s).cuda()).cpu().numpy()
    assert list(order) == list(np.argsort(-s, kind="stable"))


def _pair(seed, chi):
    r = synth.rng(seed)
    a, b = synth.canonical_pair(r, chi, chi, chi, synth.exp_spectrum(chi, chi / 4.0))
    return a, b, synth.haar_unitary(r, 4)


def _theta_t(M, out, chi, k):
    a2 = M.site_from_device(out["A"], chi, k)
    b2 = M.site_from_device(out["B"], k, chi)
    return np.tensordot(a2, b2, axes=(2, 0)), a2


@pytest.mark.parametrize("prec", [0, 1])
def test_learned_verify_accepts_or_falls_back(M, prec):
    import torch
    print(f"case learned verify prec={prec}", flush=True)
    chi = 48
    a, b, g = _pair(30, chi)
    params = torch.from_numpy((synth.rng(31).standard_normal(opn.P) * 0.5).astype(np.float32)).cuda()
    A, B = M.site_to_device(a, prec), M.site_to_device(b, prec)
    plain = M.mps_update_bond(A, B, g, chi, chi, chi, chi, prec, renormalize=False)
    tol = 1e-10 if prec == 0 else 1e-4
    for ratio in (1.0, 1e6):
        lc = M.learned_cfg(params, sketch_rows=32, verify=True, seed=5, fallback_ratio=ratio)
        out = M.mps_update_bond(A, B, g, chi, chi, chi, chi, prec, renormalize=False, learned=lc)
        info = out["info"]
        tt, a2 = _theta_t(M, out, chi, chi)
        q = a2.transpose(1, 0, 2).reshape(2 * chi, chi)
        np.testing.assert_allclose(q.conj().T @ q, np.eye(chi), atol=tol)
        ref = oracle.two_site_update(a, b, g, chi)
        th = np.tensordot(a, b, axes=(2, 0))
        th = np.einsum("xyab,labr->lxyr", g.reshape(2, 2, 2, 2), th)
        assert abs(np.linalg.norm(th - tt) ** 2 - info["trunc_err_sq"]) <= tol
        assert abs(info["qrcp_err_sq"] - plain["info"]["trunc_err_sq"]) <= tol
        if ratio == 1e6:
            assert info["fallback"] == 0
            assert abs(info["trunc_err_sq"] - info["learned_err_sq"]) <= tol
        if info["fallback"]:
            tp, _ = _theta_t(M, plain, chi, chi)
            assert np.max(np.abs(tt - tp)) <= tol
            assert info["learned_err_sq"] > ratio ** 2 * info["qrcp_err_sq"]
        else:
            assert info["learned_err_sq"] <= ratio ** 2 * info["qrcp_err_sq"] * (1 + 1e-9) + 1e-300
        del ref


def test_learned_trust_mode_is_consistent(M):
    import torch
    print("case learned trust", flush=True)
    chi = 40
    a, b, g = _pair(32, chi)
    params = torch.from_numpy((synth.rng(33).standard_normal(opn.P) * 0.5).astype(np.float32)).cuda()
    A, B = M.site_to_device(a, 0), M.site_to_device(b, 0)
    lc = M.learned_cfg(params, sketch_rows=32, verify=False, seed=6)
    out = M.mps_update_bond(A, B, g, chi, chi, chi, chi, 0, renormalize=False, learned=lc)
    info = out["info"]
    tt, _ = _theta_t(M, out, chi, chi)
    th = np.einsum("xyab,labr->lxyr", g.reshape(2, 2, 2, 2), np.tensordot(a, b, axes=(2, 0)))
    assert abs(np.linalg.norm(th - tt) ** 2 - info["trunc_err_sq"]) <= 1e-9
    if info["fallback"] == 0:
        assert abs(info["trunc_err_sq"] - info["learned_err_sq"]) <= 1e-10
    else:
        assert abs(info["trunc_err_sq"] - info["qrcp_err_sq"]) <= 1e-10


def test_training_gains_over_untrained(M):
    """Train on synthetic thetas, evaluate the excess truncation error of the
    proposed column sets on held-out thetas: trained must beat untrained."""
    import torch
    from paper_2505_06119_amd import pivnet
    print("case training gain", flush=True)
    prec = M.MPS_MIXED
    data = [pivnet.make_sample(2000 + s, 32 if s % 2 else 64, prec) for s in range(16)]
    p0 = pivnet.init_params(0)
    params = pivnet.to_device(p0)
    hist = pivnet.train(params, data, steps=600, lr=3e-3, log_every=200)
    assert hist[-1][1] < hist[0][1]

    def excess(pvec, seeds):
        ratios = []
        pd = pivnet.to_device(pvec) if isinstance(pvec, np.ndarray) else pvec
        for s in seeds:
            chi = 48
            r = synth.rng(s)
            a, b = synth.canonical_pair(r, chi, chi, chi, synth.exp_spectrum(chi, chi / 3.0))
            g = synth.haar_unitary(r, 4)
            lc = M.learned_cfg(pd, sketch_rows=64, verify=True, seed=s, fallback_ratio=1e9)
            out = M.mps_update_bond(M.site_to_device(a, prec), M.site_to_device(b, prec), g, chi, chi, chi, chi,
                                    prec, renormalize=False, learned=lc)
            i = out["info"]
            ratios.append(np.sqrt(i["learned_err_sq"] / i["qrcp_err_sq"]))
        return float(np.mean(ratios))

    held = list(range(3000, 3006))
    e_trained = excess(params, held)
    e_untrained = excess(p0, held)
    print(f"held-out mean eps_S/eps_QRCP: trained {e_trained:.4f}  untrained {e_untrained:.4f}", flush=True)
    assert e_trained < e_untrained


def test_context_with_learned_pivots(M):
    """12-qubit brickwork at chi 32 with verified learned pivots: every update
    is within 1% of plain pivoted QR's error and the state stays consistent."""
    import torch
    print("case context learned", flush=True)
    n = 12
    layers = synth.brickwork(synth.rng(100), n, 10)
    params = torch.from_numpy((synth.rng(34).standard_normal(opn.P) * 0.5).astype(np.float32)).cuda()
    st = M.MPS(n, 32, M.MPS_FP64, pivot=M.MPS_PIVOT_LEARNED)
    st.set_pivot_network(M.learned_cfg(params, sketch_rows=32, verify=True, seed=9, fallback_ratio=1.01))
    infos = st.apply_layers(layers)
    for i in infos:
        if i["fallback"] == 0 and i["qrcp_err_sq"] > 1e-20:
            assert i["learned_err_sq"] <= 1.01 ** 2 * i["qrcp_err_sq"] * (1 + 1e-9)
    sv = oracle.statevector(st.sites())
    assert abs(np.vdot(sv, sv).real - 1.0) < 1e-10
    om = oracle.MPS(synth.product_state_sites(n), chi_cap=32)
    om.apply_layers(layers)
    f_q = oracle.norm_fidelity(om.sites)
    f_l = np.exp(st.log_norm_fidelity())
    assert f_l >= f_q * 0.95
