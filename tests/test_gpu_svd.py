"""GPU parity of the SVD truncation (mps_set_truncation, MPS_TRUNC_SVD): the
Jacobi SVD updates of the small-bond chains and of the multi-kernel path
(larger bonds, or chains off) against brute-force statevectors and the
oracle's SVD MPS, update by update."""
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
    mps.set_small_bond_limit(64)
    yield mps
    mps.set_small_bond_limit(64)


def _sv(st):
    return oracle.statevector(st.sites()) * np.sqrt(np.exp(st.log_norm_fidelity()))


def _fid(a, b):
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def _svd_state(M, n, chi, prec):
    st = M.MPS(n, chi, prec)
    st.set_truncation(M.MPS_TRUNC_SVD)
    return st


@pytest.mark.parametrize("prec", [0, 1])
def test_svd_exact_vs_statevector(M, prec):
    """12 qubits, brickwork depth 10, chi cap 64: nothing is discarded."""
    print(f"case svd exact prec={prec}", flush=True)
    n = 12
    layers = synth.brickwork(synth.rng(310), n, 10)
    st = _svd_state(M, n, 64, prec)
    infos = st.apply_layers(layers)
    ref = oracle.brute_force(n, layers)
    tol = TOL[prec]
    assert np.max(np.abs(_sv(st) - ref)) <= tol * np.max(np.abs(ref))
    assert abs(st.log_norm_fidelity()) <= tol
    assert all(i["panels"] == 0 and i["qrcp_err_sq"] == -1.0 for i in infos)


@pytest.mark.parametrize("prec", [0, 1])
def test_svd_truncated_vs_oracle(M, prec):
    """chi cap 16: every update's rank and retained norm, the bond dimensions,
    the norm fidelity and the final state against the oracle's SVD MPS."""
    print(f"case svd truncated prec={prec}", flush=True)
    n = 12
    layers = synth.brickwork(synth.rng(311), n, 10)
    st = _svd_state(M, n, 16, prec)
    infos = st.apply_layers(layers)
    om = oracle.MPS(synth.product_state_sites(n), chi_cap=16, truncation="svd")
    om.apply_layers(layers)
    tol = TOL[prec]
    assert len(infos) == len(om.history)
    for gi, rec in zip(infos, om.history):
        assert gi["k"] == rec["k"]
        assert abs(gi["retained"] - (1.0 - rec["err"] ** 2 / rec["norm2"])) <= tol
    fbar_o = oracle.norm_fidelity(om.sites)
    assert fbar_o < 0.999
    assert abs(np.exp(st.log_norm_fidelity()) - fbar_o) <= tol * fbar_o
    assert st.bond_dims() == [1] + om.bond_dims() + [1]
    assert 1 - _fid(oracle.statevector(om.sites), _sv(st)) <= tol


def test_svd_first_truncation_no_worse_than_qr(M):
    """Up to the first truncation both runs hold the same state; there the
    SVD discards at most what pivoted QR discards (Eckart-Young)."""
    print("case svd vs qr first truncation", flush=True)
    n = 12
    layers = synth.brickwork(synth.rng(312), n, 10)
    a = _svd_state(M, n, 16, 0)
    b = M.MPS(n, 16, 0)
    ia = a.apply_layers(layers)
    ib = b.apply_layers(layers)
    t = next(t for t, x in enumerate(ib) if x["trunc_err_sq"] > 1e-12)
    assert all(x["trunc_err_sq"] <= 1e-20 for x in ia[:t])
    assert abs(ia[t]["norm_sq"] - ib[t]["norm_sq"]) <= 1e-10
    assert ia[t]["trunc_err_sq"] <= ib[t]["trunc_err_sq"] * (1 + 1e-10)
    assert ia[t]["trunc_err_sq"] > 0.0


def test_svd_outside_chains_runs(M):
    """With chains off every update takes the multi-kernel SVD: same result as
    the chained one."""
    print("case svd multi-kernel single gate", flush=True)
    g = synth.haar_unitary(synth.rng(9), 4)
    ref = _svd_state(M, 6, 8, 0)
    ref.apply_gate(2, g)
    st = _svd_state(M, 6, 8, 0)
    M.set_small_bond_limit(0)
    try:
        info = st.apply_gate(2, g)
    finally:
        M.set_small_bond_limit(64)
    assert info["k"] == 2 and info["qrcp_err_sq"] == -1.0
    assert st.bond_dims() == ref.bond_dims()
    a, b = _sv(st), _sv(ref)
    assert np.max(np.abs(a - b)) <= TOL[0] * np.max(np.abs(b))


@pytest.mark.parametrize("prec", [0, 1])
def test_svd_multikernel_truncated_vs_oracle(M, prec):
    """The chi cap 16 circuit with chains off: every update is a multi-kernel
    Jacobi SVD; ranks, retained norms, F-bar and the state against the oracle."""
    print(f"case svd multi-kernel truncated prec={prec}", flush=True)
    n = 12
    layers = synth.brickwork(synth.rng(311), n, 10)
    st = _svd_state(M, n, 16, prec)
    M.set_small_bond_limit(0)
    try:
        infos = st.apply_layers(layers)
    finally:
        M.set_small_bond_limit(64)
    om = oracle.MPS(synth.product_state_sites(n), chi_cap=16, truncation="svd")
    om.apply_layers(layers)
    tol = TOL[prec]
    for gi, rec in zip(infos, om.history):
        assert gi["k"] == rec["k"]
        assert abs(gi["retained"] - (1.0 - rec["err"] ** 2 / rec["norm2"])) <= tol
    fbar_o = oracle.norm_fidelity(om.sites)
    assert abs(np.exp(st.log_norm_fidelity()) - fbar_o) <= tol * fbar_o
    assert st.bond_dims() == [1] + om.bond_dims() + [1]
    assert 1 - _fid(oracle.statevector(om.sites), _sv(st)) <= tol


@pytest.mark.parametrize("prec", [0, 1])
def test_svd_bonds_above_the_chains_vs_oracle(M, prec):
    """14 qubits, brickwork depth 12, chi cap 96: the middle bonds pass 64, so
    their updates run as multi-kernel SVDs between chained runs."""
    print(f"case svd large bonds prec={prec}", flush=True)
    n, cap = 14, 96
    layers = synth.brickwork(synth.rng(312), n, 12)
    st = _svd_state(M, n, cap, prec)
    infos = st.apply_layers(layers)
    om = oracle.MPS(synth.product_state_sites(n), chi_cap=cap, truncation="svd")
    om.apply_layers(layers)
    assert max(om.bond_dims()) > 64
    tol = TOL[prec]
    for gi, rec in zip(infos, om.history):
        assert gi["k"] == rec["k"]
        assert abs(gi["retained"] - (1.0 - rec["err"] ** 2 / rec["norm2"])) <= tol
    fbar_o = oracle.norm_fidelity(om.sites)
    assert fbar_o < 0.9999
    assert abs(np.exp(st.log_norm_fidelity()) - fbar_o) <= tol * fbar_o
    assert st.bond_dims() == [1] + om.bond_dims() + [1]
    assert 1 - _fid(oracle.statevector(om.sites), _sv(st)) <= tol


def test_set_truncation_validation(M):
    st = M.MPS(4, 4, 0)
    with pytest.raises(M.MpsError):
        st.set_truncation(7)
    lr = M.MPS(4, 4, 0, M.MPS_PIVOT_LEARNED)
    with pytest.raises(M.MpsError):
        lr.set_truncation(M.MPS_TRUNC_SVD)
    lr.set_truncation(M.MPS_TRUNC_QRCP)
