"""GPU parity of the MPO application (mps_apply_mpo, zip-up with pivoted-QR
truncation, Sec. III-C.3) and of state loading (mps_load_state) against the
FP64 oracle and dense statevectors."""
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
    return mps


def _normalised(sites):
    sv = oracle.statevector(sites)
    out = [s.copy() for s in sites]
    out[0] = out[0] / np.sqrt(np.vdot(sv, sv).real)
    return out


def _gpu_sv(st):
    """The stored (normalised) state as a dense vector."""
    return oracle.statevector(st.sites())


@pytest.mark.parametrize("prec", [0, 1])
def test_load_state_round_trip(M, prec):
    print(f"case load_state prec={prec}", flush=True)
    n = 8
    sites = synth.saturated_sites(synth.rng(11), n, 8, 1.0)
    st = M.MPS(n, 16, prec)
    st.load_state(sites)
    assert st.centre() == 0
    assert st.bond_dims() == [1] + [s.shape[2] for s in sites]
    assert abs(st.log_norm_fidelity()) == 0.0
    ref = oracle.statevector(_normalised(sites))
    sv = _gpu_sv(st)
    assert np.max(np.abs(sv - ref)) <= TOL[prec] * np.max(np.abs(ref))
    for x in (0, 37, 255):
        bits = [(x >> (n - 1 - j)) & 1 for j in range(n)]
        assert abs(st.amplitude(bits) - ref[x]) <= TOL[prec] * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ["exact_m2", "exact_whole_chain", "truncated_m2", "single_site"])
def test_apply_mpo_matches_oracle(M, prec, case):
    print(f"case mpo {case} prec={prec}", flush=True)
    r = synth.rng({"exact_m2": 21, "exact_whole_chain": 22, "truncated_m2": 23, "single_site": 24}[case])
    n = 8
    cap = 6 if case == "truncated_m2" else 64
    sites = _normalised(synth.saturated_sites(r, n, min(cap, 8), 1.0))
    first, L, m = {"exact_m2": (1, 5, 2), "exact_whole_chain": (0, 8, 2), "truncated_m2": (0, 8, 2),
                   "single_site": (5, 1, 1)}[case]
    md = [1] + [m] * (L - 1) + [1]
    ws = [synth.cgauss(r, (md[t], 2, 2, md[t + 1])) for t in range(L)]
    st = M.MPS(n, cap, prec)
    st.load_state(sites)
    om = oracle.MPS([s.copy() for s in sites], chi_cap=cap, centre=n - 1)
    om.move_centre(0)
    lr = st.apply_mpo(first, ws)
    om.apply_mpo(first, ws)
    assert st.centre() == first + L - 1 == om.centre
    assert st.bond_dims()[1:-1] == [s.shape[2] for s in om.sites[:-1]]
    n2 = oracle.norm_fidelity(om.sites)
    tol = TOL[prec]
    assert abs(lr - np.log(n2)) <= tol * max(1.0, abs(np.log(n2)))
    assert abs(st.log_norm_fidelity() - np.log(n2)) <= tol * max(1.0, abs(np.log(n2)))
    want = oracle.statevector(om.sites) / np.sqrt(n2)
    got = _gpu_sv(st)
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))


@pytest.mark.parametrize("prec", [0, 1])
def test_iqft_mpos_exact_vs_dense(M, prec):
    """Inverse QFT as bond-2 MPOs on a random 7-qubit state, no truncation:
    the result equals the dense inverse QFT (before bit reversal)."""
    print(f"case iqft exact prec={prec}", flush=True)
    n = 7
    sites = _normalised(synth.saturated_sites(synth.rng(31), n, 16, 1.0))
    st = M.MPS(n, 64, prec)
    st.load_state(sites)
    exact = oracle.statevector(sites)
    for first, ws in synth.iqft_mpo_ops(n):
        st.apply_mpo(first, ws)
        exact = oracle.apply_mpo_dense(exact, n, first, ws)
    assert abs(st.log_norm_fidelity()) <= TOL[prec]
    got = _gpu_sv(st)
    assert np.max(np.abs(got - exact)) <= TOL[prec] * np.max(np.abs(exact))


@pytest.mark.parametrize("prec", [0, 1])
def test_iqft_mpos_truncated_vs_oracle(M, prec):
    """10 qubits at saturation 1 of chi = 8 with the cap at 8: the MPOs
    would double the bonds, so they truncate; the GPU follows the oracle's
    zip-up (same pivots)."""
    print(f"case iqft truncated prec={prec}", flush=True)
    n, cap = 10, 8
    sites = _normalised(synth.saturated_sites(synth.rng(41), n, 8, 1.0))
    st = M.MPS(n, cap, prec)
    st.load_state(sites)
    om = oracle.MPS([s.copy() for s in sites], chi_cap=cap, centre=n - 1)
    om.move_centre(0)
    for first, ws in synth.iqft_mpo_ops(n):
        st.apply_mpo(first, ws)
        om.apply_mpo(first, ws)
    fo = oracle.norm_fidelity(om.sites)
    assert fo < 0.99
    tol = TOL[prec]
    assert abs(st.log_norm_fidelity() - np.log(fo)) <= tol * max(1.0, abs(np.log(fo)))
    want = oracle.statevector(om.sites) / np.sqrt(fo)
    got = _gpu_sv(st)
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))


def test_apply_mpo_rejects_bad_arguments(M):
    st = M.MPS(4, 8, 0)
    w = np.zeros((1, 2, 2, 1), dtype=np.complex128)
    w[0, 0, 0, 0] = w[0, 1, 1, 0] = 1.0
    with pytest.raises(M.MpsError):
        st.apply_mpo(4, [w])                                 # out of range
    with pytest.raises(M.MpsError):
        st.apply_mpo(3, [w, w])                              # past the end
    big = np.zeros((1, 2, 2, 3), dtype=np.complex128)
    end = np.zeros((3, 2, 2, 1), dtype=np.complex128)
    with pytest.raises(M.MpsError):
        st.apply_mpo(0, [big, end])                          # bond 3 > 2
    bad = w.copy()
    bad[0, 0, 0, 0] = np.nan
    with pytest.raises(M.MpsError):
        st.apply_mpo(1, [bad])
    # nothing changed: the identity MPO still applies and leaves |0000>
    assert st.apply_mpo(1, [w]) == pytest.approx(0.0, abs=1e-14)
    assert abs(st.amplitude([0, 0, 0, 0]) - 1.0) < 1e-14
