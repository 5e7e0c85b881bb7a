"""Circuit workloads (grid random circuit with SWAP re-embedding, phase
estimation): oracle MPS against brute force and closed forms (no GPU), and
the HIP path against the oracle (GPU)."""
import numpy as np
import pytest

import oracle
from paper_2505_06119_amd import synth


def test_grid_couplers_and_embeddings():
    rows, cols = 5, 8
    row_o, col_o = synth.grid_snakes(rows, cols)
    assert sorted(row_o) == list(range(40)) and sorted(col_o) == list(range(40))
    for pat in "ABCD":
        pairs = synth.grid_couplers(rows, cols, pat)
        order = row_o if pat in "AB" else col_o
        pos = {q: p for p, q in enumerate(order)}
        for a, b in pairs:
            assert abs(pos[a] - pos[b]) == 1             # neighbours in the chosen embedding
    swaps = synth.bubble_swaps(row_o, col_o)
    # bubble sort performs exactly one swap per inversion
    key = [col_o.index(q) for q in row_o]
    inv = sum(1 for i in range(40) for j in range(i + 1, 40) if key[i] > key[j])
    assert len(swaps) == inv


def test_grid_rcs_oracle_exact():
    layers, order = synth.grid_rcs(synth.rng(5), 3, 4, 6)
    m = oracle.MPS(synth.product_state_sites(12), chi_cap=64)
    m.apply_layers(layers)
    np.testing.assert_allclose(oracle.statevector(m.sites), oracle.brute_force(12, layers), atol=1e-12)


@pytest.mark.parametrize("mm", [3, 11])
def test_qpe_exact_phase_oracle(mm):
    t = 4
    layers = synth.qpe_circuit(t, [2 * np.pi * mm / 2 ** t], target_init="one")
    m = oracle.MPS(synth.product_state_sites(t + 1), chi_cap=16)
    m.apply_layers(layers)
    p = np.abs(oracle.statevector(m.sites).reshape(2 ** t, 2)) ** 2
    assert abs(p.sum(axis=1)[mm] - 1.0) < 1e-12


def test_qpe_superposed_targets_closed_form():
    """Targets in |+>: P(y) = 2^-s sum_b |N^-1 sum_x exp(2 pi i x (phi_b - y/N))|^2."""
    t = 4
    alphas = [0.7, 2.1]
    layers = synth.qpe_circuit(t, alphas, target_init="plus")
    n = t + len(alphas)
    m = oracle.MPS(synth.product_state_sites(n), chi_cap=64)
    m.apply_layers(layers)
    p = (np.abs(oracle.statevector(m.sites).reshape(2 ** t, -1)) ** 2).sum(axis=1)
    N = 2 ** t
    x = np.arange(N)
    ref = np.zeros(N)
    for b0 in (0, 1):
        for b1 in (0, 1):
            phi = (b0 * alphas[0] + b1 * alphas[1]) / (2 * np.pi)
            for y in range(N):
                ref[y] += abs(np.exp(2j * np.pi * x * (phi - y / N)).sum() / N) ** 2 / 4
    np.testing.assert_allclose(p, ref, atol=1e-12)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
def test_grid_rcs_gpu_truncated_vs_oracle(prec):
    """3x4 grid, 8 cycles (ABCDCDAB with re-embedding SWAPs), chi cap 16."""
    from paper_2505_06119_amd import mps
    print(f"case grid rcs prec={prec}", flush=True)
    layers, _ = synth.grid_rcs(synth.rng(6), 3, 4, 8)
    st = mps.MPS(12, 16, prec)
    st.apply_layers(layers)
    om = oracle.MPS(synth.product_state_sites(12), chi_cap=16)
    om.apply_layers(layers)
    tol = 1e-10 if prec == 0 else 1e-4
    f_o = oracle.norm_fidelity(om.sites)
    f_g = np.exp(st.log_norm_fidelity())
    assert f_o < 0.9999
    assert abs(f_g - f_o) <= tol * f_o
    sv_o = oracle.statevector(om.sites)
    sv_g = oracle.statevector(st.sites()) * np.sqrt(f_g)
    fid = abs(np.vdot(sv_o, sv_g)) ** 2 / (np.vdot(sv_o, sv_o).real * np.vdot(sv_g, sv_g).real)
    assert 1 - fid <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
def test_grid_rcs_gpu_fused_vs_oracle(prec):
    """The same circuit with consecutive same-bond operations fused
    (routing.fuse_layers): chi cap 64 equals brute force of the unfused
    circuit; chi cap 16 follows the oracle MPS run on the fused circuit."""
    from paper_2505_06119_amd import mps, routing
    print(f"case grid rcs fused prec={prec}", flush=True)
    layers, _ = synth.grid_rcs(synth.rng(6), 3, 4, 8)
    fused = routing.fuse_layers(layers)
    tol = 1e-10 if prec == 0 else 1e-4
    st = mps.MPS(12, 64, prec)
    st.apply_layers(fused)
    ref = oracle.brute_force(12, layers)
    sv = oracle.statevector(st.sites()) * np.sqrt(np.exp(st.log_norm_fidelity()))
    assert np.max(np.abs(sv - ref)) <= tol * np.max(np.abs(ref))
    st = mps.MPS(12, 16, prec)
    st.apply_layers(fused)
    om = oracle.MPS(synth.product_state_sites(12), chi_cap=16)
    om.apply_layers(fused)
    f_o = oracle.norm_fidelity(om.sites)
    f_g = np.exp(st.log_norm_fidelity())
    assert f_o < 0.9999
    assert abs(f_g - f_o) <= tol * f_o
    sv_o = oracle.statevector(om.sites)
    sv_g = oracle.statevector(st.sites()) * np.sqrt(f_g)
    fid = abs(np.vdot(sv_o, sv_g)) ** 2 / (np.vdot(sv_o, sv_o).real * np.vdot(sv_g, sv_g).real)
    assert 1 - fid <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
def test_grid_rcs_gpu_lazy_routing_vs_oracle(prec):
    """The grid circuit on logical qubits routed on demand (routing.route_lazy).
    chi cap 64: the state equals the logical brute force through the final
    qubit order.  chi cap 16, truncating: the QR-truncated run follows the
    oracle MPS (SWAP-heavy routing makes exactly tied residual norms in
    untruncated updates; both sides give a tie to the smaller column 2r + b'
    of theta), and so does the SVD-truncated run."""
    from paper_2505_06119_amd import mps, routing
    print(f"case grid rcs lazy prec={prec}", flush=True)
    ops = synth.grid_rcs_logical(synth.rng(6), 3, 4, 8)
    row_order, _ = synth.grid_snakes(3, 4)
    chain, order = routing.route_lazy(12, ops, row_order)
    layers = routing.pack_layers(routing.fuse(chain))
    pos = {q: p for p, q in enumerate(order)}
    perm = [pos[q] for q in range(12)]
    ref = oracle.brute_force_ops(12, ops)
    tol = 1e-10 if prec == 0 else 1e-4
    st = mps.MPS(12, 64, prec)
    st.apply_layers(layers)
    sv = oracle.statevector(st.sites()) * np.sqrt(np.exp(st.log_norm_fidelity()))
    sv = np.transpose(sv.reshape((2,) * 12), perm).reshape(-1)
    assert np.max(np.abs(sv - ref)) <= tol * np.max(np.abs(ref))
    # pivoted QR, truncating: against the oracle MPS
    st = mps.MPS(12, 16, prec)
    st.apply_layers(layers)
    om = oracle.MPS(synth.product_state_sites(12), chi_cap=16)
    om.apply_layers(layers)
    f_o = oracle.norm_fidelity(om.sites)
    f_g = np.exp(st.log_norm_fidelity())
    assert 0.01 < f_o < 0.9999
    assert abs(f_g - f_o) <= tol * f_o
    assert st.bond_dims() == [1] + om.bond_dims() + [1]
    sv_o = oracle.statevector(om.sites)
    sv_g = oracle.statevector(st.sites()) * np.sqrt(f_g)
    fid = abs(np.vdot(sv_o, sv_g)) ** 2 / (np.vdot(sv_o, sv_o).real * np.vdot(sv_g, sv_g).real)
    assert 1 - fid <= tol
    # SVD, truncating: against the oracle
    st = mps.MPS(12, 16, prec)
    st.set_truncation(mps.MPS_TRUNC_SVD)
    st.apply_layers(layers)
    om = oracle.MPS(synth.product_state_sites(12), chi_cap=16, truncation="svd")
    om.apply_layers(layers)
    f_o = oracle.norm_fidelity(om.sites)
    f_g = np.exp(st.log_norm_fidelity())
    assert f_o < 0.9999
    assert abs(f_g - f_o) <= tol * f_o
    sv_o = oracle.statevector(om.sites)
    sv_g = oracle.statevector(st.sites()) * np.sqrt(f_g)
    fid = abs(np.vdot(sv_o, sv_g)) ** 2 / (np.vdot(sv_o, sv_o).real * np.vdot(sv_g, sv_g).real)
    assert 1 - fid <= tol


@pytest.mark.gpu
def test_qpe_gpu_exact_phase():
    from paper_2505_06119_amd import mps
    print("case qpe", flush=True)
    t, mm = 5, 19
    layers = synth.qpe_circuit(t, [2 * np.pi * mm / 2 ** t], target_init="one")
    st = mps.MPS(t + 1, 32, mps.MPS_MIXED)
    st.apply_layers(layers)
    bits = [(mm >> (t - 1 - j)) & 1 for j in range(t)] + [1]
    assert abs(abs(st.amplitude(bits)) - 1.0) < 1e-4


def _qpe_prefix(t, alphas, target_init):
    """Phase estimation up to its inverse QFT (the gates before it), with the
    controlled powers in the order the MPO inverse QFT (no final bit
    reversal) reads in natural order."""
    layers = synth.qpe_circuit(t, alphas, target_init=target_init, reversed_powers=True)
    return layers[:len(layers) - len(synth.qft_circuit(t, inverse=True))]


def test_qpe_with_mpo_iqft_oracle():
    """Phase estimation with the inverse QFT as bond-2 MPOs (Sec. III-D.1),
    on the oracle MPS: the counting register reads the exact phase m / 2^t."""
    t, mm = 5, 19
    n = t + 1
    om = oracle.MPS(synth.product_state_sites(n), chi_cap=32)
    om.apply_layers(_qpe_prefix(t, [2 * np.pi * mm / 2 ** t], "one"))
    for first, ws in synth.iqft_mpo_ops(t):
        om.apply_mpo(first, ws)
    bits = [(mm >> (t - 1 - j)) & 1 for j in range(t)] + [1]
    assert abs(abs(oracle.amplitude(om.sites, bits)) - 1.0) < 1e-12


@pytest.mark.gpu
def test_qpe_gpu_with_mpo_iqft():
    from paper_2505_06119_amd import mps
    print("case qpe mpo", flush=True)
    t, mm = 6, 45
    st = mps.MPS(t + 1, 32, mps.MPS_MIXED)
    st.apply_layers(_qpe_prefix(t, [2 * np.pi * mm / 2 ** t], "one"))
    for first, ws in synth.iqft_mpo_ops(t):
        st.apply_mpo(first, ws)
    bits = [(mm >> (t - 1 - j)) & 1 for j in range(t)] + [1]
    assert abs(abs(st.amplitude(bits)) - 1.0) < 1e-4
