"""Host-side fusion of consecutive same-bond operations (no GPU): fused
circuits give the same statevector as the original ones, by brute force and
through the oracle MPS, with fewer two-site updates."""
import numpy as np
import pytest

import oracle
from paper_2505_06119_amd import routing, synth


def _count(layers):
    return sum(len(layer) for layer in layers)


@pytest.mark.parametrize("rows,cols,cycles,seed", [(3, 4, 8, 1), (2, 5, 10, 2), (3, 3, 6, 3)])
def test_fused_grid_circuit_same_state(rows, cols, cycles, seed):
    layers, _ = synth.grid_rcs(synth.rng(seed), rows, cols, cycles)
    fused = routing.fuse_layers(layers)
    n = rows * cols
    np.testing.assert_allclose(oracle.brute_force(n, fused), oracle.brute_force(n, layers), atol=1e-12)
    assert _count(fused) < _count(layers)


def test_fusion_pairs_single_qubit_layer_with_fsim_and_swap():
    """A paired single-qubit op, then a gate, then a SWAP on one bond with
    nothing else on its sites: one update whose matrix is SWAP G S."""
    r = synth.rng(4)
    s = np.kron(synth.gate_sqrt_x(), synth.gate_sqrt_y())
    g = synth.haar_unitary(r, 4)
    ops = [(2, s), (0, g), (2, g), (4, s), (2, synth.gate_swap())]
    out = routing.fuse(ops)
    assert [i for i, _ in out] == [2, 0, 4]
    np.testing.assert_allclose(out[0][1], synth.gate_swap() @ g @ s, atol=1e-14)


def test_no_fusion_across_an_operation_on_a_shared_site():
    r = synth.rng(5)
    a, b, c = (synth.haar_unitary(r, 4) for _ in range(3))
    out = routing.fuse([(1, a), (2, b), (1, c)])
    assert [i for i, _ in out] == [1, 2, 1]


def test_pack_layers_keeps_order_and_disjointness():
    layers, _ = synth.grid_rcs(synth.rng(6), 3, 4, 6)
    ops = routing.fuse(routing.flatten(layers))
    packed = routing.pack_layers(ops)
    for layer in packed:
        bonds = [i for i, _ in layer]
        assert all(b2 >= b1 + 2 for b1, b2 in zip(bonds, bonds[1:]))
    flat = routing.flatten(packed)
    assert [i for i, _ in flat] == [i for i, _ in ops]
    for (_, g1), (_, g2) in zip(flat, ops):
        np.testing.assert_array_equal(g1, g2)


def test_fused_oracle_mps_exact():
    """The oracle MPS on the fused circuit (no truncation) equals brute force."""
    layers, _ = synth.grid_rcs(synth.rng(7), 3, 4, 8)
    fused = routing.fuse_layers(layers)
    m = oracle.MPS(synth.product_state_sites(12), chi_cap=64)
    m.apply_layers(fused)
    np.testing.assert_allclose(oracle.statevector(m.sites), oracle.brute_force(12, layers), atol=1e-12)


def _to_logical(psi_chain, order):
    n = len(order)
    pos = {q: p for p, q in enumerate(order)}
    return np.transpose(psi_chain.reshape((2,) * n), [pos[q] for q in range(n)]).reshape(-1)


@pytest.mark.parametrize("rows,cols,cycles,seed", [(3, 4, 8, 1), (2, 5, 10, 2)])
def test_grid_rcs_logical_is_the_embedded_circuit(rows, cols, cycles, seed):
    """grid_rcs (chain positions, SWAP re-embedding) and grid_rcs_logical
    (logical qubits) describe the same circuit."""
    layers, order = synth.grid_rcs(synth.rng(seed), rows, cols, cycles)
    ops = synth.grid_rcs_logical(synth.rng(seed), rows, cols, cycles)
    n = rows * cols
    np.testing.assert_allclose(_to_logical(oracle.brute_force(n, layers), order), oracle.brute_force_ops(n, ops),
                               atol=1e-12)


@pytest.mark.parametrize("rows,cols,cycles,seed", [(3, 4, 8, 1), (2, 5, 10, 2), (3, 3, 12, 3)])
def test_lazy_routing_same_state(rows, cols, cycles, seed):
    ops = synth.grid_rcs_logical(synth.rng(seed), rows, cols, cycles)
    n = rows * cols
    row_order, _ = synth.grid_snakes(rows, cols)
    chain, order = routing.route_lazy(n, ops, row_order)
    assert sorted(order) == list(range(n))
    layers = routing.pack_layers(routing.fuse(chain))
    np.testing.assert_allclose(_to_logical(oracle.brute_force(n, layers), order), oracle.brute_force_ops(n, ops),
                               atol=1e-12)


def test_lazy_routing_reorients_gates():
    """A non-symmetric gate on (a, b) with b left of a is conjugated by SWAP."""
    r = synth.rng(8)
    g = synth.haar_unitary(r, 4)
    u = synth.haar_unitary(r, 2)
    ops = [("1q", 2, u), ("2q", 2, 0, g), ("2q", 3, 0, g)]
    chain, order = routing.route_lazy(4, ops, [0, 1, 2, 3])
    layers = routing.pack_layers(chain)
    np.testing.assert_allclose(_to_logical(oracle.brute_force(4, layers), order), oracle.brute_force_ops(4, ops),
                               atol=1e-12)


def test_lazy_routing_oracle_mps_exact():
    ops = synth.grid_rcs_logical(synth.rng(9), 3, 4, 8)
    row_order, _ = synth.grid_snakes(3, 4)
    chain, order = routing.route_lazy(12, ops, row_order)
    m = oracle.MPS(synth.product_state_sites(12), chi_cap=64)
    m.apply_layers(routing.pack_layers(routing.fuse(chain)))
    np.testing.assert_allclose(_to_logical(oracle.statevector(m.sites), order), oracle.brute_force_ops(12, ops),
                               atol=1e-12)
