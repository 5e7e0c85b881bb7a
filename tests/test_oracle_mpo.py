"""Pins of the oracle's MPO application (Sec. III-C.3 zip-up) and of the
inverse-QFT MPOs (Sec. III-D.1): the MPO form against the textbook DFT, a
single MPO against the product of its gates, and the zip-up without
truncation against the dense operator."""
import numpy as np
import pytest

import oracle
from paper_2505_06119_amd import synth


def _bitrev(y: int, n: int) -> int:
    return int(format(y, f"0{n}b")[::-1], 2)


def _dense_of_ops(n: int, ops) -> np.ndarray:
    """Columns: the MPO sequence applied to each basis vector."""
    N = 2 ** n
    out = np.zeros((N, N), dtype=np.complex128)
    for y in range(N):
        psi = np.zeros(N, dtype=np.complex128)
        psi[y] = 1.0
        for first, ws in ops:
            psi = oracle.apply_mpo_dense(psi, n, first, ws)
        out[:, y] = psi
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_iqft_mpos_are_the_inverse_dft_before_bit_reversal(n):
    # the textbook QFT circuit without its final swaps is Rev . F (F[y, x] =
    # exp(2 pi i x y / N) / sqrt(N), qubit 0 the most significant bit), so its
    # inverse is F^-1 . Rev: entry (x, y) = exp(-2 pi i x rev(y) / N) / sqrt(N)
    N = 2 ** n
    m = _dense_of_ops(n, synth.iqft_mpo_ops(n))
    want = np.array([[np.exp(-2j * np.pi * x * _bitrev(y, n) / N) for y in range(N)] for x in range(N)]) / np.sqrt(N)
    np.testing.assert_allclose(m, want, atol=1e-12)


def test_one_iqft_mpo_is_its_gates():
    # the MPO for qubit 0 of 3: the controlled phases (0,1) and (0,2), then H on 0
    n = 3
    first, ws = synth.iqft_mpo_ops(n)[-1]
    assert first == 0 and len(ws) == 3
    h = synth.gate_h()
    eye = np.eye(2)

    def cp(a, b, phi):
        d = np.ones(8, dtype=np.complex128)
        for x in range(8):
            if (x >> (2 - a)) & 1 and (x >> (2 - b)) & 1:
                d[x] = np.exp(1j * phi)
        return np.diag(d)

    want = np.kron(h, np.kron(eye, eye)) @ cp(0, 1, -2 * np.pi / 4) @ cp(0, 2, -2 * np.pi / 8)
    np.testing.assert_allclose(oracle.mpo_operator(ws), want, atol=1e-13)


def _random_mps(r, n, dmax):
    dims = [1] + [min(dmax, 2 ** min(b, n - b)) for b in range(1, n)] + [1]
    sites = [synth.cgauss(r, (dims[j], 2, dims[j + 1])) for j in range(n)]
    sv = oracle.statevector(sites)
    s = 1.0 / np.sqrt(np.vdot(sv, sv).real)
    sites[0] = sites[0] * s
    return sites


@pytest.mark.parametrize("seed,first,L,m", [(0, 1, 4, 2), (1, 0, 6, 3), (2, 2, 2, 4), (3, 3, 1, 1)])
def test_zipup_without_truncation_is_the_dense_operator(seed, first, L, m):
    r = synth.rng(seed)
    n = 6
    sites = _random_mps(r, n, 8)
    md = [1] + [m] * (L - 1) + [1]
    ws = [synth.cgauss(r, (md[t], 2, 2, md[t + 1])) for t in range(L)]
    psi = oracle.MPS(sites, chi_cap=64, centre=n - 1)
    psi.move_centre(0)
    want = oracle.apply_mpo_dense(oracle.statevector(psi.sites), n, first, ws)
    psi.apply_mpo(first, ws)
    assert psi.centre == first + L - 1
    got = oracle.statevector(psi.sites)
    np.testing.assert_allclose(got, want, atol=1e-11 * np.abs(want).max())


def test_zipup_truncation_keeps_the_cap_and_loses_norm():
    r = synth.rng(7)
    n, chi = 8, 4
    sites = synth.saturated_sites(r, n, 8, 1.0)
    psi = oracle.MPS(sites, chi_cap=chi, centre=n - 1)
    psi.move_centre(0)
    sv = oracle.statevector(psi.sites)
    psi.sites[0] = psi.sites[0] / np.sqrt(np.vdot(sv, sv).real)
    exact = oracle.statevector(psi.sites)
    for first, ws in synth.iqft_mpo_ops(n):
        exact = oracle.apply_mpo_dense(exact, n, first, ws)
        psi.apply_mpo(first, ws)
    # the last MPO (qubit 0) sweeps every bond with the cap
    assert max(s.shape[2] for s in psi.sites[:-1]) <= chi
    f = oracle.norm_fidelity(psi.sites)
    assert 0.0 < f < 1.0
    # the truncated state is a projection-like approximation: its overlap with
    # the exact result cannot exceed the exact result's norm (1)
    assert oracle.overlap_fidelity(exact, psi.sites) <= 1.0 + 1e-12
