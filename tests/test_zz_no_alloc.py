"""qrcp_truncate_noalloc (static device scratch) against qrcp_truncate
(caller workspace): the same kernels on the same input, so every output is
identical; two calls in a row, the second smaller, as the static scratch
keeps the first call's contents.  Also the size limit."""
import ctypes

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


def _same(M, ref, got):
    for key in ("Q", "RPt", "piv", "diagR"):
        assert bool((ref[key] == got[key]).all().item()), key
    for key in ("k", "err", "a_fro"):
        assert ref[key] == got[key], key


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_workspace_entry(M, prec):
    import torch
    print(f"case no-alloc qrcp prec={prec}", flush=True)
    for (m, n, k, seed) in ((700, 520, 300, 60), (130, 90, 40, 61)):   # second call smaller
        a = synth.cgauss(synth.rng(seed), (m, n)) * np.exp(-np.arange(n) / (n / 4.0))[None, :]
        if prec == 1:
            a = a.astype(np.complex64).astype(np.complex128)
        A = M.colmajor(a, prec)
        ref = M.qrcp_truncate(A, k, prec)
        got = M.qrcp_truncate_noalloc(A, k, prec)
        torch.cuda.synchronize()
        _same(M, ref, got)
        # and the oracle, at the parity bar
        o = oracle.qrcp(a, k)
        scale = np.linalg.norm(a)
        assert abs(got["err"] - o["err"]) <= TOL[prec] * scale
        if prec == 0:
            assert list(got["piv"].cpu().numpy()[:k]) == list(o["piv"][:k])


def test_noalloc_refuses_problems_beyond_its_scratch(M):
    import torch
    cap = int(M.lib().qrcp_noalloc_scratch_bytes())
    assert cap == 64 << 20
    m = n = 2048                                   # FP64 needs about 140 MiB
    assert M.qrcp_work_bytes(m, n, n, M.MPS_FP64) > cap
    A = torch.zeros((n, m), dtype=torch.complex128, device="cuda").transpose(0, 1)
    with pytest.raises(M.MpsError) as e:
        M.qrcp_truncate_noalloc(A, n, M.MPS_FP64)
    assert e.value.status == 2 and "static array" in str(e.value)
