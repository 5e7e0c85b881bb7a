"""Write the oracle's result for the chi = 4096 two-site update that bench.py
times (tests/golden/chi4096_fp64.json, chi4096_c64.json).

Calls only ``oracle`` (and the seeded input generators of ``synth``): the
inputs are the canonical pair of the headline workload built on the CPU
(seed 0, middle-bond spectrum exp(-k/600), Haar 4x4 gate), in complex128 for
the FP64 file and rounded to complex64 (then read as FP64) for the mixed file.
The full greedy pivoted QR of the 8192 x 8192 theta takes about ten minutes
on eight cores, so the result is stored rather than recomputed by the tests.

The isometries come from LAPACK's QR (numpy), whose last bits depend on the
BLAS kernel and thread count; the inputs are therefore built by
synth.headline_pair, in a child process with OpenBLAS pinned to its Haswell
kernels and eight threads, which gives the same bytes on any x86-64 host
with AVX2.

Stored: a SHA-256 of the input bytes (a test that regenerates the inputs on
another host checks it before comparing), k, ||theta||^2, eps^2, the norm
fidelity factor, all k pivots with their relative margins, every 16th R_jj,
and theta_T = Q_k R_k P^T at 512 seeded positions (row 2l + a', column
2r + b', the oracle's layout).

    python tests/golden/make_chi4096.py [fp64|c64 ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2505_06119_amd import synth  # noqa: E402

CHI = 4096
HERE = os.path.dirname(os.path.abspath(__file__))


def inputs(prec: str):
    """The headline inputs (seed 0), built with the pinned BLAS settings."""
    a, b, g = synth.headline_pair(CHI, 0)
    if prec == "c64":
        a = a.astype(np.complex64).astype(np.complex128)
        b = b.astype(np.complex64).astype(np.complex128)
    return a, b, g


def input_digest(a, b, g) -> str:
    return synth.input_digest(a, b, g)


def sample_positions(n_rows: int, n_cols: int, count: int = 512):
    r = np.random.default_rng(4096)
    return r.integers(0, n_rows, count), r.integers(0, n_cols, count)


def main(precs):
    for prec in precs:
        t0 = time.time()
        a, b, g = inputs(prec)
        digest = input_digest(a, b, g)
        u = oracle.two_site_update(a, b, g, CHI)
        k = u["k"]
        q = u["A"].reshape(2 * CHI, k)                       # rows 2l + a'
        rp = u["B"].transpose(0, 2, 1).reshape(k, 2 * CHI)   # columns 2r + b'
        ri, ci = sample_positions(2 * CHI, 2 * CHI)
        tt = np.einsum("sk,ks->s", q[ri, :], rp[:, ci])
        err2 = u["err"] ** 2
        out = {
            "what": "oracle two-site update, chi 4096 headline workload (seed 0)",
            "precision": prec,
            "input_sha256": digest,
            "k": k,
            "norm2": u["norm2"],
            "err2": err2,
            "retained": 1.0 - err2 / u["norm2"],
            "piv": [int(x) for x in u["piv"][:k]],
            "gaps": [float("%.4e" % x) for x in u["gaps"]],
            "diagR_every16": [float(x) for x in u["diagR"][::16]],
            "theta_T_rows": [int(x) for x in ri],
            "theta_T_cols": [int(x) for x in ci],
            "theta_T_re": [float(x) for x in tt.real],
            "theta_T_im": [float(x) for x in tt.imag],
            "oracle_seconds": round(time.time() - t0, 1),
            "oracle_threads": oracle.num_threads(),
        }
        path = os.path.join(HERE, f"chi4096_{prec}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, separators=(",", ":"))
        print(f"{path}: eps^2 {err2:.12e} retained {out['retained']:.12e} "
              f"({out['oracle_seconds']} s, {out['oracle_threads']} threads)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["fp64", "c64"])
