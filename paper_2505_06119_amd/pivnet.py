"""Training of the pivot-proposal network on the GPU with the library's kernels.

Training data are theta matrices built by the library itself (mps_theta on
canonical site pairs with a range of bond spectra and Haar gates); labels mark
the columns that plain pivoted QR (qrcp_truncate) selects among its first k
pivots; features come from the library's sketch (pivnet_features).  The loss
gradient and the Adam step are the library's own kernels (pivnet_grad,
pivnet_adam).  Weights are stored as JSON text (97 float32 values).

    python -m paper_2505_06119_amd.pivnet --out paper_2505_06119_amd/pivnet_weights.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import mps as M
from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "pivnet_weights.json")


def init_params(seed: int = 0) -> np.ndarray:
    r = synth.rng(seed)
    p = np.zeros(M.PIVNET_PARAMS, dtype=np.float32)
    h, f = 16, M.PIVNET_FEATURES
    p[: h * f] = r.standard_normal(h * f) * 0.5
    p[h * f + h: h * f + 2 * h] = r.standard_normal(h) * 0.5
    return p


def to_device(p: np.ndarray):
    import torch
    return torch.from_numpy(np.asarray(p, dtype=np.float32).copy()).cuda()


def save(p, path: str):
    arr = p.detach().cpu().numpy() if hasattr(p, "detach") else np.asarray(p)
    with open(path, "w") as fh:
        json.dump({"format": "pivnet 4-16-1 tanh, float32", "params": [float(x) for x in arr]}, fh, indent=1)


def load(path: str = DEFAULT_WEIGHTS) -> np.ndarray:
    with open(path) as fh:
        return np.asarray(json.load(fh)["params"], dtype=np.float32)


def make_sample(seed: int, chi: int, prec: int, sketch_rows: int = 64, scale=None):
    """(phi, labels, theta) for one synthetic two-site theta of bond chi."""
    import torch
    r = synth.rng(seed)
    if scale is None:
        scale = float(np.exp(r.uniform(np.log(chi / 16.0), np.log(chi * 4.0))))
    a, b = synth.canonical_pair_device(r, chi, chi, chi, synth.exp_spectrum(chi, scale))
    g = synth.haar_unitary(r, 4)
    cd = M.cdtype(prec)
    theta = M.mps_theta(a.to(cd).contiguous(), b.to(cd).contiguous(), g, chi, chi, chi, prec)
    q = M.qrcp_truncate(theta, chi, prec)
    labels = torch.zeros(2 * chi, dtype=torch.uint8, device="cuda")
    labels[q["piv"][:chi].long()] = 1
    phi = M.pivnet_features(theta, prec, sketch_rows=sketch_rows, seed=seed + 17)
    return phi, labels, theta


def train(params, data, steps: int = 400, lr: float = 3e-3, log_every: int = 100):
    """Adam on the mean logistic loss, cycling through the samples."""
    import torch
    m1 = torch.zeros(M.PIVNET_PARAMS, dtype=torch.float32, device="cuda")
    m2 = torch.zeros_like(m1)
    hist = []
    for t in range(1, steps + 1):
        phi, lab = data[(t - 1) % len(data)][:2]
        g = M.pivnet_grad(params, phi, lab)
        M.pivnet_adam(params, g, m1, m2, t, lr)
        if t % log_every == 0 or t == 1:
            loss = float(g[M.PIVNET_PARAMS].item())
            hist.append((t, loss))
            print(f"[pivnet] step {t} loss {loss:.4f}", flush=True)
    return hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--samples", type=int, default=48)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--prec", type=int, default=M.MPS_MIXED)
    args = ap.parse_args()
    t0 = time.time()
    chis = [64, 128, 256, 512]
    data = [make_sample(1000 + s, chis[s % len(chis)], args.prec) for s in range(args.samples)]
    print(f"[pivnet] {len(data)} samples in {time.time() - t0:.1f} s", flush=True)
    params = to_device(init_params(0))
    train(params, data, steps=args.steps)
    save(params, args.out)
    print(f"[pivnet] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
