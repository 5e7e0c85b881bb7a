"""Fusion of consecutive two-site operations on the same bond (host side).

A routed circuit on an MPS chain (Sec. III-C, gates applied to neighbouring
sites; Sec. III-D.2, 2D circuits embedded in the chain and re-embedded by
SWAP networks) holds many consecutive two-site operations on one bond: the
paired single-qubit gates and the fSim that follows them, a gate and the SWAP
that moves its qubits on.  Each operation is one contraction and one
truncated decomposition.  Operations on disjoint sites commute, so an
operation on bond b can be merged into the previous operation on b whenever
no operation has touched sites b or b+1 in between: the 4x4 matrices
multiply (later one on the left) and one update replaces two.  Without
truncation the state is unchanged; with truncation there are fewer
truncations, at different points of the circuit.
"""
from __future__ import annotations

import numpy as np


def flatten(layers):
    """The sequential (bond, 4x4 gate) list of a list of layers."""
    return [(int(i), np.asarray(g, dtype=np.complex128).reshape(4, 4)) for layer in layers for i, g in layer]


def fuse(ops):
    """Merge each operation into the previous one on the same bond when no
    operation has touched either of its sites since.  Returns the fused
    sequential list (same semantics without truncation)."""
    out = []
    last = {}   # site -> index in out of the last operation touching it
    for i, g in ops:
        j = last.get(i)
        if j is not None and last.get(i + 1) == j and out[j][0] == i:
            out[j] = (i, g @ out[j][1])
        else:
            out.append((i, np.array(g, dtype=np.complex128)))
            last[i] = last[i + 1] = len(out) - 1
    return out


def pack_layers(ops):
    """Group a sequential list into layers of increasing, disjoint bonds
    (i[t+1] >= i[t] + 2), keeping the sequential order (a new layer starts
    whenever the next bond is not at least two above the previous one)."""
    layers, cur, prev = [], [], None
    for i, g in ops:
        if prev is not None and i < prev + 2:
            layers.append(cur)
            cur = []
        cur.append((i, g))
        prev = i
    if cur:
        layers.append(cur)
    return layers


def fuse_layers(layers):
    """fuse() over the layers' sequential order, packed back into layers."""
    return pack_layers(fuse(flatten(layers)))
