"""Routing of circuits onto the MPS chain and fusion of same-bond operations
(host side).

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

route_lazy places a circuit on logical qubits onto the chain on demand
instead of re-embedding the whole register between fixed orders: a
two-qubit gate on qubits at distance d moves one of them d - 1 sites by SWAP
updates and leaves it there, and single-qubit gates wait on their qubit and
join its next two-qubit gate (the approach the paper's state-of-the-art
comparison, Sec. IV, credits to quimb as the more robust one).
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


_SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def route_lazy(n: int, ops, order):
    """Place ("1q", q, U) / ("2q", a, b, U) operations on logical qubits onto
    an n-site chain whose position p holds qubit order[p].

    A two-qubit gate whose qubits are not neighbours first moves b towards a
    by SWAP updates; b stays where it arrives.  The gate, with the pending
    single-qubit gates of a and b folded in (U kron(u_a, u_b)) and re-oriented
    when b sits left of a (SWAP U SWAP), is one update on their bond.  Pending
    single-qubit gates left at the end become updates with a neighbour.
    Returns the sequential (bond, 4x4) list and the final order."""
    order = list(order)
    pos = {q: p for p, q in enumerate(order)}
    pend = {}
    out = []
    for op in ops:
        if op[0] == "1q":
            _, q, u = op
            pend[q] = np.asarray(u, dtype=np.complex128) @ pend.get(q, _I2)
            continue
        _, a, b, u = op
        while abs(pos[a] - pos[b]) > 1:
            pb = pos[b]
            pn = pb - 1 if pos[a] < pb else pb + 1
            qn = order[pn]
            out.append((min(pb, pn), _SWAP))
            order[pb], order[pn] = qn, b
            pos[qn], pos[b] = pb, pn
        g = np.asarray(u, dtype=np.complex128) @ np.kron(pend.pop(a, _I2), pend.pop(b, _I2))
        if pos[a] > pos[b]:
            g = _SWAP @ g @ _SWAP
        out.append((min(pos[a], pos[b]), g))
    for q in sorted(pend):
        p = pos[q]
        out.append((p, np.kron(pend[q], _I2)) if p + 1 < n else (p - 1, np.kron(_I2, pend[q])))
    return out, order
