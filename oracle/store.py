"""Temporal subsampling, linear interpolation and storage accounting (Section 2, Fig. 1b, Fig. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Subsampling keeps the interface fields of every k-th step only and rebuilds
the missing steps by linear interpolation in time (Section 2).  The kept
steps are anchored at the end of the run, where the reverse pass starts:
    K = {T-1, T-1-k, T-1-2k, ...}  (ceil(T/k) steps, all >= 0)
plus an exact zero anchor at step -1 (every field is zero before the run).
For a step n between kept neighbours n0 < n < n1 (n0 possibly the anchor):
    w = (n - n0) / (n1 - n0),   v(n) = (1 - w) v(n0) + w v(n1).

The compression factor of the Fig. 3 caption is the bit-width ratio to
float32 times k; storage bytes count the payload of the kept steps.
"""

from __future__ import annotations

import math

from .codec import STORAGE_BITS


def kept_steps(T: int, k: int):
    """K in decreasing order (the order the reverse pass meets them)."""
    return [T - 1 - j * k for j in range(math.ceil(T / k))]


def bracket(n: int, T: int, k: int):
    """(n0, n1, w) for step n; n in K gives (n, n, 0.0); n0 = -1 is the zero anchor."""
    if (T - 1 - n) % k == 0:
        return n, n, 0.0
    j1 = (T - 1 - n) // k
    n1 = T - 1 - j1 * k
    n0 = n1 - k
    if n0 < 0:
        n0 = -1
    return n0, n1, (n - n0) / (n1 - n0)


def interpolate(n: int, T: int, k: int, kept: dict, zero):
    """Value at step n from the kept values {step: array}; the anchor -1 is ``zero``."""
    n0, n1, w = bracket(n, T, k)
    if n0 == n1:
        return kept[n]
    v0 = zero if n0 == -1 else kept[n0]
    v1 = kept[n1]
    return (1.0 - w) * v0 + w * v1


def cubic_nodes(n: int, T: int, k: int):
    """Nodes and weights of the cubic reconstruction at step n (an option beside the
    paper's linear interpolation, not from the paper).

    The nodes are the zero anchor -1 and the kept steps, in increasing time order.  For
    n strictly between two neighbouring nodes, the four consecutive nodes with n in the
    middle interval are used, shifted inward at either end of the run; the weights are
    those of the Lagrange polynomial of degree 3 through them, evaluated at n.  Returns
    [(node, weight)]; a kept n gives [(n, 1.0)].  With fewer than four nodes the linear
    rule applies.
    """
    kept = sorted(kept_steps(T, k))
    if n in kept:
        return [(n, 1.0)]
    nodes = [-1] + kept
    if len(nodes) < 4:
        n0, n1, w = bracket(n, T, k)
        return [(n0, 1.0 - w), (n1, w)]
    i = max(j for j in range(len(nodes)) if nodes[j] < n)       # nodes[i] < n < nodes[i + 1]
    s = min(max(i - 1, 0), len(nodes) - 4)
    sel = nodes[s:s + 4]
    out = []
    for a in sel:
        w = 1.0
        for b in sel:
            if b != a:
                w *= (n - b) / (a - b)
        out.append((a, w))
    return out


def interpolate_cubic(n: int, T: int, k: int, kept: dict, zero):
    """Value at step n from the kept values {step: array} by cubic_nodes; the anchor -1 is ``zero``."""
    total = None
    for node, w in cubic_nodes(n, T, k):
        v = zero if node == -1 else kept[node]
        total = w * v if total is None else total + w * v
    return total


def shell_values_per_step(nx: int, ny: int, nz: int, pml: int) -> int:
    """Tangential H on the 3 low faces + tangential E on the 3 high faces, interior extent."""
    if pml == 0:
        return 0
    mx, my, mz = nx - 2 * pml, ny - 2 * pml, nz - 2 * pml
    return 4 * (my * mz + mx * mz + mx * my)


def storage_bytes(nx, ny, nz, pml, T, k, mode):
    """(payload bytes, scale bytes) of the interface store."""
    slices = math.ceil(T / k)
    payload = shell_values_per_step(nx, ny, nz, pml) * slices * STORAGE_BITS[mode] // 8
    scales = slices * 12 * 4 if mode == "fp8_e4m3fn_scaled" else 0
    return payload, scales


def compression_factor(mode: str, k: int) -> float:
    """Fig. 3 caption: memory saved by the smaller bit width times k, relative to float32, k = 1."""
    return 32.0 / STORAGE_BITS[mode] * k
