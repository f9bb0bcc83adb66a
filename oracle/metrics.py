"""Gradient-agreement metrics.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np


def cosine_similarity(x, y) -> float:
    """Eq. 2: S(x, y) = x . y / (||x|| ||y||) over the flattened arrays, in FP64."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    return float(np.dot(x, y) / (np.linalg.norm(x) * np.linalg.norm(y)))


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 in FP64."""
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
