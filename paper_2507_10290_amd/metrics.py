"""Host-side evaluation of returned trajectories (not part of the GPU path).

e_simi (Sec. IV, segment-count study): lg of the summed distance between the
trajectory and its reference curve at M points uniformly spaced in time,
e_simi = lg(sum_i |p_i - p_ref_i|), with M = 8192 as in the paper.
"""
from __future__ import annotations

import numpy as np


def evaluate(coeffs: np.ndarray, durations: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Positions of one trajectory at global times t: coeffs [N, 3, n] monomial in local time."""
    starts = np.concatenate([[0.0], np.cumsum(durations)[:-1]])
    idx = np.clip(np.searchsorted(starts, t, side="right") - 1, 0, len(durations) - 1)
    tau = t - starts[idx]
    n = coeffs.shape[2]
    powers = tau[:, None] ** np.arange(n)[None, :]                   # [M, n]
    return np.einsum("man,mn->ma", coeffs[idx], powers)


def e_simi(coeffs: np.ndarray, durations: np.ndarray, reference, m: int = 8192) -> float:
    """reference(t) -> [len(t), 3] positions of the reference at global times t."""
    total = float(np.sum(durations))
    t = (np.arange(m) + 0.5) * total / m
    d = np.linalg.norm(evaluate(coeffs, durations, t) - reference(t), axis=1)
    return float(np.log10(np.sum(d)))
