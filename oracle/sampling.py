"""Sampling probabilities and the index sampler (Section 3.1 and
Algorithm 1, steps 1-2).

Part of the FP64 reference checker (test infrastructure only).

The paper names the two probability families (QMCUR_length and
QMCUR_uniform) but not how indices are drawn from them.  The reading used
here, shared with the library so that draws can be compared bit for bit:

  1. integer weights w_j = floor(p_j * 2^60), exact for p_j in [0, 1];
  2. inclusive prefix sums S_j of the current weights, exact in integers;
  3. draw t uses u = the n-th output of SplitMix64 seeded with `seed`,
     n = set_id * 2^32 + t (Steele, Lea, Flood, OOPSLA 2014);
  4. target tau = floor(u * T / 2^64) with T the current weight total;
  5. pick the smallest j with S_j > tau;
  6. without replacement, remove j (T -= w_j, w_j = 0) before the next draw;
  7. the index set is returned sorted ascending (0-based).
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
SPLITMIX_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_mix(z: int) -> int:
    """SplitMix64 output function (the 'mix64' variant of Steele et al.)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_nth(seed: int, n: int) -> int:
    """The n-th (0-based) output of SplitMix64 started from state `seed`.

    The generator adds the golden-gamma constant to its state and mixes the
    new state, so output n is mix(seed + (n + 1) * gamma mod 2^64).
    """
    return splitmix64_mix((seed + (n + 1) * SPLITMIX_GAMMA) & MASK64)


def uniform64(seed: int, set_id: int, t: int) -> int:
    return splitmix64_nth(seed & MASK64, ((set_id & 0xFFFFFFFF) << 32) + t)


def probs_length(A: np.ndarray):
    """QMCUR_length (Section 3.1): p_j = ||X(:,j)||^2 / ||X||_F^2 over columns,
    q_i = ||X(i,:)||^2 / ||X||_F^2 over rows.  |x|^2 sums the four planes.

    Returns (p, q, fro2).  Raises ValueError when ||X||_F = 0.
    """
    sq = A * A
    col2 = sq.sum(axis=(0, 1))
    row2 = sq.sum(axis=(0, 2))
    f2 = float(col2.sum())
    if not np.isfinite(f2) or f2 <= 0.0:
        raise ValueError("length probabilities need a finite, nonzero Frobenius norm")
    return col2 / f2, row2 / f2, f2


def probs_uniform(m: int, n: int):
    """QMCUR_uniform (Section 3.1): p_j = 1/n and q_i = 1/m."""
    return np.full(n, 1.0 / n), np.full(m, 1.0 / m)


def weights(p: np.ndarray) -> list:
    """w_j = floor(p_j * 2^60) as exact Python integers."""
    w = []
    for x in np.asarray(p, dtype=np.float64):
        x = float(x)
        if not math.isfinite(x) or x < 0.0 or x > 1.0:
            raise ValueError("probabilities must lie in [0, 1]")
        w.append(int(math.floor(x * 2.0 ** 60)))
    return w


def draw(p: np.ndarray, count: int, seed: int, set_id: int, with_replacement: bool = False) -> np.ndarray:
    """Draw `count` indices from the probabilities p (steps 1-7 above)."""
    w = weights(p)
    n = len(w)
    if count < 0:
        raise ValueError("count must be >= 0")
    if count == 0:
        return np.zeros(0, dtype=np.int64)
    if not with_replacement and sum(1 for x in w if x > 0) < count:
        raise ValueError("fewer positive weights than draws")
    if sum(w) == 0:
        raise ValueError("all weights are zero")
    out = []
    for t in range(count):
        T = sum(w)
        tau = (uniform64(seed, set_id, t) * T) >> 64
        # smallest j with inclusive prefix sum S_j > tau
        s = 0
        for j in range(n):
            s += w[j]
            if s > tau:
                break
        out.append(j)
        if not with_replacement:
            w[j] = 0
    return np.array(sorted(out), dtype=np.int64)
