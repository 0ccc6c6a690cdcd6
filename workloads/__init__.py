"""Seeded synthetic inputs for the quaternion CUR workloads.

This module is shared by the tests, the benchmark and the reference
checker.  It only draws random numbers and does plain real arithmetic
(scaling, adding noise, real matrix products of real factors); it holds
none of the CUR method's own arithmetic (no quaternion products, no
norms used for sampling, no pseudoinverses, no sampling of index sets
from data-dependent probabilities).

Quaternion matrices are numpy arrays of shape (4, rows, cols) in float64;
plane 0 is the real part, planes 1..3 the i, j and k parts.

Where a workload is a product of two quaternion factors, the generator
returns the factors and the caller forms the product with its own
quaternion multiplication (the checker with its plain CPU code, the
benchmark with the library).

Workloads (sizes as used by the benchmark and the large parity tests):
  * lowrank_gaussian: A = L * Rt with L (m x k) and Rt (k x n) quaternion,
    all four components i.i.d. N(0,1), optional N(0, noise^2) on every plane.
  * color_like: a pure quaternion matrix shaped like a colour image: the
    imaginary planes are F @ G_c with F (m x k) and G_c (k x n) i.i.d.
    U(0,1), divided by their global maximum so that values lie in [0,1],
    plus N(0, noise^2) on the imaginary planes only.
  * batch_problems: many pure quaternion problems of uneven sizes with real
    Gaussian factors F (m x k), G_c (k x n) and N(0, noise^2) on the
    imaginary planes.
  * bernoulli_mask: a uint8 observation mask with P(1) = p.
  * uniform_index_set: a fixed, sorted index set drawn uniformly without
    replacement (used where an index set is an input, not a draw of the
    method).
  * perturbation_factors: the inputs of the Theorem 1 experiment
    (Example 4.1): Gaussian quaternion matrices whose polar factors the
    caller takes as W_k and V_k, the positive diagonal of Sigma_k and a
    unit Gaussian noise matrix E0 (the caller scales it).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for",
    "lowrank_gaussian_factors",
    "color_like",
    "batch_problems",
    "bernoulli_mask",
    "uniform_index_set",
    "perturbation_factors",
    "gaussian_quat",
    "small_int_quat",
    "WORKLOADS",
]


def rng_for(seed: int, *path: int) -> np.random.Generator:
    """A PCG64 generator for the stream (seed, *path) via SeedSequence."""
    ss = np.random.SeedSequence([int(seed), *[int(p) for p in path]])
    return np.random.Generator(np.random.PCG64(ss))


def gaussian_quat(rows: int, cols: int, rng: np.random.Generator, std: float = 1.0) -> np.ndarray:
    return rng.standard_normal((4, rows, cols)) * std


def small_int_quat(rows: int, cols: int, rng: np.random.Generator, lim: int = 4) -> np.ndarray:
    """Integer-valued entries in [-lim, lim]; exact in every tested precision."""
    return rng.integers(-lim, lim + 1, size=(4, rows, cols)).astype(np.float64)


def lowrank_gaussian_factors(m: int, n: int, k: int, seed: int, noise: float = 0.0):
    """Factors of A = L * Rt (+ noise).

    Returns (L, Rt, E): L (4,m,k), Rt (4,k,n) with i.i.d. N(0,1) components
    and E (4,m,n) i.i.d. N(0, noise^2) on every plane (zeros if noise == 0).
    """
    L = gaussian_quat(m, k, rng_for(seed, 0))
    Rt = gaussian_quat(k, n, rng_for(seed, 1))
    if noise > 0:
        E = rng_for(seed, 2).standard_normal((4, m, n)) * noise
    else:
        E = np.zeros((4, m, n))
    return L, Rt, E


def color_like(m: int, n: int, k: int, seed: int, noise: float = 0.01) -> np.ndarray:
    """Pure quaternion, colour-image-shaped, quaternion rank k plus noise.

    Imaginary plane c is F @ G_c / s with F (m x k), G_c (k x n) i.i.d.
    U(0,1) and s the maximum over all three products, so the noiseless
    values lie in [0, 1] and the matrix has quaternion rank k (the left
    factor is real).  N(0, noise^2) is added to planes 1..3; no clipping.
    """
    r = rng_for(seed, 0)
    F = r.random((m, k))
    G = rng_for(seed, 1).random((3, k, n))
    P = np.stack([F @ G[c] for c in range(3)])
    P /= P.max()
    A = np.zeros((4, m, n))
    A[1:] = P
    if noise > 0:
        A[1:] += rng_for(seed, 2).standard_normal((3, m, n)) * noise
    return A


def batch_problems(count: int, seed: int, mn_range=(64, 512), k_range=(8, 32), noise: float = 1e-3):
    """Uneven batch: per problem m, n ~ U{mn_range}, k ~ U{k_range} i.i.d.

    Each problem is pure quaternion F @ (G1 i + G2 j + G3 k) with F (m x k)
    and G_c (k x n) i.i.d. N(0,1), plus N(0, noise^2) on planes 1..3.
    Returns a list of dicts {A, m, n, k}.
    """
    sizes = rng_for(seed, 0)
    out = []
    for b in range(count):
        m = int(sizes.integers(mn_range[0], mn_range[1] + 1))
        n = int(sizes.integers(mn_range[0], mn_range[1] + 1))
        k = int(sizes.integers(k_range[0], k_range[1] + 1))
        r = rng_for(seed, 1, b)
        F = r.standard_normal((m, k))
        G = r.standard_normal((3, k, n))
        A = np.zeros((4, m, n))
        for c in range(3):
            A[1 + c] = F @ G[c]
        if noise > 0:
            A[1:] += r.standard_normal((3, m, n)) * noise
        out.append({"A": A, "m": m, "n": n, "k": k})
    return out


def bernoulli_mask(m: int, n: int, p: float, seed: int) -> np.ndarray:
    return (rng_for(seed, 7).random((m, n)) < p).astype(np.uint8)


def uniform_index_set(n: int, count: int, seed: int, stream: int) -> np.ndarray:
    """Sorted int64 index set drawn uniformly without replacement."""
    idx = rng_for(seed, 9, stream).choice(n, size=count, replace=False)
    return np.sort(idx).astype(np.int64)


# The five workloads with their sizes.  "product" marks workloads whose
# matrix is the quaternion product L * Rt (+E) formed by the caller.
def perturbation_factors(m: int, n: int, k: int, seed: int):
    """Inputs of the Theorem 1 experiment (Example 4.1).

    Returns (GW, GV, sig, E0): GW (4,m,k) and GV (4,n,k) with i.i.d. N(0,1)
    components (the caller orthonormalises them: the polar factor of each is
    the unitary W_k, V_k), sig (k,) i.i.d. U(1, 10) sorted descending (the
    positive diagonal of Sigma_k) and E0 (4,m,n) i.i.d. N(0,1) (the noise
    E = s * E0 for a scale s chosen by the caller).
    """
    GW = gaussian_quat(m, k, rng_for(seed, 0))
    GV = gaussian_quat(n, k, rng_for(seed, 1))
    sig = np.sort(1.0 + 9.0 * rng_for(seed, 2).random(k))[::-1].copy()
    E0 = gaussian_quat(m, n, rng_for(seed, 3))
    return GW, GV, sig, E0


WORKLOADS = {
    "plain_f64_256": dict(kind="product", m=256, n=256, k=10, noise=0.0, c=40, r=40,
                          sampling="uniform", core="wpinv", seed=1),
    "color_1024": dict(kind="color", m=1024, n=1024, k=50, noise=0.01, c=200, r=200,
                       sampling="length", core="car", seed=2),
    "dense_4096": dict(kind="product", m=4096, n=4096, k=100, noise=1e-3, c=400, r=400,
                       sampling="length", core="car", seed=3),
    "batch_512": dict(kind="batch", count=512, mn_range=(64, 512), k_range=(8, 32),
                      noise=1e-3, sampling="length", core="car", seed=4),
    "adjoint_2048": dict(kind="product", m=2048, n=2048, k=64, noise=0.0, c=256, r=256,
                         sampling="fixed", core="wpinv", max_rank=64, mask_p=0.5, seed=5),
    # completion (Algorithm 2): colour-image-shaped 512 x 768 (the size of the
    # paper's completion test images), rank 20 + N(0, 0.01^2), 70% missing,
    # c = r = ceil(20 ln 20) = 60 fixed uniform index sets, t_max 200, tol 1e-4
    "complete_512x768": dict(kind="color", m=512, n=768, k=20, noise=0.01, c=60, r=60, mask_p=0.3,
                             max_iter=200, tol=1e-4, seed=6),
    # Example 4.2 shape: rank 10 plus noise, QMCUR against the QSVD baseline
    "qsvd_500": dict(kind="product", m=500, n=500, k=10, noise=1e-4, sampling="length", core="car", seed=7),
    # Example 4.1: X = W_k Sigma_k V_k^H (500 x 500, k = 50) plus Gaussian noise
    # N(0, sigma^2) in every component, c = r = ceil(k ln k)
    "theorem1_500": dict(kind="perturbation", m=500, n=500, k=50,
                         sigmas=[1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6], sampling="length", seed=11),
}
