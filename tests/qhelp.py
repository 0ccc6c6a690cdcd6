"""Small helpers shared by the tests (not part of the checker or the library)."""
import numpy as np

from oracle.quat import chi, unchi


def random_isometry(rows: int, cols: int, rng) -> np.ndarray:
    """A quaternion matrix with orthonormal columns (Q^H Q = I): the polar
    factor of a Gaussian matrix, computed on its complex adjoint."""
    X = rng.standard_normal((4, rows, cols))
    M = chi(X)
    H = M.conj().T @ M
    ev, V = np.linalg.eigh(H)
    Q = M @ (V / np.sqrt(ev)) @ V.conj().T
    return unchi(Q, rows, cols)


def lowrank_svd_form(m: int, n: int, sigmas, rng):
    """X = Wk diag(sigmas) Vk^H with random isometries Wk (m x k), Vk (n x k)."""
    from oracle.quat import qmul, qH
    k = len(sigmas)
    Wk = random_isometry(m, k, rng)
    Vk = random_isometry(n, k, rng)
    S = np.zeros((4, k, k))
    S[0] = np.diag(sigmas)
    return qmul(qmul(Wk, S), qH(Vk)), Wk, Vk


def basis(name: str) -> np.ndarray:
    e = np.zeros((4, 1, 1))
    e[{"1": 0, "i": 1, "j": 2, "k": 3}[name], 0, 0] = 1.0
    return e
