"""Differentiation through the gathers and the pseudoinverse (MI355X):
the masked CUR loss and the CUR map against the FP64 reference gradients
and FP64 central differences (h = 1e-6), small and at the full adjoint
workload (2048 x 2048, rank 64, c = r = 256, max_rank 64, Bernoulli(0.5)
mask, FP32 adjoint)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.quat import qmul, fro2, inner
from oracle.grad import cur_vjp, masked_loss, masked_loss_grad, central_difference

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2402_19147_amd")
DEV = torch.device("cuda:0")


def T(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def N(t):
    return t.detach().to(torch.float64).cpu().numpy()


def rel(x, ref):
    return np.sqrt(fro2(x - ref)) / np.sqrt(fro2(ref))


@pytest.fixture(autouse=True)
def _clean():
    q.sync_status()
    yield
    q.sync_status()


def _small(seed=3, noise=0.05):
    L, Rt, E = workloads.lowrank_gaussian_factors(80, 72, 4, seed, noise)
    A = qmul(L, Rt) + E
    rng = np.random.default_rng(seed)
    I = np.sort(rng.choice(80, 12, replace=False))
    J = np.sort(rng.choice(72, 10, replace=False))
    mask = (rng.random((80, 72)) < 0.5).astype(np.uint8)
    return A, I, J, mask, rng


def test_cur_loss_value_and_gradient_f64():
    A, I, J, mask, _ = _small()
    At = T(A).requires_grad_(True)
    loss = q.cur_loss(At, T(I, torch.int64), T(J, torch.int64), torch.tensor(mask, device=DEV))
    loss.backward()
    ref = masked_loss(A, I, J, mask)
    assert float(loss.detach()) == pytest.approx(ref, rel=1e-10)
    assert rel(N(At.grad), masked_loss_grad(A, I, J, mask)) < 1e-9


def test_cur_map_vjp_and_target_loss_f64():
    A, I, J, mask, rng = _small(4)
    Y = A + 0.01 * rng.standard_normal(A.shape)
    At = T(A).requires_grad_(True)
    B = q.cur(At, T(I, torch.int64), T(J, torch.int64))
    Mt = torch.tensor(mask, device=DEV, dtype=torch.float64)
    loss = (((T(Y) - B) * Mt) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(masked_loss(A, I, J, mask, Y=Y), rel=1e-10)
    assert rel(N(At.grad), masked_loss_grad(A, I, J, mask, Y=Y)) < 1e-9
    # finite differences of the reference loss along a random direction
    V = rng.standard_normal(A.shape)
    fd = central_difference(lambda X: masked_loss(X, I, J, mask, Y=Y), A, V, h=1e-6)
    assert inner(N(At.grad), V) == pytest.approx(fd, rel=1e-6)


@pytest.fixture(scope="module")
def adjoint_workload():
    cfg = workloads.WORKLOADS["adjoint_2048"]
    m, k, c = cfg["m"], cfg["k"], cfg["c"]
    L, Rt, _ = workloads.lowrank_gaussian_factors(m, m, k, cfg["seed"])
    A = qmul(L, Rt)
    I = workloads.uniform_index_set(m, c, cfg["seed"], 0)
    J = workloads.uniform_index_set(m, c, cfg["seed"], 1)
    mask = workloads.bernoulli_mask(m, m, cfg["mask_p"], cfg["seed"])
    return A, I, J, mask, cfg["max_rank"]


def test_adjoint_workload_exact_rank_gives_zero_gradient(adjoint_workload):
    # A has rank 64 and rank W = 64, so CUR(A) = A: the loss and its gradient vanish
    A, I, J, mask, kmax = adjoint_workload
    At = T(A, torch.float32).requires_grad_(True)
    loss = q.cur_loss(At, T(I, torch.int64), T(J, torch.int64), torch.tensor(mask, device=DEV), max_rank=kmax)
    loss.backward()
    nA = np.sqrt(fro2(A))
    assert float(loss.detach()) < (1e-5 * nA) ** 2
    assert np.sqrt(fro2(N(At.grad))) < 1e-4 * nA


def test_adjoint_workload_vjp_matches_reference(adjoint_workload):
    A, I, J, mask, kmax = adjoint_workload
    rng = np.random.default_rng(55)
    gB = rng.standard_normal(A.shape)
    At = T(A, torch.float32).requires_grad_(True)
    B = q.cur(At, T(I, torch.int64), T(J, torch.int64), max_rank=kmax)
    B.backward(T(gB, torch.float32))
    ref = cur_vjp(A, I, J, gB, max_rank=kmax)
    assert rel(N(At.grad), ref) < 1e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adjoint_workload_target_loss_against_finite_differences(adjoint_workload, dtype):
    A, I, J, mask, kmax = adjoint_workload
    rng = np.random.default_rng(56)
    Y = A + 1e-2 * rng.standard_normal(A.shape)
    At = T(A, dtype).requires_grad_(True)
    B = q.cur(At, T(I, torch.int64), T(J, torch.int64), max_rank=kmax)
    Mt = torch.tensor(mask, device=DEV, dtype=dtype)
    loss = (((T(Y, dtype) - B) * Mt) ** 2).sum()
    loss.backward()
    g = N(At.grad)
    ref = masked_loss_grad(A, I, J, mask, Y=Y, max_rank=kmax)
    # the cotangent 2 P(Y - B) is ~||A|| / ||P(Y - B)|| times more sensitive to the
    # forward rounding of B (itself ~ u * kappa(W) relative) than B is
    from oracle.grad import cur_of
    from oracle.pinv import singular_values
    W = A[:, I][:, :, J]
    sw = singular_values(W)[:kmax]
    resid = np.sqrt(fro2((Y - cur_of(A, I, J, max_rank=kmax)) * mask[None]))
    u = 2.0 ** -52 if dtype == torch.float64 else 2.0 ** -24
    tol = max(1e-8 if dtype == torch.float64 else 1e-4, 4 * u * (sw[0] / sw[-1]) * np.sqrt(fro2(A)) / resid)
    assert rel(g, ref) < tol
    # FP64 central differences pin the reference gradient at this point
    V = rng.standard_normal(A.shape)
    fd = central_difference(lambda X: masked_loss(X, I, J, mask, Y=Y, max_rank=kmax), A, V, h=1e-6)
    assert inner(ref, V) == pytest.approx(fd, rel=1e-6)
    assert abs(inner(g, V) - fd) <= tol * np.sqrt(fro2(ref)) * np.sqrt(fro2(V))
