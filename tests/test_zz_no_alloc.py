"""qcur_probs_noalloc, the entry point that allocates nothing (its partial
sums live in the library's static device scratch), against qcur_probs with
a caller workspace on the same inputs: bitwise equal results on two calls in
a row, the second with a smaller matrix, and the host-side refusal of a
matrix too large for the scratch."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

Q = pytest.importorskip("paper_2402_19147_amd.qcur")
DEV = torch.device("cuda:0")


def _noalloc(A, sampling):
    _, m, n = A.shape
    p = torch.full((n,), -1.0, dtype=torch.float64, device=DEV)
    q = torch.full((m,), -1.0, dtype=torch.float64, device=DEV)
    f2 = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
    st = Q.lib().qcur_probs_noalloc(Q._h(A), Q._qp(A), sampling, Q._ptr(p), Q._ptr(q), Q._ptr(f2))
    return st, p, q, f2


def _reference(A, sampling):
    _, m, n = A.shape
    p = torch.empty(n, dtype=torch.float64, device=DEV)
    q = torch.empty(m, dtype=torch.float64, device=DEV)
    f2 = torch.empty(1, dtype=torch.float64, device=DEV)
    ws = torch.empty(Q.lib().qcur_probs_workspace(m, n), dtype=torch.uint8, device=DEV)
    st = Q.lib().qcur_probs(Q._h(A), Q._qp(A), sampling, Q._ptr(p), Q._ptr(q), Q._ptr(f2), Q._ptr(ws), ws.numel())
    assert st == 0
    return p, q, f2


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_probs_noalloc_matches_probs_twice(dtype):
    rng = np.random.default_rng(17)
    # two calls in a row on the shared scratch, the second with a smaller matrix
    for (m, n) in ((2048, 3000), (300, 257)):
        A = torch.tensor(rng.standard_normal((4, m, n)), dtype=dtype, device=DEV)
        for sampling in (Q.LENGTH, Q.UNIFORM):
            st, p, q, f2 = _noalloc(A, sampling)
            assert st == 0
            pr, qr, fr = _reference(A, sampling)
            Q.sync_status()
            assert torch.equal(p, pr) and torch.equal(q, qr) and torch.equal(f2, fr)


def test_probs_noalloc_refuses_oversize():
    # partial sums of a 40000 x 40000 matrix do not fit the scratch: refused
    # on the host before anything is enqueued (the pointer is never read)
    h = Q.handle(0).bind()
    big = Q.QMat(0x10000, 40000, 40000, 40000, 40000 * 40000, Q.F32)
    st = Q.lib().qcur_probs_noalloc(h, ctypes.byref(big), Q.LENGTH, ctypes.c_void_p(0x10000),
                                    ctypes.c_void_p(0x10000), None)
    assert st == 8 and "scratch" in Q.lib().qcur_last_error().decode()
