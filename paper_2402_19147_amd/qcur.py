"""Thin ctypes binding of libqcur (include/qcur.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Quaternion matrices are torch tensors of shape (4, rows, cols) on a GPU
(plane 0 real, planes 1..3 the i, j, k parts) whose last dimension is
contiguous; float64, float32 and bfloat16 map to QCUR_F64/F32/BF16.
Workspaces are allocated as torch uint8 tensors on the same device.
Calls are enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcur.so")

F64, F32, BF16 = 0, 1, 2
BF16X3 = 3  # compute only: FP32 operands as BF16 hi + lo, three BF16 products
OP_N, OP_H = 0, 1
LENGTH, UNIFORM = 0, 1
SCRATCH_BYTES = 32 << 20  # QCUR_SCRATCH_BYTES: the static device scratch of qcur_probs_noalloc
CORE_WPINV, CORE_CAR = 0, 1

STATUS = {0: "QCUR_OK", 1: "QCUR_ERR_ARG", 2: "QCUR_ERR_SHAPE", 3: "QCUR_ERR_DTYPE",
          4: "QCUR_ERR_WORKSPACE", 5: "QCUR_ERR_SAMPLE", 6: "QCUR_ERR_NUMERIC",
          7: "QCUR_ERR_DEVICE", 8: "QCUR_ERR_UNSUPPORTED"}

_TORCH_DT = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
_QCUR_DT = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}


class QcurError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class QMat(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("pstride", ctypes.c_int64), ("dtype", ctypes.c_int32)]


_lib = None
_lock = threading.Lock()


def _declare(L):
    c_i64, c_p, c_d, c_int, c_u64, c_sz = (ctypes.c_int64, ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t)
    QP = ctypes.POINTER(QMat)
    sig = {
        "qcur_create": (c_int, [ctypes.POINTER(c_p), c_int]),
        "qcur_destroy": (c_int, [c_p]),
        "qcur_set_stream": (c_int, [c_p, c_p]),
        "qcur_sync_status": (c_int, [c_p]),
        "qcur_status_string": (ctypes.c_char_p, [c_int]),
        "qcur_last_error": (ctypes.c_char_p, []),
        "qcur_version": (c_int, []),
        "qcur_probs_workspace": (c_sz, [c_i64, c_i64]),
        "qcur_pinv_workspace": (c_sz, [c_i64, c_i64]),
        "qcur_approx_workspace": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_int, c_int]),
        "qcur_residual_workspace": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_int]),
        "qcur_backward_workspace": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_int]),
        "qcur_gemm_workspace": (c_sz, [c_i64, c_i64, c_i64, c_int]),
        "qcur_probs": (c_int, [c_p, QP, c_int, c_p, c_p, c_p, c_p, c_sz]),
        "qcur_draw": (c_int, [c_p, c_p, c_i64, c_i64, c_u64, c_u64, c_int, c_p]),
        "qcur_gather": (c_int, [c_p, QP, c_p, c_i64, c_p, c_i64, QP, QP, QP]),
        "qcur_pinv": (c_int, [c_p, QP, c_d, c_i64, QP, c_p, c_p, c_sz]),
        "qcur_gemm": (c_int, [c_p, c_int, c_int, c_d, QP, QP, c_d, QP, c_int, c_p, c_sz]),
        "qcur_approx": (c_int, [c_p, QP, QP, QP, QP, c_int, c_int, c_int, c_d, c_i64, QP, QP, c_p,
                                c_p, c_sz]),
        "qcur_residual": (c_int, [c_p, QP, QP, QP, QP, c_p, c_i64, c_int, c_p, QP, c_d, c_p, c_sz]),
        "qcur_backward": (c_int, [c_p, QP, c_p, c_i64, c_p, c_i64, QP, c_p, c_i64, c_d, c_i64, c_int,
                                  QP, c_p, c_p, c_sz]),
        "qcur_cast": (c_int, [c_p, QP, QP]),
        "qcur_solve": (c_int, [c_p, QP, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_int, c_int, c_d, c_i64, c_p,
                               c_p, QP, c_p, c_p, c_p, c_p, QP, QP, QP, QP, c_p, c_sz]),
        "qcur_solve_workspace": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_int, c_int]),
        "qcur_probs_noalloc": (c_int, [c_p, QP, c_int, c_p, c_p, c_p]),
        "qcur_batch_workspace": (c_sz, [ctypes.c_int32, c_p, c_int, c_int, c_int, c_int, c_int]),
        "qcur_batch_prepare": (c_int, [c_p, ctypes.c_int32, c_p, c_int, c_int, c_int, c_int, c_int, c_p, c_sz]),
        "qcur_batch_plans": (c_int, [c_p, c_p, c_p, c_p, c_int]),
        "qcur_complete": (c_int, [c_p, QP, c_p, c_i64, c_p, c_i64, c_p, c_i64, c_int, c_d, c_i64, c_int, c_d, QP,
                                  c_p, c_p, c_p, c_sz]),
        "qcur_complete_workspace": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_int]),
        "qcur_complete_resampled": (c_int, [c_p, QP, c_p, c_i64, c_i64, c_i64, c_int, c_u64, c_int, c_d, c_i64,
                                            c_int, c_d, QP, c_p, c_p, c_p, c_p, c_p, c_sz]),
        "qcur_complete_resampled_workspace": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_int, c_int]),
        "qcur_sample_size": (c_i64, [c_i64, c_i64]),
        "qcur_svd": (c_int, [c_p, QP, c_p, QP, QP, c_p, c_sz]),
        "qcur_svd_workspace": (c_sz, [c_i64, c_i64]),
        "qcur_solve_batched": (c_int, [c_p, ctypes.c_int32, c_p, QP, c_i64, c_int, c_int, c_u64, c_int, c_int, c_d,
                                       c_i64, c_p, c_p, QP, c_i64, c_p, c_p, c_p, c_p, QP, c_i64, c_p, c_sz]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def lib():
    """Loads the in-tree libqcur.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise ImportError(f"{LIB_PATH} is missing: build it with "
                                      "`python -m paper_2402_19147_amd.build`")
                _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _check(status: int):
    if status != 0:
        raise QcurError(status, lib().qcur_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def qmat(t: torch.Tensor) -> QMat:
    if t.dim() != 3 or t.shape[0] != 4:
        raise ValueError(f"quaternion matrices are (4, rows, cols) tensors, got {tuple(t.shape)}")
    if t.dtype not in _QCUR_DT:
        raise ValueError(f"unsupported dtype {t.dtype}")
    if t.shape[2] > 1 and t.stride(2) != 1:
        raise ValueError("the column dimension must be contiguous")
    ld = t.stride(1) if t.shape[1] > 1 else max(t.shape[2], 1)
    return QMat(t.data_ptr(), t.shape[1], t.shape[2], ld, t.stride(0), _QCUR_DT[t.dtype])


def _qp(t):
    return ctypes.byref(qmat(t)) if t is not None else None


class Handle:
    """A libqcur handle bound to one device, using torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().qcur_create(ctypes.byref(h), device))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().qcur_destroy(self.h)
        except Exception:
            pass

    def bind(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().qcur_set_stream(self.h, ctypes.c_void_p(s)))
        return self.h


_handles = {}


def handle(device=None) -> Handle:
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def _h(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("libqcur operates on GPU tensors")
    return handle(t.device).bind()


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def sync_status(device=None):
    """Synchronises and raises QcurError if a kernel flagged a data error."""
    _check(lib().qcur_sync_status(handle(device).bind()))


def empty(rows: int, cols: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    return torch.empty((4, rows, cols), dtype=dtype, device=device)


# ---- the eight calls -------------------------------------------------------

def probs(A: torch.Tensor, sampling: int = LENGTH):
    """(p_col, q_row, fro2) as float64 device tensors."""
    _, m, n = A.shape
    p = torch.empty(n, dtype=torch.float64, device=A.device)
    q = torch.empty(m, dtype=torch.float64, device=A.device)
    f = torch.empty(1, dtype=torch.float64, device=A.device)
    ws = _ws(lib().qcur_probs_workspace(m, n), A.device)
    _check(lib().qcur_probs(_h(A), _qp(A), sampling, _ptr(p), _ptr(q), _ptr(f), _ptr(ws), ws.numel()))
    return p, q, f


def probs_noalloc(A: torch.Tensor, sampling: int = LENGTH, p=None, q=None, fro2=None):
    """probs() through qcur_probs_noalloc: no workspace; the library's static
    device scratch holds the partial sums.  p, q, fro2 may be given (caller
    buffers, e.g. under graph capture); missing ones are allocated here."""
    _, m, n = A.shape
    dev = A.device
    p = torch.empty(n, dtype=torch.float64, device=dev) if p is None else p
    q = torch.empty(m, dtype=torch.float64, device=dev) if q is None else q
    fro2 = torch.empty(1, dtype=torch.float64, device=dev) if fro2 is None else fro2
    _check(lib().qcur_probs_noalloc(_h(A), _qp(A), sampling, _ptr(p), _ptr(q), _ptr(fro2)))
    return p, q, fro2


def draw(probs_: torch.Tensor, count: int, seed: int, set_id: int, with_replacement: bool = False):
    idx = torch.empty(count, dtype=torch.int64, device=probs_.device)
    _check(lib().qcur_draw(_h(probs_), _ptr(probs_), probs_.numel(), count, seed & (2 ** 64 - 1),
                           set_id & (2 ** 64 - 1), int(with_replacement), _ptr(idx)))
    return idx


def gather(A: torch.Tensor, I: torch.Tensor, J: torch.Tensor, dtype=None, want=("C", "R", "W")):
    _, m, n = A.shape
    r, c = I.numel(), J.numel()
    dt = dtype or A.dtype
    C = empty(m, c, dt, A.device) if "C" in want else None
    R = empty(r, n, dt, A.device) if "R" in want else None
    W = empty(r, c, dt, A.device) if "W" in want else None
    _check(lib().qcur_gather(_h(A), _qp(A), _ptr(I), r, _ptr(J), c, _qp(C), _qp(R), _qp(W)))
    return C, R, W


def pinv(X: torch.Tensor, rtol: float = -1.0, max_rank: int = 0):
    """(X^+, rank) in FP64."""
    _, p, q = X.shape
    Xp = empty(q, p, torch.float64, X.device)
    rank = torch.zeros(1, dtype=torch.int64, device=X.device)
    ws = _ws(lib().qcur_pinv_workspace(p, q), X.device)
    _check(lib().qcur_pinv(_h(X), _qp(X), rtol, max_rank, _qp(Xp), _ptr(rank), _ptr(ws), ws.numel()))
    return Xp, rank


def gemm(A, B, opA=OP_N, opB=OP_N, alpha=1.0, beta=0.0, D=None, compute=None):
    compute = _QCUR_DT[A.dtype] if compute is None else compute
    M = A.shape[1] if opA == OP_N else A.shape[2]
    K = A.shape[2] if opA == OP_N else A.shape[1]
    N = B.shape[2] if opB == OP_N else B.shape[1]
    if D is None:
        D = torch.zeros((4, M, N), dtype=torch.float64 if compute == F64 else torch.float32,
                        device=A.device)
    ws = _ws(lib().qcur_gemm_workspace(M, N, K, compute), A.device)
    _check(lib().qcur_gemm(_h(A), opA, opB, alpha, _qp(A), _qp(B), beta, _qp(D), compute, _ptr(ws),
                           ws.numel()))
    return D


def approx(A=None, C=None, R=None, W=None, core=CORE_CAR, compute=F64, refine_steps=0, rtol=-1.0,
           max_rank=0, want_B=False):
    """Core U (and B = C U R when want_B); returns (U, B, ranks[2])."""
    if core == CORE_WPINV:
        r, c = W.shape[1], W.shape[2]
        dev = W.device
    else:
        c, r = C.shape[2], R.shape[1]
        dev = A.device
    m = C.shape[1] if C is not None else 0
    n = R.shape[2] if R is not None else 0
    odt = torch.float64 if compute == F64 else torch.float32
    U = empty(c, r, odt, dev)
    B = empty(m, n, odt, dev) if want_B else None
    ranks = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = _ws(lib().qcur_approx_workspace(m, n, c, r, core, compute), dev)
    ref = W if core == CORE_WPINV else A
    _check(lib().qcur_approx(_h(ref), _qp(A), _qp(C), _qp(R), _qp(W), core, compute, refine_steps, rtol,
                             max_rank, _qp(U), _qp(B), _ptr(ranks), _ptr(ws), ws.numel()))
    return U, B, ranks


def residual(A, C, U, R, mask=None, compute=F64, want_E=False, e_scale=1.0):
    """(||P_Omega(A - CUR)||_F as a device double[1], optional E)."""
    _, m, n = A.shape
    c, r = C.shape[2], R.shape[1]
    fro = torch.empty(1, dtype=torch.float64, device=A.device)
    E = empty(m, n, torch.float64 if compute == F64 else torch.float32, A.device) if want_E else None
    ws = _ws(lib().qcur_residual_workspace(m, n, c, r, compute), A.device)
    mld = mask.stride(0) if mask is not None else 0
    _check(lib().qcur_residual(_h(A), _qp(A), _qp(C), _qp(U), _qp(R), _ptr(mask), mld, compute,
                               _ptr(fro), _qp(E), e_scale, _ptr(ws), ws.numel()))
    return fro, E


def backward(A, I, J, gB=None, mask=None, rtol=-1.0, max_rank=0, want_dA=True):
    """(dA, loss): dA for the VJP of CUR(A) (gB given) or for the masked loss
    (gB None, which also returns the loss as a device double[1]); with
    want_dA False (masked-loss mode only) dA is None and only the loss is
    computed."""
    compute = _QCUR_DT[A.dtype]
    _, m, n = A.shape
    r, c = I.numel(), J.numel()
    if not want_dA and gB is not None:
        raise ValueError("want_dA=False needs the masked-loss mode (gB None)")
    dA = torch.empty_like(A) if want_dA else None
    loss = torch.zeros(1, dtype=torch.float64, device=A.device)
    ws = _ws(lib().qcur_backward_workspace(m, n, c, r, compute), A.device)
    mld = mask.stride(0) if mask is not None else 0
    _check(lib().qcur_backward(_h(A), _qp(A), _ptr(I), r, _ptr(J), c, _qp(gB), _ptr(mask), mld, rtol,
                               max_rank, compute, _qp(dA), _ptr(loss), _ptr(ws), ws.numel()))
    return dA, loss


def cast(X: torch.Tensor, dtype) -> torch.Tensor:
    Y = torch.empty(X.shape, dtype=dtype, device=X.device)
    _check(lib().qcur_cast(_h(X), _qp(X), _qp(Y)))
    return Y


# ---- the whole path ----------------------------------------------------------

class Solver:
    """Reusable buffers for repeated native solves (qcur_solve) of one shape."""

    def __init__(self, m: int, n: int, c: int, r: int, core: int = CORE_CAR, compute: int = F64, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.shape = (m, n, c, r)
        self.core, self.compute = core, compute
        odt = torch.float64 if compute == F64 else torch.float32
        self.I = torch.empty(r, dtype=torch.int64, device=dev)
        self.J = torch.empty(c, dtype=torch.int64, device=dev)
        self.U = empty(c, r, odt, dev)
        self.residual = torch.empty(1, dtype=torch.float64, device=dev)
        self.ranks = torch.zeros(2, dtype=torch.int64, device=dev)
        self.ws = _ws(lib().qcur_solve_workspace(m, n, c, r, core, compute), dev)

    def __call__(self, A: torch.Tensor, sampling: int = LENGTH, seed: int = 0, refine_steps: int = 0,
                 rtol: float = -1.0, max_rank: int = 0, with_replacement: bool = False, B: torch.Tensor = None):
        """One solve; B (optional, (4, m, n) in U's dtype) receives C U R."""
        m, n, c, r = self.shape
        if tuple(A.shape) != (4, m, n):
            raise ValueError("A does not match the solver's shape")
        _check(lib().qcur_solve(_h(A), _qp(A), c, r, sampling, self.core, self.compute, seed & (2 ** 64 - 1),
                                int(with_replacement), refine_steps, rtol, max_rank, _ptr(self.I), _ptr(self.J),
                                _qp(self.U), _ptr(self.residual), _ptr(self.ranks), None, None, None, None, None,
                                _qp(B), _ptr(self.ws), self.ws.numel()))
        return self


def solve(A: torch.Tensor, c: int, r: int, sampling: int = LENGTH, core: int = CORE_CAR, compute: int = F64,
          seed: int = 0, refine_steps: int = 0, rtol: float = -1.0, max_rank: int = 0,
          with_replacement: bool = False, want_B: bool = False):
    """Algorithm 1 on the GPU: probabilities, draws of J (set 0) and I (set 1),
    gathers, core and residual.  Returns a dict of device tensors."""
    p, q, f2 = probs(A, sampling)
    J = draw(p, c, seed, 0, with_replacement)
    I = draw(q, r, seed, 1, with_replacement)
    C, R, W = gather(A, I, J, dtype=None)
    U, B, ranks = approx(A, C, R, W, core=core, compute=compute, refine_steps=refine_steps, rtol=rtol,
                         max_rank=max_rank, want_B=want_B)
    fro, _ = residual(A, C, U, R, compute=compute)
    return dict(p=p, q=q, fro2=f2, I=I, J=J, C=C, R=R, W=W, U=U, B=B, ranks=ranks, residual=fro)


def _slots(t: torch.Tensor) -> tuple:
    """(QMat of slot 0, slot stride) for a (count, 4, rows, cols) tensor."""
    if t.dim() != 4 or t.shape[1] != 4:
        raise ValueError(f"batched quaternion matrices are (count, 4, rows, cols) tensors, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError("batched operands must be contiguous")
    if t.dtype not in _QCUR_DT:
        raise ValueError(f"unsupported dtype {t.dtype}")
    _, _, rows, cols = t.shape
    return QMat(t.data_ptr(), rows, cols, cols, rows * cols, _QCUR_DT[t.dtype]), t.stride(0)


class BatchSolver:
    """Batched QMCUR (qcur_solve_batched) for a fixed list of problem sizes.

    dims: (count, 4) integers (m_b, n_b, c_b, r_b).  Inputs are (count, 4,
    MX, NX) tensors holding A_b in the top-left corner of slot b (MX, NX at
    least the largest m_b, n_b); see pack_batch.  Outputs after a call:
    I (count, rx), J (count, cx), U (count, 4, cx, rx), residual (count,),
    ranks (count, 2), p (count, nx), q (count, mx), each problem in the
    leading part of its row/slot, and with want_B=True also B (count, 4, mx,
    nx) = C_b U_b R_b.  The call enqueues kernels only, so it may be
    captured in a torch.cuda.CUDAGraph after one eager call.  With
    autotune=True the first eager call times the candidate launch plans of
    every GEMM stage and keeps the fastest (see plans())."""

    def __init__(self, dims, compute: int = F32, sampling: int = LENGTH, refine_steps: int = 0,
                 a_dtype=torch.float32, device=None, autotune: bool = False, want_B: bool = False):
        import numpy as np
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 4))
        self.dims = d
        self.count = int(d.shape[0])
        self.mx, self.nx, self.cx, self.rx = (int(v) for v in d.max(axis=0))
        self.compute, self.sampling, self.refine_steps = compute, sampling, refine_steps
        self.a_dtype = a_dtype
        odt = torch.float64 if compute == F64 else torch.float32
        n = self.count
        self.I = torch.full((n, self.rx), -1, dtype=torch.int64, device=dev)
        self.J = torch.full((n, self.cx), -1, dtype=torch.int64, device=dev)
        self.U = torch.zeros((n, 4, self.cx, self.rx), dtype=odt, device=dev)
        self.residual = torch.zeros(n, dtype=torch.float64, device=dev)
        self.ranks = torch.zeros((n, 2), dtype=torch.int64, device=dev)
        self.p = torch.zeros((n, self.nx), dtype=torch.float64, device=dev)
        self.q = torch.zeros((n, self.mx), dtype=torch.float64, device=dev)
        self.B = torch.zeros((n, 4, self.mx, self.nx), dtype=odt, device=dev) if want_B else None
        dptr = ctypes.c_void_p(d.ctypes.data)
        self.autotune = int(bool(autotune))
        nbytes = lib().qcur_batch_workspace(n, dptr, _QCUR_DT[a_dtype], sampling, compute, refine_steps,
                                            self.autotune)
        if nbytes == 0:
            raise QcurError(1, "invalid batch sizes or options")
        self.ws = _ws(nbytes, dev)
        with torch.cuda.device(dev):
            _check(lib().qcur_batch_prepare(handle(dev).bind(), n, dptr, _QCUR_DT[a_dtype], sampling, compute,
                                            refine_steps, self.autotune, _ptr(self.ws), self.ws.numel()))
        self.device = dev

    STAGES = ("gram_C", "gram_R", "q1_C", "q1_R", "gram2", "p2p1", "q1p2", "AQr", "QcT", "QcM", "MPr", "PcW",
              "residual")

    def plans(self):
        """{stage: (tile, splits)} kept by the autotuner, or None before it ran."""
        n = len(self.STAGES)
        tiles = (ctypes.c_int * n)()
        splits = (ctypes.c_int * n)()
        got = lib().qcur_batch_plans(handle(self.device).h, _ptr(self.ws), tiles, splits, n)
        if got == 0:
            return None
        return {name: (tiles[i], splits[i]) for i, name in enumerate(self.STAGES)}

    def __call__(self, A: torch.Tensor, seed: int = 0, rtol: float = -1.0, max_rank: int = 0,
                 with_replacement: bool = False):
        if A.dtype != self.a_dtype:
            raise ValueError(f"A must be {self.a_dtype} (the dtype the batch was prepared for)")
        if A.shape[0] != self.count:
            raise ValueError("A has the wrong number of slots")
        qa, sa = _slots(A)
        qu, su = _slots(self.U)
        qb, sb = _slots(self.B) if self.B is not None else (None, 0)
        _check(lib().qcur_solve_batched(_h(A), self.count, ctypes.c_void_p(self.dims.ctypes.data), ctypes.byref(qa),
                                        sa, self.sampling, self.compute, seed & (2 ** 64 - 1), int(with_replacement),
                                        self.refine_steps, rtol, max_rank, _ptr(self.I), _ptr(self.J),
                                        ctypes.byref(qu), su, _ptr(self.residual), _ptr(self.ranks), _ptr(self.p),
                                        _ptr(self.q), ctypes.byref(qb) if qb is not None else None, sb,
                                        _ptr(self.ws), self.ws.numel()))
        return self


def pack_batch(mats, dtype=torch.float32, device="cuda", slot=None) -> torch.Tensor:
    """Copies a list of (4, m_b, n_b) arrays into the top-left corners of the
    slots of a zero (count, 4, MX, NX) tensor (MX, NX = the largest sizes, or
    `slot`)."""
    mx = max(int(a.shape[1]) for a in mats) if slot is None else slot[0]
    nx = max(int(a.shape[2]) for a in mats) if slot is None else slot[1]
    out = torch.zeros((len(mats), 4, mx, nx), dtype=dtype)
    for b, a in enumerate(mats):
        t = torch.as_tensor(a)
        out[b, :, : t.shape[1], : t.shape[2]] = t.to(dtype)
    return out.to(device)


def complete(Y: torch.Tensor, mask: torch.Tensor, I: torch.Tensor, J: torch.Tensor, compute: int = F64,
             rtol: float = -1.0, max_rank: int = 0, max_iter: int = 200, tol: float = 1e-4):
    """Completion from the observed entries (Algorithm 2) with the fixed index
    sets I, J.  Returns (X, iterations, last relative change)."""
    _, m, n = Y.shape
    if mask.dtype != torch.uint8 or tuple(mask.shape) != (m, n) or mask.stride(1) != 1:
        raise ValueError("mask must be a row-major uint8 (m, n) tensor")
    r, c = I.numel(), J.numel()
    odt = torch.float64 if compute == F64 else torch.float32
    X = empty(m, n, odt, Y.device)
    ws = _ws(lib().qcur_complete_workspace(m, n, c, r, compute), Y.device)
    iters, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    _check(lib().qcur_complete(_h(Y), _qp(Y), _ptr(mask), mask.stride(0), _ptr(I), r, _ptr(J), c, compute, rtol,
                               max_rank, max_iter, tol, _qp(X), ctypes.byref(iters), ctypes.byref(rel), _ptr(ws),
                               ws.numel()))
    return X, iters.value, rel.value


def complete_resampled(Y: torch.Tensor, mask: torch.Tensor, r: int, c: int, sampling: int = LENGTH, seed: int = 0,
                       compute: int = F64, rtol: float = -1.0, max_rank: int = 0, max_iter: int = 200,
                       tol: float = 1e-4):
    """Completion (Algorithm 2) with I (r rows) and J (c columns) drawn again
    at every step from the probabilities of the iterate (seed + step).
    Returns (X, iterations, last relative change, I, J of the last step)."""
    _, m, n = Y.shape
    if mask.dtype != torch.uint8 or tuple(mask.shape) != (m, n) or mask.stride(1) != 1:
        raise ValueError("mask must be a row-major uint8 (m, n) tensor")
    odt = torch.float64 if compute == F64 else torch.float32
    X = empty(m, n, odt, Y.device)
    I = torch.empty(r, dtype=torch.int64, device=Y.device)
    J = torch.empty(c, dtype=torch.int64, device=Y.device)
    ws = _ws(lib().qcur_complete_resampled_workspace(m, n, c, r, sampling, compute), Y.device)
    iters, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    _check(lib().qcur_complete_resampled(_h(Y), _qp(Y), _ptr(mask), mask.stride(0), r, c, sampling, seed, compute,
                                         rtol, max_rank, max_iter, tol, _qp(X), _ptr(I), _ptr(J),
                                         ctypes.byref(iters), ctypes.byref(rel), _ptr(ws), ws.numel()))
    return X, iters.value, rel.value, I, J


def svd(X: torch.Tensor, vectors: bool = True):
    """Thin QSVD X = U diag(s) V^H (one-sided Jacobi, FP64).  Returns (s, U, V)
    with s descending (k = min(p, q)); U, V are None when vectors is False."""
    _, p, q = X.shape
    k = min(p, q)
    s = torch.empty(k, dtype=torch.float64, device=X.device)
    U = empty(p, k, torch.float64, X.device) if vectors else None
    V = empty(q, k, torch.float64, X.device) if vectors else None
    ws = _ws(lib().qcur_svd_workspace(p, q), X.device)
    _check(lib().qcur_svd(_h(X), _qp(X), _ptr(s), _qp(U) if vectors else None, _qp(V) if vectors else None,
                          _ptr(ws), ws.numel()))
    return s, U, V


def sample_size(k: int, limit: int) -> int:
    """ceil(k ln k) clipped to [k, limit]: the k log k size of C and R."""
    return int(lib().qcur_sample_size(k, limit))
