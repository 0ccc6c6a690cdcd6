"""libqcur: quaternion CUR (QMCUR) low-rank approximation on AMD MI355X.

The compute path is the HIP library libqcur.so (built in-tree by
`python -m paper_2402_19147_amd.build`); this package is its ctypes binding
plus a torch.autograd.Function for the masked CUR loss.  Importing the
package does not load the library; the first call does, and fails loudly
if it has not been built.
"""
from . import qcur  # noqa: F401
from . import autograd  # noqa: F401
from . import perturbation  # noqa: F401
from .autograd import cur_loss, cur  # noqa: F401
from .qcur import (F64, F32, BF16, BF16X3, OP_N, OP_H, LENGTH, UNIFORM, CORE_WPINV, CORE_CAR,  # noqa: F401
                   QcurError, probs, draw, gather, pinv, gemm, approx, residual, backward, cast,
                   solve, sync_status, lib, Solver, BatchSolver, pack_batch, complete,
                   complete_resampled, sample_size, svd)

__all__ = ["qcur", "autograd", "perturbation", "cur_loss", "cur", "probs", "draw", "gather", "pinv", "gemm", "approx", "residual", "backward", "cast",
           "solve", "sync_status", "lib", "QcurError", "Solver",
           "BatchSolver", "pack_batch", "complete", "complete_resampled", "sample_size", "svd"]
