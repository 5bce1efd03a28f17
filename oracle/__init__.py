"""FP64 CPU oracle for sparse coupled Tucker SGD (S^3CMTF, arXiv 1708.08640).

TEST INFRASTRUCTURE ONLY: the reference that the HIP library is checked
against. Only the tests, the smoke check and the benchmark's CPU-baseline leg
use it; the library never does. The arithmetic lives in plain C
(``s3_oracle.c``, double precision, sequential loops that follow the paper's
definitions); this module only marshals numpy arrays into it.

Every function here cites the part of the paper it follows:

* ``predict``             -- Tucker model, Eq (4)
* ``tensor_item_grad``    -- per-entry gradients, Eq (8) / Algorithm 2
* ``tensor_item_grad_opt``-- reuse form, Definitions 4-5, Lemmas 2-3, Algorithm 3
* ``matrix_item_grad``    -- coupled-matrix entry, Eq (8) / Algorithm 1
* ``sgd_epoch``           -- Algorithm 1 with one worker
* ``minibatch_epoch``     -- the library's deterministic batched reading of it
                             (optionally evaluated by several threads, summed
                             in the same order: bitwise the same result)
* ``loss``                -- Eq (7), per-entry form
* ``rmse``                -- held-out RMSE, Section 4.1
* ``full_grad``           -- sum of per-entry gradients (= gradient of Eq 7)
* ``adjoint``             -- transpose of the prediction map (Eq 4 and u.v)
* ``qr_orthogonalize``    -- Algorithm 1's closing QR step

Every function is pinned by tests/test_oracle.py; none is parity unpinned.
"""
from .api import (  # noqa: F401
    Params,
    build,
    lib_path,
    counts,
    predict,
    matrix_predict,
    tensor_item_grad,
    tensor_item_grad_opt,
    tensor_item_w,
    matrix_item_grad,
    sgd_epoch,
    minibatch_epoch,
    loss,
    rmse,
    full_grad,
    adjoint,
    qr_orthogonalize,
    eta_at,
)
