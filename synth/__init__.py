"""Seeded synthetic inputs for the sparse coupled Tucker SGD path.

This package draws data only: COO index sets, values, splits, initial
parameters and item orders. It holds none of the factorisation's arithmetic
(no prediction, gradient or loss), so that the FP64 oracle and the HIP path can
both be fed from it without sharing any of the method's code.
"""
from .gen import (  # noqa: F401
    Config,
    MatrixSpec,
    Problem,
    CONFIGS,
    get_config,
    make_problem,
    init_params,
    item_order,
    zipf_ranks,
)
