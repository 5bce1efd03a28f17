"""MI355X (gfx950) library for sparse coupled matrix-tensor factorisation with a
Tucker model trained by per-entry SGD (S^3CMTF, arXiv 1708.08640).

The computation lives in the HIP shared library ``libs3cmtf.so`` (C ABI in
``include/s3cmtf.h``); this package only marshals arguments to it and uses
torch for device memory and streams.
"""
from ._abi import S3Error, load, EXPORTS  # noqa: F401
from .plan import S3Plan  # noqa: F401
from .autograd import SparseTuckerCMTF, predictions  # noqa: F401
