"""The allocation-free prediction entry point (s3_predict_noalloc) against
s3_predict, through the C ABI: two calls in a row on one plan, the second
with a smaller input, each bitwise equal to the workspace-backed call (same
kernels, same padded core)."""
import ctypes as C

import numpy as np
import pytest
import torch

from tests.gpu_util import setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,dtype", [("cfg1", "f64"), ("cfg2_slice", "f32"), ("cfg5_slice", "f32")])
def test_predict_noalloc_matches_predict(name, dtype):
    cfg, p, plan, ref, order = setup(name, dtype=dtype, batch=4096)
    plan.det_batches(0, 1, 0.05)  # move the parameters off their start
    lib = plan.lib
    idx = torch.as_tensor(np.ascontiguousarray(p.test_idx), dtype=torch.int32, device="cuda").contiguous()
    n1 = idx.shape[1]
    for nnz in (n1, n1 // 3 + 1):
        sub = idx[:, :nnz].contiguous()
        want = plan.predict(sub.cpu().numpy())
        got = torch.full((nnz,), float("nan"), dtype=plan.tdtype, device="cuda")
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.s3_predict_noalloc(plan.h, C.c_void_p(sub.data_ptr()), nnz, C.c_void_p(got.data_ptr()), st)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"{name}: {nnz} entries differ"


def test_predict_noalloc_rejects_out_of_range_index():
    cfg, p, plan, ref, order = setup("tiny3", dtype="f64", batch=8)
    bad = np.ascontiguousarray(p.test_idx).copy()
    bad[0, 0] = cfg.dims[0]
    sub = torch.as_tensor(bad, dtype=torch.int32, device="cuda").contiguous()
    out = torch.empty(sub.shape[1], dtype=torch.float64, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert plan.lib.s3_predict_noalloc(plan.h, C.c_void_p(sub.data_ptr()), sub.shape[1],
                                       C.c_void_p(out.data_ptr()), st) == -2
    # and a good call afterwards still works (the flag is cleared per call)
    good = torch.as_tensor(np.ascontiguousarray(p.test_idx), dtype=torch.int32, device="cuda").contiguous()
    assert plan.lib.s3_predict_noalloc(plan.h, C.c_void_p(good.data_ptr()), good.shape[1],
                                       C.c_void_p(out.data_ptr()), st) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, plan.predict(p.test_idx))
