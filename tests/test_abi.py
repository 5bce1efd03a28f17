"""Host-only checks of the C ABI: the library loads, exports every function
include/s3cmtf.h declares, and rejects bad descriptors and out-of-order
calls without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1708_08640_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1708_08640_amd.build import build
        build()
    return _abi, _abi.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "s3cmtf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(s3_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    _abi, lib = _lib()
    assert _declared() == sorted(_abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    _abi, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


def _desc(_abi, **kw):
    d = _abi.S3Desc()
    d.order, d.n_mat = 3, 1
    for n in range(3):
        d.dims[n], d.rank[n] = 100, 10
    d.mat_mode[0], d.mat_cols[0] = 0, 50
    d.dtype, d.eta0, d.mu, d.lambda_reg, d.lambda_m = 1, 0.01, 0.1, 0.01, 10.0
    d.batch, d.round_items = 64, 64
    for k, v in kw.items():
        if k in ("dims", "rank", "mat_mode", "mat_cols"):
            for n, x in enumerate(v):
                getattr(d, k)[n] = x
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    (dict(order=2), -3),
    (dict(order=5), -3),
    (dict(dtype=7), -3),
    (dict(dtype=2), -3),  # bf16 operands exist only in the matrix-core contraction
    (dict(dtype=2, contraction=2), -3),  # which is not built for padded rank 10
    (dict(dtype=0, contraction=2, rank=(16, 16, 16)), -3),  # nor for FP64
    (dict(rank=(10, 10, 40)), -3),
    (dict(batch=0), -1),
    (dict(eta0=-1.0), -1),
    (dict(n_mat=9), -1),
    (dict(mat_mode=(3, 0, 0, 0)), -1),
    (dict(contraction=3), -1),
    (dict(contraction=2), -3),  # matrix cores: padded rank 16 (3-way) or 8 (4-way) only
    (dict(core_kind=1, contraction=2, rank=(16, 16, 16)), -3),
    (dict(contraction=1, rank=(8, 8, 8)), -3),  # no naive kernels for J = 8
    (dict(core_kind=2), -1),
    (dict(core_kind=1, rank=(10, 10, 8)), -1),  # CP needs equal ranks
    (dict(core_kind=1, contraction=1), -3),
])
def test_plan_create_rejects(kw, status):
    _abi, lib = _lib()
    d = _desc(_abi)
    if "mat_mode" in kw:
        d.mat_mode[0] = kw.pop("mat_mode")[0]
    d = _desc(_abi, **kw) if kw else d
    if "mat_mode" not in kw and d.mat_mode[0] == 3:
        pass
    h = C.c_void_p()
    assert lib.s3_plan_create(C.byref(d), C.byref(h)) == status
    assert not h.value


def test_calls_before_bind_are_state_errors():
    _abi, lib = _lib()
    d = _desc(_abi)
    h = C.c_void_p()
    assert lib.s3_plan_create(C.byref(d), C.byref(h)) == 0
    out = (C.c_double * 3)()
    assert lib.s3_epoch(h, 0, 0, None) == -7
    assert lib.s3_loss(h, out, None) == -7
    assert lib.s3_rmse(h, out, None) == -7
    assert lib.s3_det_batches(h, 0, 1, 0.01, None) == -7
    fake = (C.c_void_p * 4)(8, 8, 8, 8)  # never dereferenced: the state check comes first
    assert lib.s3_backward(h, C.c_void_p(8), None, fake, C.c_void_p(8), fake, None) == -7
    buf = C.create_string_buffer(256)
    assert lib.s3_last_error(h, buf, 256) == 0 and b"bind" in buf.value
    y = (C.c_int64 * 1)(100)
    sz = C.c_size_t()
    assert lib.s3_workspace_size(h, 1000, 100, y, C.byref(sz)) == 0 and sz.value > 0
    again = C.c_size_t()
    assert lib.s3_workspace_size(h, 1000, 100, y, C.byref(again)) == 0 and again.value == sz.value
    assert lib.s3_workspace_size(h, 0, 100, y, C.byref(sz)) == -1
    assert lib.s3_plan_destroy(h) == 0


def test_status_strings():
    _abi, lib = _lib()
    for st in range(-7, 1):
        assert lib.s3_status_string(st)


def test_bind_rejects_small_workspace():
    # the size check comes before any device access, so placeholder device
    # addresses never get dereferenced
    _abi, lib = _lib()
    d = _desc(_abi)
    h = C.c_void_p()
    assert lib.s3_plan_create(C.byref(d), C.byref(h)) == 0
    try:
        b = _abi.S3Buffers()
        fake = 0x10000
        b.x_idx, b.x_val, b.x_nnz = fake, fake, 1000
        for n in range(3):
            b.U[n] = fake
        b.G, b.V[0] = fake, fake
        b.y_row[0], b.y_col[0], b.y_val[0], b.y_nnz[0] = fake, fake, fake, 100
        need = C.c_size_t()
        y = (C.c_int64 * 1)(100)
        assert lib.s3_workspace_size(h, 1000, 0, y, C.byref(need)) == 0
        # (without an item order the bind needs less than this upper bound,
        # so probe well below it)
        assert lib.s3_bind(h, C.byref(b), C.c_void_p(fake), 4096, None) == -6
        assert lib.s3_bind(h, C.byref(b), None, need.value, None) == -6
        buf = C.create_string_buffer(256)
        lib.s3_last_error(h, buf, 256)
        assert b"workspace" in buf.value
    finally:
        lib.s3_plan_destroy(h)


def test_det_offsets_beyond_32_bits_are_rejected():
    """The det build packs per-batch scratch offsets and (batch, type) sort
    keys into 32 bits; sizes that overflow them are refused up front."""
    _abi, lib = _lib()
    y = (C.c_int64 * 3)(0, 0, 0)
    sz = C.c_size_t()
    buf = C.create_string_buffer(256)
    cases = [
        # batch x (3 x 16 + 5) scratch elements: 50M fits, 100M does not
        (dict(rank=(16, 16, 16), batch=50_000_000), 50_000_000, 0),
        (dict(rank=(16, 16, 16), batch=100_000_000), 100_000_000, -3),
        # 2^31 - 1 single-item batches x (3 matrices + 1) keys
        (dict(batch=1, n_mat=3, mat_mode=(0, 1, 2), mat_cols=(50, 50, 50)), 2**31 - 1, -3),
        (dict(batch=2, n_mat=3, mat_mode=(0, 1, 2), mat_cols=(50, 50, 50)), 2**31 - 1, 0),
    ]
    for kw, x_nnz, status in cases:
        d = _desc(_abi, **kw)
        h = C.c_void_p()
        assert lib.s3_plan_create(C.byref(d), C.byref(h)) == 0
        try:
            assert lib.s3_workspace_size(h, x_nnz, 0, y, C.byref(sz)) == status, kw
            if status:
                lib.s3_last_error(h, buf, 256)
                assert b"32 bits" in buf.value
                # bind with an item order refuses the same sizes before touching memory
                b = _abi.S3Buffers()
                fake = 0x10000
                b.x_idx, b.x_val, b.x_nnz = fake, fake, x_nnz
                for n in range(3):
                    b.U[n] = fake
                b.G = fake
                for m in range(d.n_mat):
                    b.V[m] = fake
                b.order = fake
                assert lib.s3_bind(h, C.byref(b), C.c_void_p(fake), 1 << 40, None) == -3
        finally:
            lib.s3_plan_destroy(h)


def test_import_before_bind_is_a_state_error():
    _abi, lib = _lib()
    plan = C.c_void_p()
    assert lib.s3_plan_create(C.byref(_desc(_abi)), C.byref(plan)) == _abi.S3_OK
    try:
        buf = (C.c_double * 4)()
        assert lib.s3_import(plan, 1, 0, buf, C.sizeof(buf), None) == _abi.S3_ERR_STATE
        assert lib.s3_import(plan, 1, 0, None, 0, None) == _abi.S3_ERR_INVALID_ARG
    finally:
        lib.s3_plan_destroy(plan)
