"""Error paths of the C ABI that need a device (bind-time validation)."""
import numpy as np
import pytest

from synth import get_config, init_params, item_order, make_problem

pytestmark = pytest.mark.gpu


def test_bind_rejects_out_of_range_index():
    from paper_1708_08640_amd import S3Error, S3Plan
    cfg = get_config("cfg1")
    p = make_problem(cfg)
    p.train_idx = p.train_idx.copy()
    p.train_idx[2, 17] = cfg.dims[2]  # one past the end of mode 3
    with pytest.raises(S3Error) as ei:
        S3Plan.from_problem(p, init_params(cfg), dtype="f64", batch=100, order=item_order(p.n_items, 1))
    assert ei.value.status == -2


def test_bind_rejects_bad_order():
    from paper_1708_08640_amd import S3Error, S3Plan
    cfg = get_config("cfg1")
    p = make_problem(cfg)
    order = item_order(p.n_items, 1).copy()
    order[3] = p.n_items + 5
    with pytest.raises(S3Error) as ei:
        S3Plan.from_problem(p, init_params(cfg), dtype="f64", batch=100, order=order)
    assert ei.value.status == -2


def test_loss_reports_divergence():
    from paper_1708_08640_amd import S3Error, S3Plan
    cfg = get_config("cfg1")
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    plan = S3Plan.from_problem(p, (U, G, V), dtype="f64", batch=4096, order=item_order(p.n_items, 1), eta0=1e4)
    plan.epoch(0, "det")
    plan.epoch(1, "det")
    with pytest.raises(S3Error) as ei:
        plan.loss()
    assert ei.value.status == -4
