"""GPU: the autotuner picks valid plans per bucket; tuned batches stay bit-exact."""
import json
import os

import pytest
import torch

import oracle as O
from paper_0809_0063_amd import inputs
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_tuner_buckets_and_tuned_batch(tmp_path):
    device()
    from paper_0809_0063_amd import dqt as D
    from paper_0809_0063_amd import tune as T
    cache = os.path.join(str(tmp_path), "tune.json")
    tu = T.Tuner(cache)
    table = tu.tune(primes=(3, 7), buckets=(0, 3, 5), reps=3)
    assert set(table) == {"3:0", "3:3", "3:5", "7:0", "7:3", "7:5"}
    for key, plan in table.items():
        assert plan.us > 0
        assert plan.algo in (D.GEMM_CMM, D.GEMM_PLAIN, D.GEMM_DOT4, D.GEMM_DOT8)
    tu.save()
    again = T.Tuner(cache)
    assert again.table == tu.table
    assert json.load(open(cache))
    # a batch built from the tuned plans is exact
    items = inputs.batch_items(40, nmin=16, nmax=600, primes=(3, 7), seed=17)
    ops, host = [], []
    for it in items:
        A, B = inputs.item_operands(it)
        d = {"A": to_dev(A), "B": to_dev(B), "C": torch.empty((it.n, it.n), dtype=torch.uint8, device=device()),
             "p": it.p}
        d.update(tu.desc_fields(it.p, it.n))
        ops.append(d)
        host.append((A, B))
    descs = D.make_descs(ops)
    need = max(D.fgemm_batched_workspace_size(descs, *shape) for shape in T.LAUNCH_SHAPES)
    ws = torch.empty(need, dtype=torch.uint8, device=device())
    launch = tu.tune_launch(descs, ws)
    assert launch in T.LAUNCH_SHAPES
    D.fgemm_batched(descs, ws, *launch)
    for d, (A, B), it in zip(ops, host, items):
        assert (to_host(d["C"]) == O.fgemm(A, B, it.p)).all(), it
