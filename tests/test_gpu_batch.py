"""GPU parity: batched F_p products in one persistent launch (bit-exact vs the oracle), graph replays."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_0809_0063_amd import inputs
from tests.gpu_util import device, digest, load_digests, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dqt():
    device()
    from paper_0809_0063_amd import dqt as D
    return D


def _make(D, items, algo_of=lambda i, it: 0):
    ops, host = [], []
    for i, it in enumerate(items):
        A, B = inputs.item_operands(it)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.full((it.n, it.n), 255, dtype=torch.uint8, device=device())
        ops.append({"A": dA, "B": dB, "C": dC, "p": it.p, "algo": algo_of(i, it)})
        host.append((A, B))
    return ops, host


@pytest.mark.parametrize("tile_rows,ksplit,tile_cols", [(16, 4, 2), (8, 2, 2), (16, 2, 2), (8, 4, 2), (8, 4, 4),
                                                        (8, 2, 4), (16, 2, 4), (16, 4, 4), (8, 8, 4),
                                                        (8, 8, 2), (16, 8, 2)])
def test_batch_small_mixed(dqt, tile_rows, ksplit, tile_cols):
    items = inputs.batch_items(60, nmin=1, nmax=300, seed=99)
    algos = [dqt.GEMM_AUTO, dqt.GEMM_CMM, dqt.GEMM_PLAIN, dqt.GEMM_DOT4, dqt.GEMM_DOT8]
    ops, host = _make(dqt, items, lambda i, it: algos[i % 5])
    descs = dqt.make_descs(ops)
    ws = torch.empty(dqt.fgemm_batched_workspace_size(descs, tile_rows, ksplit, tile_cols), dtype=torch.uint8,
                     device=device())
    dqt.fgemm_batched(descs, ws, tile_rows, ksplit, tile_cols)
    for op, (A, B), it in zip(ops, host, items):
        assert (to_host(op["C"]) == O.fgemm(A, B, it.p)).all(), (it, op["algo"])


def test_batch_epilogues_and_intervals(dqt):
    items = inputs.batch_items(40, nmin=16, nmax=400, seed=5)
    ops, host = _make(dqt, items, lambda i, it: dqt.GEMM_CMM)
    for i, op in enumerate(ops):
        op["epilogue"] = i % 2
        op["interval"] = [0, 4, 16, 64][i % 4]
    descs = dqt.make_descs(ops)
    ws = torch.empty(dqt.fgemm_batched_workspace_size(descs), dtype=torch.uint8, device=device())
    dqt.fgemm_batched(descs, ws)
    for op, (A, B), it in zip(ops, host, items):
        assert (to_host(op["C"]) == O.fgemm(A, B, it.p)).all(), it


def test_batch_graph_replays(dqt):
    """The prepared batch captured in a graph: every replay equals the eager result."""
    items = inputs.batch_items(30, nmin=16, nmax=256, seed=7)
    ops, host = _make(dqt, items)
    descs = dqt.make_descs(ops)
    ws = torch.empty(dqt.fgemm_batched_workspace_size(descs), dtype=torch.uint8, device=device())
    batch = dqt.Batch(descs, ws)
    batch.run()
    torch.cuda.synchronize()
    eager = [to_host(op["C"]).copy() for op in ops]
    for op, (A, B), it, e in zip(ops, host, items, eager):
        assert (e == O.fgemm(A, B, it.p)).all()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            batch.run()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        for op in ops:
            op["C"].fill_(255)            # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for op, e in zip(ops, eager):
            assert (to_host(op["C"]) == e).all(), rep
    batch.close()


def _batch_digests():
    rows = load_digests("batch_10000_digests.txt")
    items = inputs.batch_items(10000)
    assert len(rows) == len(items)
    for r, it in zip(rows, items):   # the golden file describes exactly these items
        assert (int(r[1]), int(r[2]), int(r[3])) == (it.n, it.p, it.seed)
    return items, [r[4] for r in rows]


def _check_all(items, outs, want):
    bad = []
    for i, (it, C) in enumerate(zip(items, outs)):
        if digest(to_host(C)) != want[i]:
            bad.append((i, it.n, it.p))
    assert not bad, f"{len(bad)} of {len(items)} products differ from the oracle, first {bad[:5]}"


def test_batch_workload_10000_default_plans(dqt):
    """The batched workload (10,000 products, n log-uniform in [16, 1024], p in {2,3,5,7}) with the
    library's default plan for every product: every output equals the oracle's (stored digests)."""
    items, want = _batch_digests()
    ops = []
    for it in items:
        A, B = inputs.item_operands(it)
        ops.append({"A": to_dev(A), "B": to_dev(B), "C": torch.full((it.n, it.n), 255, dtype=torch.uint8,
                                                                    device=device()), "p": it.p})
    descs = dqt.make_descs(ops)
    ws = torch.empty(dqt.fgemm_batched_workspace_size(descs), dtype=torch.uint8, device=device())
    dqt.fgemm_batched(descs, ws)
    torch.cuda.synchronize()
    _check_all(items, [op["C"] for op in ops], want)


def test_batch_workload_10000_as_benchmarked(dqt):
    """The same 10,000 products exactly as the benchmark runs them: the tuner's per-bucket plans and
    launch shape, one packing launch and one persistent launch captured in a graph and replayed;
    every output of the replays equals the oracle's (stored digests)."""
    from paper_0809_0063_amd import tune as T
    from paper_0809_0063_amd import workloads as W
    items, want = _batch_digests()
    seen = {}

    def verify(its, outs):
        assert [(a.n, a.p, a.seed) for a in its] == [(b.n, b.p, b.seed) for b in items]
        _check_all(its, outs, want)
        seen["n"] = len(outs)

    res = W.batched(10000, replays=2, tuner=T.Tuner(), verify=verify)
    assert seen.get("n") == 10000
    assert res["products"] == 10000


def test_batch_workload_10000_packed_forced(dqt):
    """The same batch with the packed middle product forced on every product (as benchmarked)."""
    from paper_0809_0063_amd import tune as T
    from paper_0809_0063_amd import workloads as W
    items, want = _batch_digests()
    seen = {}

    def verify(its, outs):
        _check_all(its, outs, want)
        seen["n"] = len(outs)

    W.batched(10000, replays=1, tuner=T.Tuner(), algo=dqt.GEMM_CMM, verify=verify)
    assert seen.get("n") == 10000
