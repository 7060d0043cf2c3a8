"""GPU: the continuous-batching request loop (results alone == in the mix == oracle, admission by budget)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_0809_0063_amd import inputs
from tests.gpu_util import device, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    device()
    from paper_0809_0063_amd import serve as S
    return S


def _check_against_oracle(pool, item, out):
    pl = pool[item]
    a, b = inputs.payload_operands(pl)
    if pl.kind == "gemm":
        if pl.n <= 160:
            assert (out == O.fgemm(a, b, pl.p)).all()
        g = np.random.default_rng(item)
        rows, cols = g.integers(0, pl.n, 64), g.integers(0, pl.n, 64)
        assert (out[rows, cols] == O.fgemm_entries(a, b, pl.p, rows, cols)).all()
    else:
        assert (out == O.polymul(a, b, pl.p)).all()


def test_serve_mix_equals_alone(serve):
    pool = inputs.serve_pool(n_gemm=24, n_poly=24, gemm_range=(32, 600), seed=321)
    server = serve.Server(pool, hbm_budget=1 << 30, slots=6, chunk_macs=1 << 24)
    n_req = 150
    arr = inputs.poisson_arrivals(n_req, qps=3000.0, seed=1)
    seq = inputs.request_sequence(n_req, len(pool), seed=2)
    done = server.run(arr, seq, max_wall=120.0)
    assert len(done) == n_req
    # overlapping: at some point more than one request was in flight
    spans = sorted((r.admitted, r.done) for r in done)
    overlap = any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert overlap
    alone = {}
    for r in done:
        out = to_host(r.out)
        if r.item not in alone:
            alone[r.item] = to_host(serve.run_alone(server, r.item))
            _check_against_oracle(pool, r.item, alone[r.item])
        assert (out == alone[r.item]).all(), (r.rid, r.item)
    stats = serve.Server.summary(done, 0, pool)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    assert server.cache.hits > 0   # repeated payloads stay resident


def test_serve_admission_waits_when_over_budget(serve):
    """With a tiny budget a request waits for memory instead of failing; all complete, results exact."""
    pool = inputs.serve_pool(n_gemm=6, n_poly=6, gemm_range=(200, 400), seed=9)
    server = serve.Server(pool, hbm_budget=3 << 20, slots=4, chunk_macs=1 << 22, cache_fraction=0.3)
    arr = inputs.poisson_arrivals(30, qps=1e5, seed=3)
    seq = inputs.request_sequence(30, len(pool), seed=4)
    done = server.run(arr, seq, max_wall=60.0)
    assert len(done) == 30
    peak_concurrent = 0
    ev = sorted([(r.admitted, 1) for r in done] + [(r.done, -1) for r in done])
    cur = 0
    for _, d in ev:
        cur += d
        peak_concurrent = max(peak_concurrent, cur)
    assert peak_concurrent <= 4
    for r in done:
        _check_against_oracle(pool, r.item, to_host(r.out))
