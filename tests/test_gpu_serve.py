"""GPU: the continuous-batching request loop (results alone == in the mix == oracle, admission by budget)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_0809_0063_amd import inputs
from tests.gpu_util import device, digest, load_digests, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    device()
    from paper_0809_0063_amd import serve as S
    return S


def _pool_digests():
    rows = load_digests("serve_pool_digests.txt")
    pool = inputs.serve_pool()
    assert len(rows) == len(pool)
    for r, pl in zip(rows, pool):   # the golden file describes exactly this pool
        assert (r[1], int(r[2]), int(r[3]), int(r[4]), int(r[5])) == (pl.kind, pl.n, pl.deg, pl.p, pl.seed)
    return pool, [r[6] for r in rows]


def test_serve_full_pool_every_result_is_the_oracles(serve):
    """The serving workload's whole pool (600 F_p products of order 32..2048, 600 batches of polynomial
    products of degree 2..15 and batch 1..4096, p in {2,3,5,7,11}) served as a Poisson stream in which
    every payload appears at least once and some repeat (residency-cache hits): every served result
    equals the oracle's (stored digests), requests overlapped, device memory stayed within the budget
    plus the outputs already delivered, and results computed alone equal those from the mix."""
    pool, want = _pool_digests()
    budget = 16 << 30
    server = serve.Server(pool, hbm_budget=budget, slots=8)
    g = np.random.default_rng(5)
    seq = np.concatenate([g.permutation(len(pool)), g.integers(0, len(pool), size=300)])
    arr = inputs.poisson_arrivals(len(seq), qps=4000.0, seed=17)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    peak = {"over": 0}

    def on_step(active, finished):
        delivered = sum(r.out.numel() for r in finished)
        peak["over"] = max(peak["over"], torch.cuda.memory_allocated() - base - delivered - budget)

    done = server.run(arr, seq, max_wall=600.0, on_step=on_step)
    assert len(done) == len(seq)
    assert peak["over"] <= 0, peak
    spans = sorted((r.admitted, r.done) for r in done)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))   # work overlapped
    bad = [(r.rid, r.item) for r in done if digest(to_host(r.out)) != want[r.item]]
    assert not bad, f"{len(bad)} results differ from the oracle, first {bad[:5]}"
    assert server.cache.hits > 0
    # alone == in the mix, on a sample that includes the largest products
    by_item = {}
    for r in done:
        by_item.setdefault(r.item, r)
    gemms = sorted((i for i, pl in enumerate(pool) if pl.kind == "gemm"), key=lambda i: -pool[i].n)
    sample = gemms[:4] + list(g.choice(len(pool), size=24, replace=False))
    for i in sample:
        alone = to_host(serve.run_alone(server, int(i)))
        assert (alone == to_host(by_item[int(i)].out)).all(), i


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
        pl = pool[r.item]
        a, b = inputs.payload_operands(pl)
        want = O.fgemm(a, b, pl.p) if pl.kind == "gemm" else O.polymul(a, b, pl.p)
        assert (to_host(r.out) == want).all(), r.item
        # only the output outlives a finished request
        assert r.A is None and r.B is None and r.CA is None and r.CB is None
