"""Host-side logic without a GPU: the tuner's models, plans and bucketing."""
import json
import os

import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_tab_mulpol_examples():
    """The two worked examples after Table tab:mulpol reproduce under the stated reading."""
    from paper_0809_0063_amd import tune as T
    rows = GOLDEN["tab_mulpol_examples"]["rows"]
    r0 = rows[0]
    dma, dred, fma, fred = T.fqt_model(r0["N"], r0["p"], r0["d"], r0["beta"])
    assert abs(dma - r0["delayed_muladd"]) / r0["delayed_muladd"] < 0.01
    assert abs(dred - r0["delayed_reductions"]) / r0["delayed_reductions"] < 0.01
    assert abs(fma - r0["fqt_muladd"]) / r0["fqt_muladd"] < 0.01
    assert abs(fred - r0["fqt_reductions"]) / r0["fqt_reductions"] < 0.02
    assert round(dma / fma) == r0["ratio"] or int(dma / fma) == r0["ratio"]
    r1 = rows[1]
    _, _, fma1, fred1 = T.fqt_model(r1["N"], r1["p"], r1["d"], r1["beta"])
    assert abs(fma1 - r1["fqt_muladd"]) / r1["fqt_muladd"] < 0.02
    assert abs(fred1 - r1["fqt_reductions"]) / r1["fqt_reductions"] < 0.02


def test_cmm_interval_bounds():
    from paper_0809_0063_amd import tune as T
    # eq:lower with a Kronecker pair in a 16-bit lane: (p-1)(Q+1) < 2^16, L (p-1)^2 < Q
    assert T.cmm_interval_max(3, 1024) == 4092
    assert T.cmm_interval_max(7, 1024) == 224
    assert T.cmm_interval_max(2, 1024) == 32764
    assert T.cmm_interval_max(251, 1024) == 0
    for p in (2, 3, 5, 7, 11, 13):
        L = T.cmm_interval_max(p, 10 ** 6)
        bmax = max(b for b in range(1, 17) if (p - 1) * ((1 << b) + 1) < 65536)
        assert L * (p - 1) ** 2 < 2 ** bmax and (L + 4) * (p - 1) ** 2 >= 2 ** bmax - 4 * (p - 1) ** 2


def test_model_prefers_most_macs_per_instruction():
    """The seed model orders the candidates by multiply-adds per instruction: eight (dot8, p <= 16),
    then four (packed CMM or dot4); no CMM where (p-1)^2 leaves no delayed interval, no dot8 above 16."""
    from paper_0809_0063_amd import dqt as D
    from paper_0809_0063_amd import tune as T
    cands = T.candidates(3, 512)
    best = min(cands, key=lambda c: T.model_cost(3, 512, c))
    assert best.algo == D.GEMM_DOT8
    c17 = T.candidates(17, 512)
    assert all(c.algo != D.GEMM_DOT8 for c in c17)
    assert min(c17, key=lambda c: T.model_cost(17, 512, c)).algo in (D.GEMM_CMM, D.GEMM_DOT4)
    assert all(c.algo not in (D.GEMM_CMM, D.GEMM_DOT8) for c in T.candidates(251, 512))


def test_buckets():
    from paper_0809_0063_amd import tune as T
    assert T.bucket_of(16) == 0 and T.bucket_of(31) == 0 and T.bucket_of(32) == 1
    assert T.bucket_of(1024) == len(T.BUCKET_EDGES) - 2
    for b in range(len(T.BUCKET_EDGES) - 1):
        n = T.representative(b)
        assert T.BUCKET_EDGES[b] <= n < T.BUCKET_EDGES[b + 1]
