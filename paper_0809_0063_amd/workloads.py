"""The batched and serving workloads as measured by the benchmark.

* batched: 10,000 square F_p products, n log-uniform in [16, 1024], p in
  {2,3,5,7}; all of them in one packing launch plus one persistent launch,
  captured in a graph; the time of a replay and the F_p op rate.
* serving: a Poisson stream over a pool of payloads (F_p products of order
  32..2048 and polynomial-product batches of degree 2..15, batch 1..4096,
  p in {2,3,5,7,11}); p50/p99 latency and throughput at 0.5, 0.8 and 1.2 of
  the loop's measured saturation rate (all of a sample of requests arriving at
  once).
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Optional

import numpy as np
import torch

from . import dqt as D
from . import inputs
from . import serve as S

PEAK_LANE_OPS = 256 * 64 * 2.4e9


def _graph_of(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return g


def _replay_seconds(g, replays: int) -> float:
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / replays


def batched(n_items: int = 10000, replays: int = 3, tuner=None, seed: int = inputs.SEED_BATCH,
            algo: Optional[int] = None, verify: Optional[Callable] = None, launch=None) -> Dict[str, float]:
    """The whole batch as one graph, replayed: once with packing (one packing launch + one persistent
    launch) and once on the resident packed operands (the persistent launch only, the packed copies
    left by the previous replay; section 7.1's reuse of compressed matrices).  `algo` forces one
    algorithm for every product (otherwise the tuner's per-bucket plan, or the library default).
    `verify(items, outputs)`, if given, receives the items and their output tensors after the
    resident replays, whose outputs were cleared beforehand.  `launch` (rows, k-split, columns)
    overrides the tuner's launch shape."""
    dev = torch.device("cuda:0")
    items = inputs.batch_items(n_items, seed=seed)
    t0 = time.perf_counter()
    ops, macs, dot_ops = [], 0.0, 0.0
    for it in items:
        A, B = inputs.item_operands(it)
        d = {"A": torch.from_numpy(A).to(dev), "B": torch.from_numpy(B).to(dev),
             "C": torch.empty((it.n, it.n), dtype=torch.uint8, device=dev), "p": it.p}
        if algo is not None:
            d["algo"] = algo
        elif tuner is not None:
            d.update(tuner.desc_fields(it.p, it.n))
        ops.append(d)
        macs += float(it.n) ** 3
        dot_ops += float(it.n) * it.n * ((it.n + 3) // 4)
    gen_s = time.perf_counter() - t0
    algo_count: Dict[int, int] = {}
    for d in ops:
        a = d.get("algo", 0)
        algo_count[a] = algo_count.get(a, 0) + 1
    descs = D.make_descs(ops)
    if launch is None:
        launch = tuner.launch if (tuner is not None and tuner.launch) else (16, 2, 4)
    ws = torch.empty(D.fgemm_batched_workspace_size(descs, *launch), dtype=torch.uint8, device=dev)
    batch = D.Batch(descs, ws, *launch)
    batch.run()
    torch.cuda.synchronize()
    sec = _replay_seconds(_graph_of(batch.run), replays)
    # a cheap spot check of the packed replays' output
    C0 = ops[0]["C"].cpu().numpy()
    A0, B0 = inputs.item_operands(items[0])
    assert (C0[:1] == (A0[:1].astype(np.int64) @ B0.astype(np.int64)) % items[0].p).all()
    g_res = _graph_of(batch.compute)
    for d in ops:
        d["C"].fill_(255)
    torch.cuda.synchronize()
    sec_res = _replay_seconds(g_res, replays)
    if verify is not None:
        verify(items, [d["C"] for d in ops])
    batch.close()
    return {"products": n_items, "ms_per_replay": round(sec * 1e3, 3), "fp_gop_s": round(2 * macs / sec / 1e9, 1),
            "packed_lane_op_frac": round(dot_ops / sec / PEAK_LANE_OPS, 4),
            "ms_per_replay_resident": round(sec_res * 1e3, 3),
            "fp_gop_s_resident": round(2 * macs / sec_res / 1e9, 1),
            "packed_lane_op_frac_resident": round(dot_ops / sec_res / PEAK_LANE_OPS, 4),
            "launch": list(launch),
            "tuned_buckets": len(tuner.table) if (tuner is not None and algo is None) else 0,
            "algos": {str(k): v for k, v in sorted(algo_count.items())},
            "input_gen_s": round(gen_s, 1)}


def batched_buckets(n_items: int = 10000, tuner=None, reps: int = 3, seed: int = inputs.SEED_BATCH,
                    launch=(16, 2, 4)) -> Dict[str, Dict]:
    """The batch split by order bucket: for each bucket, the persistent launch on resident packed
    operands timed with every algorithm (and the tuner's choice), with each algorithm's VALU
    lane-instruction fraction (n^2 ceil(n/e) instructions per product, e entries per word)."""
    from . import tune as T
    dev = torch.device("cuda:0")
    items = inputs.batch_items(n_items, seed=seed)
    per_word = {D.GEMM_CMM: 4, D.GEMM_DOT4: 4, D.GEMM_DOT8: 8, D.GEMM_PLAIN: 1}
    names = {D.GEMM_CMM: "cmm", D.GEMM_DOT4: "dot4", D.GEMM_DOT8: "dot8", D.GEMM_PLAIN: "plain"}
    out = {}
    for bk in range(len(T.BUCKET_EDGES) - 1):
        sub = [it for it in items if T.bucket_of(it.n) == bk]
        if not sub:
            continue
        ops = []
        for it in sub:
            A, B = inputs.item_operands(it)
            ops.append({"A": torch.from_numpy(A).to(dev), "B": torch.from_numpy(B).to(dev),
                        "C": torch.empty((it.n, it.n), dtype=torch.uint8, device=dev), "p": it.p})
        row = {"n_range": [T.BUCKET_EDGES[bk], T.BUCKET_EDGES[bk + 1] - 1], "products": len(sub)}
        plans = ([("tuned", None)] if tuner is not None else []) + [(names[a], a) for a in per_word]
        for name, a in plans:
            for d, it in zip(ops, sub):
                for k in ("algo", "interval", "log2Q", "epilogue"):
                    d.pop(k, None)
                if a is None:
                    d.update(tuner.desc_fields(it.p, it.n))
                else:
                    d["algo"] = a
            descs = D.make_descs(ops)
            ws = torch.empty(D.fgemm_batched_workspace_size(descs, *launch), dtype=torch.uint8, device=dev)
            b = D.Batch(descs, ws, *launch)
            b.run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                b.compute()
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / 1e3 / reps
            b.close()
            ent = {"ms": round(sec * 1e3, 3)}
            if a is not None:
                instr = sum(float(it.n) * it.n * ((it.n + per_word[a] - 1) // per_word[a]) for it in sub)
                ent["lane_op_frac"] = round(instr / sec / PEAK_LANE_OPS, 4)
            else:
                cnt: Dict[str, int] = {}
                for d in ops:
                    cnt[names.get(d["algo"], str(d["algo"]))] = cnt.get(names.get(d["algo"], str(d["algo"])), 0) + 1
                ent["algos"] = cnt
            row[name] = ent
            del ws
        out[f"bucket{bk}"] = row
        del ops
        torch.cuda.empty_cache()
    return out


def serving(n_requests: int = 5000, warmup: int = 500, loads=(0.5, 0.8, 1.2), n_gemm: int = 600,
            n_poly: int = 600, hbm_budget: int = 16 << 30, seed: int = inputs.SEED_SERVE) -> Dict[str, object]:
    """The serving loop at fixed fractions of its measured saturation throughput.

    Saturation is measured first (a sample of requests all arriving at once); then, for each
    load factor, a Poisson stream of warmup + n_requests requests at that fraction of the
    saturation rate, of which the last n_requests are measured (p50/p99 latency from arrival
    to result, throughput, residency-cache hit rate).  Above 1.0 the queue grows and admission
    back-pressure shows in the latency."""
    pool = inputs.serve_pool(n_gemm=n_gemm, n_poly=n_poly, seed=seed)
    server = S.Server(pool, hbm_budget=hbm_budget, slots=8)
    n_sat = max(200, n_requests // 5)
    seq = inputs.request_sequence(n_sat, len(pool), seed=seed + 3)
    done = server.run(np.zeros(n_sat), seq, max_wall=120.0)
    span = max(r.done for r in done) if done else 1.0
    sat = len(done) / span
    out: Dict[str, object] = {"saturation_req_per_s": round(sat, 1), "requests": n_requests, "warmup": warmup}
    for i, f in enumerate(loads):
        qps = f * sat
        arr = inputs.poisson_arrivals(n_requests + warmup, qps, seed=seed + 1 + 10 * i)
        seq = inputs.request_sequence(n_requests + warmup, len(pool), seed=seed + 2 + 10 * i)
        h0, m0 = server.cache.hits, server.cache.misses
        done = server.run(arr, seq, max_wall=240.0)
        st = S.Server.summary(done, warmup, pool)
        st["qps_offered"] = qps
        st["completed"] = len(done)
        hits, misses = server.cache.hits - h0, server.cache.misses - m0
        st["cache_hit_rate"] = hits / max(1, hits + misses)
        out[f"load_{f:g}"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    return out


def main(argv=None):
    """Run the batched and/or serving workload alone and print the results (one JSON line each)."""
    import argparse
    import json

    from . import tune as T
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--batched", action="store_true")
    ap.add_argument("--serving", action="store_true")
    ap.add_argument("--replays", type=int, default=3)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--packed", action="store_true", help="batched: the packed middle product on every product")
    ap.add_argument("--buckets", action="store_true", help="batched: every algorithm on each order bucket")
    args = ap.parse_args(argv)
    if args.batched:
        if args.packed:
            print(json.dumps({"batched_10000_packed_cmm": batched(10000, replays=args.replays, tuner=T.Tuner(),
                                                                 algo=D.GEMM_CMM)}), flush=True)
        else:
            print(json.dumps({"batched_10000_tuned": batched(10000, replays=args.replays, tuner=T.Tuner())}),
                  flush=True)
    if args.buckets:
        print(json.dumps({"batched_10000_by_bucket": batched_buckets(10000, tuner=T.Tuner())}), flush=True)
    if args.serving:
        print(json.dumps({"serving": serving(n_requests=args.requests, warmup=args.requests // 10)}), flush=True)


if __name__ == "__main__":
    main()
