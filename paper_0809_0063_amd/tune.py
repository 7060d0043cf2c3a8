"""Autotuner for the batched F_p products: per (size, p) bucket plan choice.

For each bucket (a range of orders n and a prime p) the tuner times the
candidate plans on one representative square product and keeps the fastest:

* algo: packed CMM (four entries per word, middle product on 16-bit Kronecker
  pairs), plain (one entry per word), dot4 (four u8 entries per word), dot8
  (eight 4-bit entries per word, p <= 16);
* the delayed-reduction interval of the packed path (the largest allowed by
  eq:lower, or a fraction of it) and the matching Q;
* the epilogue (one REDC per output, or REDQ over gathered dot products).

The launch shape of the persistent kernel (rows per wave, waves splitting k,
columns per lane) is one per batch; `tune_launch` times the candidates on the batch itself.
Results are cached as JSON keyed by the device architecture and the library
version.  Every candidate produces the same bytes (the parity tests cover all
of them), so tuning only changes speed.

Cost model seed: the paper's section 5.3 counts multiply-adds and reductions;
here the counts are one instruction per four multiply-adds (packed), one per
multiply-add (plain), plus one reduction per output, and the measured times
replace the model once the tuner has run.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from . import dqt as D

BUCKET_EDGES = (16, 32, 64, 128, 256, 512, 1025)
# persistent-launch shapes (rows per wave, waves splitting k, columns per lane)
LAUNCH_SHAPES = ((16, 4, 2), (8, 2, 2), (16, 2, 2), (8, 4, 2), (8, 4, 4), (8, 2, 4), (16, 2, 4), (16, 4, 4),
                 (8, 8, 4), (8, 8, 2), (16, 8, 2))
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


@dataclass(frozen=True)
class BucketPlan:
    algo: int
    interval: int = 0
    log2Q: int = 0
    epilogue: int = 0
    us: float = 0.0

    def desc_fields(self) -> Dict[str, int]:
        return {"algo": self.algo, "interval": self.interval, "log2Q": self.log2Q, "epilogue": self.epilogue}


def bucket_of(n: int) -> int:
    for i in range(len(BUCKET_EDGES) - 1):
        if n < BUCKET_EDGES[i + 1]:
            return i
    return len(BUCKET_EDGES) - 2


def representative(bucket: int) -> int:
    lo, hi = BUCKET_EDGES[bucket], BUCKET_EDGES[bucket + 1] - 1
    return int(round(math.sqrt(lo * hi)))


def cmm_interval_max(p: int, kdim: int) -> int:
    """Largest delayed-reduction interval of the packed path: L (p-1)^2 < Q with (p-1)(Q+1) < 2^16."""
    e2 = (p - 1) ** 2
    bmax = max(b for b in range(1, 17) if (p - 1) * ((1 << b) + 1) < 65536)
    lmax = ((1 << bmax) - 1) // e2 if e2 else kdim
    return (lmax // 4) * 4


def model_cost(p: int, n: int, plan: BucketPlan) -> float:
    """Instruction-count model (seed ordering before measurement)."""
    macs = float(n) ** 3
    if plan.algo == D.GEMM_CMM:
        return macs / 4 + n * n * (3 if plan.epilogue == 0 else 5)
    if plan.algo == D.GEMM_DOT4:
        return macs / 4 + 3 * n * n
    if plan.algo == D.GEMM_DOT8:
        return macs / 8 + 3 * n * n
    return macs + 3 * n * n


def fqt_model(N: int, p: int, d: int, beta: int) -> Tuple[float, float, float, float]:
    """Table tab:mulpol (section 5.3) for a degree-N product: (delayed mul&add, delayed REDC,
    FQT mul&add, FQT REDQ) with n_d, n_q as printed after the table.

    Reading: q = 2^(beta/(2d+1)) with a real exponent, and the FQT mul&add count
    includes the ceil((2d+2)/2) multiply-adds of each REDQ_{2d+1}; with these the
    paper's two worked examples reproduce.
    """
    Dq = -(-(N + 1) // (d + 1)) - 1
    nd = (2 ** (beta + 1)) // ((p - 1) ** 2)
    q = 2.0 ** (beta / (2 * d + 1))
    nq = int(q // ((d + 1) * (p - 1) ** 2))
    delayed_ma = float(2 * N + 1) ** 2
    delayed_red = float(2 * N + 1) * -(-(2 * N + 1) // nd)
    fqt_red = float(2 * Dq + 1) * -(-(2 * Dq + 1) // nq)
    fqt_ma = float(2 * Dq + 1) ** 2 + fqt_red * -(-(2 * d + 2) // 2)
    return delayed_ma, delayed_red, fqt_ma, fqt_red


def candidates(p: int, n: int) -> List[BucketPlan]:
    out = [BucketPlan(D.GEMM_PLAIN), BucketPlan(D.GEMM_DOT4)]
    if p <= 16:
        out.append(BucketPlan(D.GEMM_DOT8))
    lmax = cmm_interval_max(p, n)
    if lmax >= 4:
        ivals = sorted({min(lmax, ((n + 3) // 4) * 4), max(4, (lmax // 2) // 4 * 4)})
        for iv in ivals:
            for epi in (D.EPI_REDC, D.EPI_REDQ):
                out.append(BucketPlan(D.GEMM_CMM, interval=iv if iv < n else 0, epilogue=epi))
    return out


def _time_plan(p: int, n: int, plan: BucketPlan, reps: int = 20, launch=(16, 4)) -> float:
    """Microseconds per product of a batch of identical-size products run with this plan.

    The products of a bucket are run the way the batched workload runs them
    (one packing launch + one persistent launch over all of them), enough of
    them that the launches are not the measurement.
    """
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(1234 + n * 7 + p)
    A = torch.randint(0, p, (n, n), dtype=torch.uint8, generator=g).to(dev)
    B = torch.randint(0, p, (n, n), dtype=torch.uint8, generator=g).to(dev)
    count = int(min(2048, max(16, (1 << 33) // (n ** 3))))
    Cs = torch.empty((count, n, n), dtype=torch.uint8, device=dev)
    fields = plan.desc_fields()
    descs = D.make_descs([dict(A=A, B=B, C=Cs[i], p=p, **fields) for i in range(count)])
    ws = torch.empty(D.fgemm_batched_workspace_size(descs, *launch), dtype=torch.uint8, device=dev)
    batch = D.Batch(descs, ws, *launch)
    for _ in range(2):
        batch.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.run()
    e1.record()
    torch.cuda.synchronize()
    batch.close()
    return e0.elapsed_time(e1) * 1e3 / reps / count


def time_table_windows(p: int, k: int, count: int = 1 << 22, reps: int = 5) -> Dict[int, float]:
    """Microseconds per call of the fused one-word polynomial product for each REDQ
    correction-table window (1 = none, 2, 3; section 3.5's time-memory trade-off)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(4321 + p * 10 + k)
    a = torch.randint(0, p, (count, k), dtype=torch.uint8, generator=g).to(dev)
    b = torch.randint(0, p, (count, k), dtype=torch.uint8, generator=g).to(dev)
    out = torch.empty((count, 2 * k - 1), dtype=torch.uint8, device=dev)
    res = {}
    try:
        for j in (1, 2, 3):
            D.set_table_window(j)
            for _ in range(2):
                D.polymul_u8(a, b, p, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                D.polymul_u8(a, b, p, out=out)
            e1.record()
            torch.cuda.synchronize()
            res[j] = e0.elapsed_time(e1) * 1e3 / reps
    finally:
        D.set_table_window(0)
    return res


class Tuner:
    def __init__(self, cache_path: Optional[str] = DEFAULT_CACHE):
        self.cache_path = cache_path
        self.key = self._key()
        self.table: Dict[str, BucketPlan] = {}
        self.launch: Optional[Tuple[int, int]] = None
        self._load()

    @staticmethod
    def _key() -> str:
        arch = "cpu"
        if torch.cuda.is_available():
            arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        try:
            ver = D.version()
        except Exception:
            ver = "unbuilt"
        return f"{arch}|{ver}|rocm{torch.version.hip}"

    def _load(self):
        if self.cache_path and os.path.exists(self.cache_path):
            try:
                data = json.load(open(self.cache_path))
            except (OSError, ValueError):
                return
            ent = data.get(self.key)
            if ent:
                self.table = {k: BucketPlan(**v) for k, v in ent.get("buckets", {}).items()}
                if ent.get("launch"):
                    self.launch = tuple(ent["launch"])

    def save(self):
        if not self.cache_path:
            return
        data = {}
        if os.path.exists(self.cache_path):
            try:
                data = json.load(open(self.cache_path))
            except (OSError, ValueError):
                data = {}
        data[self.key] = {"buckets": {k: asdict(v) for k, v in self.table.items()},
                          "launch": list(self.launch) if self.launch else None,
                          "saved": time.strftime("%Y-%m-%d %H:%M:%S")}
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def plan(self, p: int, n: int) -> BucketPlan:
        """Tuned plan of the bucket of n (model order if the bucket was not measured)."""
        k = f"{p}:{bucket_of(n)}"
        if k in self.table:
            return self.table[k]
        cands = candidates(p, n)
        return min(cands, key=lambda c: model_cost(p, n, c))

    def tune_bucket(self, p: int, bucket: int, reps: int = 5) -> BucketPlan:
        n = representative(bucket)
        best = None
        for c in candidates(p, n):
            us = _time_plan(p, n, c, reps)
            c = BucketPlan(c.algo, c.interval, c.log2Q, c.epilogue, round(us, 3))
            if best is None or c.us < best.us:
                best = c
        # the interval was tuned at the representative order; the largest allowed
        # interval for the bucket is kept when the whole range fits one interval
        self.table[f"{p}:{bucket}"] = best
        return best

    def tune(self, primes: Sequence[int], buckets: Optional[Sequence[int]] = None, reps: int = 5,
             progress: Optional[Callable[[str], None]] = None):
        for p in primes:
            for b in (buckets if buckets is not None else range(len(BUCKET_EDGES) - 1)):
                best = self.tune_bucket(p, b, reps)
                if progress is not None:
                    progress(f"{p}:{b} {best}")
        return self.table

    def tune_launch(self, descs, ws: torch.Tensor, shapes=LAUNCH_SHAPES, reps: int = 3):
        """Pick (rows per wave, k-split, columns per lane) for a batch by timing its persistent launch."""
        best = None
        for shape in shapes:
            tm, ks, tn = (tuple(shape) + (2,))[:3]
            need = D.fgemm_batched_workspace_size(descs, tm, ks, tn)
            if need == 0 or need > ws.numel():
                continue
            b = D.Batch(descs, ws, tm, ks, tn)
            b.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                b.run()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            b.close()
            if best is None or dt < best[0]:
                best = (dt, tm, ks, tn)
        if best:
            self.launch = (best[1], best[2], best[3])
        return self.launch

    def desc_fields(self, p: int, n: int) -> Dict[str, int]:
        return self.plan(p, n).desc_fields()


def main(argv=None):
    """Tune every (bucket, p) of the batched workload and its launch shape; write the cache."""
    import argparse

    from . import inputs
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--primes", type=int, nargs="+", default=list(inputs.BATCH_PRIMES))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--launch-items", type=int, default=2000,
                    help="products of the batched workload used to time the launch shapes")
    args = ap.parse_args(argv)
    t = Tuner(args.out)
    t0 = time.time()
    t.tune(args.primes, reps=args.reps, progress=lambda m: print(m, flush=True))
    # launch shape on a prefix of the batched workload with the tuned plans
    dev = torch.device("cuda:0")
    items = inputs.batch_items(10000)[: args.launch_items]
    ops = []
    for it in items:
        A, B = inputs.item_operands(it)
        d = {"A": torch.from_numpy(A).to(dev), "B": torch.from_numpy(B).to(dev),
             "C": torch.empty((it.n, it.n), dtype=torch.uint8, device=dev), "p": it.p}
        d.update(t.desc_fields(it.p, it.n))
        ops.append(d)
    descs = D.make_descs(ops)
    need = max(D.fgemm_batched_workspace_size(descs, *shape) for shape in LAUNCH_SHAPES)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    print("launch", t.tune_launch(descs, ws), flush=True)
    t.save()
    print(f"tuned in {time.time() - t0:.1f} s -> {args.out}", flush=True)


if __name__ == "__main__":
    main()
