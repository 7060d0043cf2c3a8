"""Writes the oracle digests of the batched and serving workloads.

Test infrastructure.  Every expected value written here comes from the CPU
oracle (``oracle/``) applied to the seeded inputs of
``paper_0809_0063_amd.inputs`` (a module that draws random numbers and holds
none of the method's arithmetic); nothing here loads or calls the HIP library.

* ``batch_10000_digests.txt``: the 10,000 square F_p products of the batched
  workload (``inputs.batch_items(10000)``: n log-uniform in [16, 1024], p in
  {2, 3, 5, 7}).  One line per product: index, n, p, seed, digest of the
  uint8 row-major C = A.B mod p.
* ``serve_pool_digests.txt``: the 1,200 payloads of the serving pool
  (``inputs.serve_pool()``: 600 F_p products of order 32..2048 and 600
  batches of polynomial products of degree 2..15, batch 1..4096, p in
  {2, 3, 5, 7, 11}).  One line per payload: index, kind, n, deg, p, seed,
  digest of the uint8 result (C, or the [batch][2 deg + 1] products).

The digest is the first 32 hex digits (128 bits) of SHA-256 over the result
bytes in C order.  The whole run takes about 40 minutes of 8 host cores.

Usage: ``python tests/golden/make_digests.py [--batch] [--serve]`` (both when
neither is given).
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_0809_0063_amd import inputs  # noqa: E402

BATCH_FILE = os.path.join(HERE, "batch_10000_digests.txt")
SERVE_FILE = os.path.join(HERE, "serve_pool_digests.txt")
DIGEST_HEX = 32


def digest(x: np.ndarray) -> str:
    """Digest of an array's bytes in C order (128-bit prefix of SHA-256)."""
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()[:DIGEST_HEX]


def write_batch(path: str = BATCH_FILE) -> None:
    items = inputs.batch_items(10000)
    t0 = time.time()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("# oracle digests of the batched workload: inputs.batch_items(10000), seed %d\n" % inputs.SEED_BATCH)
        f.write("# index n p seed sha256[:32] of C = A.B mod p (uint8, row-major)\n")
        for i, it in enumerate(items):
            A, B = inputs.item_operands(it)
            f.write("%d %d %d %d %s\n" % (i, it.n, it.p, it.seed, digest(O.fgemm(A, B, it.p))))
            if i % 500 == 499:
                f.flush()
                print("batch %d/%d  %.0f s" % (i + 1, len(items), time.time() - t0), flush=True)
    os.replace(tmp, path)


def write_serve(path: str = SERVE_FILE) -> None:
    pool = inputs.serve_pool()
    t0 = time.time()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("# oracle digests of the serving pool: inputs.serve_pool(), seed %d\n" % inputs.SEED_SERVE)
        f.write("# index kind n deg p seed sha256[:32] of the result (gemm: C uint8 [n][n]; "
                "polymul: uint8 [n][2 deg + 1])\n")
        for i, pl in enumerate(pool):
            a, b = inputs.payload_operands(pl)
            out = O.fgemm(a, b, pl.p) if pl.kind == "gemm" else O.polymul(a, b, pl.p)
            f.write("%d %s %d %d %d %d %s\n" % (i, pl.kind, pl.n, pl.deg, pl.p, pl.seed, digest(out)))
            if i % 50 == 49:
                f.flush()
                print("serve %d/%d  %.0f s" % (i + 1, len(pool), time.time() - t0), flush=True)
    os.replace(tmp, path)


def load(path: str):
    """Rows of a digest file as lists of strings (comment lines skipped)."""
    with open(path) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--serve", action="store_true")
    args = ap.parse_args(argv)
    both = not (args.batch or args.serve)
    if args.batch or both:
        write_batch()
    if args.serve or both:
        write_serve()


if __name__ == "__main__":
    main()
