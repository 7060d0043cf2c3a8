"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random data only; it holds none of the packed-DQT / REDQ
arithmetic and imports neither the HIP library nor the CPU oracle.  The same
bytes are handed to both sides.

Generator: numpy ``Generator(PCG64(seed))``.  Workload seeds are
``SEED_BASE + i`` for workload i = 1..5 (small polymul, 1024^3 F_p product,
GF(p^k) products, batched products, serving stream).

The paper measures on unspecified random data (no public dataset), so every
input is uniform over [0, p) with the shapes below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

SEED_BASE = 8090063
SEED_POLYMUL = SEED_BASE + 1
SEED_FGEMM = SEED_BASE + 2
SEED_GF = SEED_BASE + 3
SEED_BATCH = SEED_BASE + 4
SEED_SERVE = SEED_BASE + 5


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_residues(shape, p: int, seed: int) -> np.ndarray:
    """uint8 array of the given shape, iid uniform over [0, p)."""
    return rng(seed).integers(0, p, size=shape, dtype=np.uint8)


def polymul_pairs(count: int, k: int, p: int, seed: int = SEED_POLYMUL, kb: int | None = None):
    """(a, b): uint8 [count, k] and [count, kb] coefficient arrays (degree < k), uniform in [0, p)."""
    g = rng(seed)
    a = g.integers(0, p, size=(count, k), dtype=np.uint8)
    b = g.integers(0, p, size=(count, kb if kb is not None else k), dtype=np.uint8)
    return a, b


def gemm_pair(m: int, n: int, kdim: int, p: int, seed: int = SEED_FGEMM):
    """(A, B): uint8 [m, kdim] and [kdim, n], row-major, uniform in [0, p)."""
    g = rng(seed)
    A = g.integers(0, p, size=(m, kdim), dtype=np.uint8)
    B = g.integers(0, p, size=(kdim, n), dtype=np.uint8)
    return A, B


def _has_factor(poly: Sequence[int], p: int, deg: int) -> bool:
    """True if some monic polynomial of degree `deg` divides `poly` (trial division)."""
    k = len(poly) - 1
    for idx in range(p ** deg):
        div = [(idx // p ** i) % p for i in range(deg)] + [1]
        rem = [c % p for c in poly]
        for j in range(k, deg - 1, -1):
            c = rem[j]
            if c:
                for i in range(deg + 1):
                    rem[j - deg + i] = (rem[j - deg + i] - c * div[i]) % p
        if not any(rem[:deg]):
            return True
    return False


def irreducible(p: int, k: int, seed: int = SEED_GF) -> List[int]:
    """A seeded monic irreducible polynomial of degree k over F_p (k+1 coefficients, low first).

    Rejection sampling: draw c_0..c_{k-1} uniform in [0, p), append the
    leading 1, reject when c_0 == 0 or when a monic factor of degree
    1..floor(k/2) divides it.  Field set-up, not part of the packed path.
    """
    g = rng(seed * 1000 + p * 16 + k)
    while True:
        c = [int(x) for x in g.integers(0, p, size=k)] + [1]
        if c[0] == 0:
            continue
        if any(_has_factor(c, p, dg) for dg in range(1, k // 2 + 1)):
            continue
        return c


def gf_pairs(count: int, k: int, p: int, seed: int = SEED_GF):
    """(a, b): uint8 [count, k] uniform field elements (any degree < k polynomial is reduced)."""
    g = rng(seed + 7919 * p + k)
    a = g.integers(0, p, size=(count, k), dtype=np.uint8)
    b = g.integers(0, p, size=(count, k), dtype=np.uint8)
    return a, b


def worst_case(shape, p: int) -> np.ndarray:
    """All entries p-1: the largest digits the a priori bounds must absorb."""
    return np.full(shape, p - 1, dtype=np.uint8)


# --- batched products -----------------------------------------------------------

BATCH_PRIMES = (2, 3, 5, 7)


@dataclass
class GemmItem:
    n: int
    p: int
    seed: int


def batch_items(count: int = 10000, nmin: int = 16, nmax: int = 1024, primes=BATCH_PRIMES,
                seed: int = SEED_BATCH) -> List[GemmItem]:
    """Square F_p products with n = round(exp(U[ln nmin, ln nmax])) and p uniform in `primes`."""
    g = rng(seed)
    ln = g.uniform(math.log(nmin), math.log(nmax), size=count)
    ns = np.clip(np.rint(np.exp(ln)).astype(np.int64), nmin, nmax)
    ps = g.choice(np.asarray(primes), size=count)
    seeds = g.integers(0, 2 ** 31 - 1, size=count)
    return [GemmItem(int(n), int(p), int(s)) for n, p, s in zip(ns, ps, seeds)]


def item_operands(item: GemmItem):
    """(A, B) of one square product item."""
    return gemm_pair(item.n, item.n, item.n, item.p, seed=item.seed)


# --- serving stream -----------------------------------------------------------

SERVE_PRIMES = (2, 3, 5, 7, 11)


@dataclass
class Payload:
    kind: str          # "gemm" or "polymul"
    p: int
    n: int             # gemm: matrix order; polymul: batch size
    deg: int           # polymul: degree (k = deg + 1 coefficients); 0 for gemm
    seed: int


def serve_pool(n_gemm: int = 600, n_poly: int = 600, gemm_range=(32, 2048), deg_range=(2, 15),
               batch_range=(1, 4096), primes=SERVE_PRIMES, seed: int = SEED_SERVE) -> List[Payload]:
    """Pool of request payloads: GEMM order uniform in gemm_range, polymul degree and batch uniform."""
    g = rng(seed)
    pool = []
    for _ in range(n_gemm):
        pool.append(Payload("gemm", int(g.choice(primes)), int(g.integers(gemm_range[0], gemm_range[1] + 1)), 0,
                            int(g.integers(0, 2 ** 31 - 1))))
    for _ in range(n_poly):
        pool.append(Payload("polymul", int(g.choice(primes)), int(g.integers(batch_range[0], batch_range[1] + 1)),
                            int(g.integers(deg_range[0], deg_range[1] + 1)), int(g.integers(0, 2 ** 31 - 1))))
    return pool


def payload_operands(pl: Payload):
    if pl.kind == "gemm":
        return gemm_pair(pl.n, pl.n, pl.n, pl.p, seed=pl.seed)
    return polymul_pairs(pl.n, pl.deg + 1, pl.p, seed=pl.seed)


def poisson_arrivals(count: int, qps: float, seed: int = SEED_SERVE + 1000) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    g = rng(seed)
    return np.cumsum(g.exponential(1.0 / qps, size=count))


def request_sequence(count: int, pool_size: int, seed: int = SEED_SERVE + 2000) -> np.ndarray:
    """Pool indices referenced by successive requests (uniform, with repeats)."""
    return rng(seed).integers(0, pool_size, size=count)
