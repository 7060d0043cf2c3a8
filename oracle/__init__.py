"""Plain CPU oracle for the packed-DQT / REDQ hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_0809_0063_amd``) and never imports it; the two
meet only through the seeded input generator, which holds none of the method's
arithmetic.

Two kinds of functions live here:

* Plain definitions (bulk, in ``oracle.c``, wrapped below): polynomial product
  over F_p, F_p matrix product, GF(p^k) multiplication by product + long
  division, radix conversion + mod p, Euclidean quotient.  The packed path
  must reach exactly these results.
* Step-by-step models of the paper's algorithms where a plain definition does
  not expose what the paper prints (REDQ's intermediate ``s`` and ``u_i``,
  FDIV/AFDIV under each rounding mode, the table decomposition of the REDQ
  correction, the two-table reduction of FGDP), written in Python with exact
  integers and rationals so that they can be checked against the paper's worked
  examples and tables by eye.

Parity pins for every function are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc (plain -O2, OpenMP) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.orc_polymul.argtypes = [P, I32, P, I32, I64, I32, P, I32]
        lib.orc_fgemm.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, I32, I32]
        lib.orc_fgemm_entries.argtypes = [P, I64, P, I64, I64, I32, P, P, I64, P, I32]
        lib.orc_gf_mul.argtypes = [P, P, I64, I32, I32, P, P, I32]
        lib.orc_radix_mod.argtypes = [P, I64, I32, I32, I32, P, I32]
        lib.orc_floor_div.argtypes = [P, I64, U64, P]
        lib.orc_dqt_eval.argtypes = [P, I64, I32, I32, I32, P]
        lib.orc_max_threads.restype = I32
        for f in ("orc_polymul", "orc_fgemm", "orc_fgemm_entries", "orc_gf_mul", "orc_radix_mod",
                  "orc_floor_div", "orc_dqt_eval"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def max_threads() -> int:
    return int(_load().orc_max_threads())


# ----------------------------------------------------------------------------
# Plain definitions (bulk, C)
# ----------------------------------------------------------------------------

def polymul(a: np.ndarray, b: np.ndarray, p: int, threads: int = 0) -> np.ndarray:
    """Products of polynomials over F_p (eq:mult, section 2.1).

    a: uint8 [N, ka], b: uint8 [N, kb] (coefficient i is that of X^i).
    Returns uint8 [N, ka+kb-1], every coefficient in [0, p).
    """
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    assert a.ndim == 2 and b.ndim == 2 and a.shape[0] == b.shape[0]
    n, ka = a.shape
    kb = b.shape[1]
    out = np.empty((n, ka + kb - 1), dtype=np.uint8)
    _load().orc_polymul(_ptr(a), ka, _ptr(b), kb, n, p, _ptr(out), threads)
    return out


def fgemm(A: np.ndarray, B: np.ndarray, p: int, threads: int = 0) -> np.ndarray:
    """C = A.B mod p over F_p (section 7.1), reducing after every operation."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n), dtype=np.uint8)
    _load().orc_fgemm(_ptr(A), k, _ptr(B), n, _ptr(C), n, m, n, k, p, threads)
    return C


def fgemm_entries(A: np.ndarray, B: np.ndarray, p: int, rows, cols, threads: int = 0) -> np.ndarray:
    """Entries C[rows[s], cols[s]] of A.B mod p, each computed on its own."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    m, k = A.shape
    n = B.shape[1]
    assert rows.shape == cols.shape
    assert rows.size == 0 or (rows.min() >= 0 and rows.max() < m and cols.min() >= 0 and cols.max() < n)
    out = np.empty(rows.shape, dtype=np.uint8)
    _load().orc_fgemm_entries(_ptr(A), k, _ptr(B), n, k, p, _ptr(rows), _ptr(cols), rows.size, _ptr(out), threads)
    return out


def gf_mul(a: np.ndarray, b: np.ndarray, p: int, modulus: Sequence[int], threads: int = 0) -> np.ndarray:
    """Products in GF(p^k) = F_p[X]/(modulus) (section 6): product then long division.

    modulus: k+1 coefficients, low degree first, monic (modulus[k] == 1).
    """
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    mod = np.ascontiguousarray(np.asarray(modulus, dtype=np.uint8))
    n, k = a.shape
    assert b.shape == (n, k) and mod.size == k + 1 and mod[k] == 1 and k <= 16
    out = np.empty((n, k), dtype=np.uint8)
    _load().orc_gf_mul(_ptr(a), _ptr(b), n, k, p, _ptr(mod), _ptr(out), threads)
    return out


def gf_dot(a: np.ndarray, b: np.ndarray, p: int, modulus: Sequence[int], threads: int = 0) -> np.ndarray:
    """Dot products over GF(p^k) (algorithm FGDP's result): out[t] = sum_l a[t,l] b[t,l] in the field.

    a, b: uint8 [N, n, k].  Every product is the plain field product (gf_mul);
    the sum is coefficient-wise mod p, reduced after every addition.
    """
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    N, n, k = a.shape
    prods = gf_mul(a.reshape(N * n, k), b.reshape(N * n, k), p, modulus, threads).reshape(N, n, k)
    out = np.zeros((N, k), dtype=np.int64)
    for l in range(n):
        out = (out + prods[:, l, :]) % p
    return out.astype(np.uint8)


def gf_matmul(a: np.ndarray, b: np.ndarray, p: int, modulus: Sequence[int], threads: int = 0) -> np.ndarray:
    """Matrix products over GF(p^k) (section 6: algorithm FGDP's dot products arranged as a matrix
    product): out[i, j] = sum_l a[i, l] b[l, j] in the field.

    a: uint8 [m, kd, k], b: uint8 [kd, n, k] -> uint8 [m, n, k]; each entry is the dot product
    (gf_dot) of row i of a and column j of b.
    """
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    m, kd, k = a.shape
    kd2, n, k2 = b.shape
    assert kd2 == kd and k2 == k
    if m == 0 or n == 0:
        return np.zeros((m, n, k), dtype=np.uint8)
    rows = np.broadcast_to(a[:, None, :, :], (m, n, kd, k)).reshape(m * n, kd, k)
    cols = np.broadcast_to(b.transpose(1, 0, 2)[None, :, :, :], (m, n, kd, k)).reshape(m * n, kd, k)
    return gf_dot(rows, cols, p, modulus, threads).reshape(m, n, k)


def radix_mod(r: np.ndarray, p: int, logq: int, nres: int, threads: int = 0) -> np.ndarray:
    """REDQ's specification (alg:REDQ ENSURE): digits of r in base q = 2^logq, each mod p.

    The lower nres-1 digits are in [0, q); the top digit is everything above.
    """
    r = np.ascontiguousarray(r, dtype=np.uint64)
    out = np.empty((r.size, nres), dtype=np.uint8)
    _load().orc_radix_mod(_ptr(r), r.size, p, logq, nres, _ptr(out), threads)
    return out


def floor_div(r: np.ndarray, p: int) -> np.ndarray:
    """Euclidean quotient floor(r/p) (the value FDIV approximates, section 4.2)."""
    r = np.ascontiguousarray(r, dtype=np.uint64)
    out = np.empty_like(r)
    _load().orc_floor_div(_ptr(r), r.size, p, _ptr(out))
    return out


def dqt_eval(c: np.ndarray, logq: int, reverse: bool = False) -> np.ndarray:
    """Evaluation at q = 2^logq (eq:dqt) by Horner's rule, as uint64 words."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    n, k = c.shape
    out = np.empty(n, dtype=np.uint64)
    _load().orc_dqt_eval(_ptr(c), n, k, logq, 1 if reverse else 0, _ptr(out))
    return out


# ----------------------------------------------------------------------------
# Small exact models (pure Python integers / rationals)
# ----------------------------------------------------------------------------

def dqt_int(coeffs: Sequence[int], q: int) -> int:
    """Evaluation at an arbitrary integer q (eq:dqt), Horner from the top."""
    v = 0
    for c in reversed(list(coeffs)):
        v = v * q + int(c)
    return v


def radix_digits(r: int, q: int, ndig: int) -> List[int]:
    """Radix conversion of r in base q into ndig digits (top digit unbounded)."""
    out = []
    for _ in range(ndig - 1):
        out.append(r % q)
        r //= q
    out.append(r)
    return out


def redq_steps(r: int, p: int, q: int, nres: int) -> Tuple[int, List[int], List[int]]:
    """Algorithm REDQ (section 3.2) step by step, on exact integers.

    Compression: s = floor(r/p); u_i = floor(r/q^i) - p*floor(s/q^i).
    Correction (only when p does not divide q): mu_d = u_d and
    mu_i = (u_i - q*u_{i+1}) mod p, least non-negative residue.
    Returns (s, [u_0..u_d], [mu_0..mu_d]) with d = nres - 1.
    """
    d = nres - 1
    s = r // p
    u = [r // q ** i - p * (s // q ** i) for i in range(d + 1)]
    if q % p == 0:
        mu = list(u)
    else:
        mu = [0] * (d + 1)
        mu[d] = u[d]
        for i in range(d):
            mu[i] = (u[i] - q * u[i + 1]) % p
    return s, u, mu


def q_matrix(k: int, q: int, p: int) -> List[List[int]]:
    """Matrix Q_k of the REDQ correction (section 3.4): unit upper bidiagonal, -q mod p above."""
    m = [[0] * k for _ in range(k)]
    for i in range(k):
        m[i][i] = 1
        if i + 1 < k:
            m[i][i + 1] = (-q) % p
    return m


def correct_direct(u: Sequence[int], q: int, p: int) -> List[int]:
    """mu = Q_k u mod p, the correction written as a matrix-vector product."""
    k = len(u)
    m = q_matrix(k, q, p)
    return [sum(m[i][j] * u[j] for j in range(k)) % p for i in range(k)]


def correct_by_tables(u: Sequence[int], q: int, p: int, j: int) -> Tuple[List[int], int]:
    """The REDQ correction by lookups in a table of the first j-1 rows of Q_{j-1}.

    The table maps j consecutive residues (u_i .. u_{i+j-1}) to j-1 corrected
    ones (section 3.5, example ex:tmto with j = 3).  Blocks overlap by one
    residue; the last block is shifted down so that it ends at u_d.  Returns
    (mu, number of table accesses).
    """
    k = len(u)
    assert 2 <= j <= k
    table = {}

    def lookup(block):
        key = tuple(block)
        if key not in table:
            table[key] = [(block[t] - q * block[t + 1]) % p for t in range(j - 1)]
        return table[key]

    mu = [None] * k
    mu[k - 1] = u[k - 1]
    start, accesses = 0, 0
    while start < k - 1:
        s = min(start, k - j)
        out = lookup(u[s:s + j])
        accesses += 1
        for t in range(j - 1):
            mu[s + t] = out[t]
        start = s + j - 1
    return mu, accesses


# --- FDIV / AFDIV (section 4) with exact rational rounding --------------------

UP, NEAREST, DOWN = "up", "nearest", "down"


def round_beta(x: Fraction, beta: int, mode: str) -> Fraction:
    """Round a non-negative rational to a beta-bit binary floating-point number.

    up = towards +inf, down = towards -inf, nearest = to nearest with ties to
    even (ties are irrelevant to the paper's results).  Unbounded exponent.
    """
    x = Fraction(x)
    if x == 0:
        return Fraction(0)
    assert x > 0
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    # now 2^e <= x < 2^(e+1); ulp = 2^(e - beta + 1)
    ulp = Fraction(2) ** (e - beta + 1)
    m = x / ulp
    fl = m.numerator // m.denominator
    if m == fl:
        r = fl
    elif mode == UP:
        r = fl + 1
    elif mode == DOWN:
        r = fl
    else:
        rem = m - fl
        if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
            r = fl + 1
        else:
            r = fl
    return r * ulp


def fdiv(r: int, p: int, beta: int, mode1: str, mode2: str) -> int:
    """Algorithm FDIV: invp = o1(1/p); x = o2(r*invp); return floor(x)."""
    invp = round_beta(Fraction(1, p), beta, mode1)
    x = round_beta(r * invp, beta, mode2)
    return x.numerator // x.denominator


def afdiv(r: int, p: int, beta: int, mode: str) -> int:
    """Algorithm AFDIV for the current rounding mode (section 4.6).

    invp is precomputed per mode (nearest for mode up, up for the two others),
    the bound B per mode, and one test corrects y when r >= B.
    """
    b_updn = Fraction(2 ** beta) / (3 + Fraction(2) ** (1 - beta))
    bound = {UP: b_updn, NEAREST: b_updn, DOWN: Fraction(2 ** (beta - 1))}[mode]
    invp = round_beta(Fraction(1, p), beta, NEAREST if mode == UP else UP)
    x = round_beta(r * invp, beta, mode)
    y = x.numerator // x.denominator
    if r >= bound and p * y > r:
        y -= 1
    return y


# --- Small polynomial arithmetic over F_p (pure Python, for GF tables/pins) ----

def poly_mul(a: Sequence[int], b: Sequence[int], p: int) -> List[int]:
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] = (out[i + j] + x * y) % p
    return out


def poly_trim(a: Sequence[int]) -> List[int]:
    a = list(a)
    while len(a) > 1 and a[-1] == 0:
        a.pop()
    return a


def poly_divmod(a: Sequence[int], m: Sequence[int], p: int) -> Tuple[List[int], List[int]]:
    """Quotient and remainder of a by m over F_p (m's leading coefficient invertible)."""
    a = poly_trim([x % p for x in a])
    m = poly_trim([x % p for x in m])
    inv_lead = pow(m[-1], p - 2, p)
    dm = len(m) - 1
    if len(a) - 1 < dm:
        return [0], a
    q = [0] * (len(a) - dm)
    r = list(a)
    for j in range(len(a) - 1, dm - 1, -1):
        c = (r[j] * inv_lead) % p
        q[j - dm] = c
        if c:
            for i in range(dm + 1):
                r[j - dm + i] = (r[j - dm + i] - c * m[i]) % p
    rem = poly_trim(r[:dm]) if dm > 0 else [0]
    return poly_trim(q), rem


def gf_mul_py(a: Sequence[int], b: Sequence[int], p: int, modulus: Sequence[int]) -> List[int]:
    """One GF(p^k) product (pure Python): product then remainder, padded to k coefficients."""
    k = len(modulus) - 1
    _, r = poly_divmod(poly_mul(a, b, p), modulus, p)
    return (list(r) + [0] * k)[:k]


def all_elements(p: int, k: int):
    """Every polynomial of degree < k over F_p, as coefficient lists (low degree first)."""
    for idx in range(p ** k):
        yield [(idx // p ** i) % p for i in range(k)]


def gf_inverse_bruteforce(a: Sequence[int], p: int, modulus: Sequence[int]) -> List[int]:
    """The inverse of a nonzero element, by trying every element of the field."""
    k = len(modulus) - 1
    one = [1] + [0] * (k - 1)
    for c in all_elements(p, k):
        if gf_mul_py(a, c, p, modulus) == one:
            return c
    raise ValueError("not invertible")


def gf_inverse_euclid(a: Sequence[int], p: int, modulus: Sequence[int]) -> List[int]:
    """The inverse by the extended Euclidean algorithm in F_p[X]."""
    k = len(modulus) - 1

    def sub(x, y):
        n = max(len(x), len(y))
        x = list(x) + [0] * (n - len(x))
        y = list(y) + [0] * (n - len(y))
        return poly_trim([(u - v) % p for u, v in zip(x, y)])

    r0, r1 = poly_trim(modulus), poly_trim(a)
    s0, s1 = [0], [1]
    while r1 != [0]:
        qt, rm = poly_divmod(r0, r1, p)
        r0, r1 = r1, rm
        s0, s1 = s1, sub(s0, poly_mul(qt, s1, p))
    if len(r0) != 1:
        raise ValueError("not invertible")
    c = pow(r0[0], p - 2, p)
    inv = [(x * c) % p for x in s0]
    _, inv = poly_divmod(inv, modulus, p)
    return (list(inv) + [0] * k)[:k]


def is_irreducible(modulus: Sequence[int], p: int) -> bool:
    """Irreducibility by the field criterion: every nonzero residue class is invertible.

    Checked by brute force over all p^k - 1 nonzero classes (tiny fields only):
    F_p[X]/(P) is a field exactly when P is irreducible.
    """
    k = len(modulus) - 1
    one = [1] + [0] * (k - 1)
    elems = [e for e in all_elements(p, k) if any(e)]
    for a in elems:
        if not any(gf_mul_py(a, c, p, modulus) == one for c in elems):
            return False
    return True


def fgdp_reduce(u: Sequence[int], q: int, p: int, modulus: Sequence[int]) -> List[int]:
    """The two-table reduction of algorithm FGDP on compressed residues u_0 .. u_{2k-2} (theorem thm:fgdp).

    L is computed from (u_0 .. u_{k-1}) alone, H from (u_{k-1} .. u_{2k-2})
    alone, and R = H + L in the field.  This is the paper's two-table
    reduction, evaluated directly (no tables); it must equal the plain
    product reduced mod the modulus.
    """
    k = len(modulus) - 1
    assert len(u) == 2 * k - 1
    low = [(u[i] - q * u[i + 1]) % p for i in range(k - 1)]          # mu_0 .. mu_{k-2}
    high = [0] * (2 * k - 1)
    for i in range(k - 1, 2 * k - 2):
        high[i] = (u[i] - q * u[i + 1]) % p                              # mu_{k-1} .. mu_{2k-3}
    high[2 * k - 2] = u[2 * k - 2] % p                                   # mu_{2k-2}
    _, h = poly_divmod(high, modulus, p)
    h = (list(h) + [0] * k)[:k]
    low = (low + [0] * k)[:k]
    return [(x + y) % p for x, y in zip(h, low)]


# --- Compressed matrix products (section 7.4, 7.5): the words, by definition ----

def compressed_words(A: Sequence[Sequence[int]], B: Sequence[Sequence[int]], er: int, ec: int,
                     logQ: int) -> List[List[int]]:
    """CC = CA x CB as exact integers, with CA packing er consecutive rows of A in
    powers of Q and CB packing ec consecutive columns of B in powers of Theta =
    Q^er (section 7.5; er = 1 is Right compression, ec = 1 Left, section 7.4).
    Small inputs only (pure Python)."""
    Q = 1 << logQ
    theta = Q ** er
    m, k, n = len(A), len(B), len(B[0]) if B else 0
    mw, nw = -(-m // er), -(-n // ec)
    CA = [[sum((A[i * er + s][l] if i * er + s < m else 0) * Q ** s for s in range(er)) for l in range(k)]
          for i in range(mw)]
    CB = [[sum((B[l][j * ec + t] if j * ec + t < n else 0) * theta ** t for t in range(ec)) for j in range(nw)]
          for l in range(k)]
    return [[sum(CA[i][l] * CB[l][j] for l in range(k)) for j in range(nw)] for i in range(mw)]


def compressed_digits(CC: Sequence[Sequence[int]], er: int, ec: int, logQ: int, m: int, n: int) -> List[List[int]]:
    """Read C back from the words: digit s + er t of word (i, j) is entry (er i + s, ec j + t)."""
    C = [[0] * n for _ in range(m)]
    for i, row in enumerate(CC):
        for j, w in enumerate(row):
            for s in range(er):
                for t in range(ec):
                    r, c = er * i + s, ec * j + t
                    if r < m and c < n:
                        C[r][c] = (w >> (logQ * (s + er * t))) & ((1 << logQ) - 1)
    return C


# --- A priori bounds (closed forms) -------------------------------------------

def dqt_bounds_ok(p: int, k: int, n: int, logq: int, beta: int) -> bool:
    """Theorem eq:bounds: q > n k (p-1)^2 and (2k-1) log2 q <= beta."""
    return (1 << logq) > n * k * (p - 1) ** 2 and (2 * k - 1) * logq <= beta


def cmm_bounds_ok(p: int, kdim: int, logQ: int, d: int, beta: int) -> bool:
    """eq:lower k (p-1)^2 < Q and eq:upper Q^(d+1) < 2^beta (section 7.2)."""
    return kdim * (p - 1) ** 2 < (1 << logQ) and logQ * (d + 1) < beta


def compression_factor(logQ: int, beta: int) -> int:
    """e = floor(beta / log2 Q) (section 7.6.1)."""
    return beta // logQ
