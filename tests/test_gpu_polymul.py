"""GPU parity: one-word polynomial products, REDQ unpack, GF(p^k) products (bit-exact vs the oracle).

All calls go through the C ABI (paper_0809_0063_amd.dqt).  Inputs come from the
seeded generator; expected values from the CPU oracle only.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle as O
from paper_0809_0063_amd import inputs
from tests.gpu_util import device, to_dev, to_host, unaligned_like, unaligned_empty

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dqt():
    device()
    from paper_0809_0063_amd import dqt as D
    return D


def test_small_polymul_workload(dqt):
    """65,536 products of degree-3 polynomials over F_3 (q = 2^6, one 64-bit word)."""
    a, b = inputs.polymul_pairs(65536, 4, 3)
    ref = O.polymul(a, b, 3)
    got = to_host(dqt.polymul_u8(to_dev(a), to_dev(b), 3, log2q=6))
    assert got.shape == (65536, 7)
    assert (got == ref).all()
    # every admissible q gives the same bytes (q > 16 and 7 log2 q <= 53)
    for lq in (5, 7):
        assert (to_host(dqt.polymul_u8(to_dev(a), to_dev(b), 3, log2q=lq)) == ref).all()
    with pytest.raises(dqt.DQTError) as e:
        dqt.polymul_u8(to_dev(a), to_dev(b), 3, log2q=4)
    assert e.value.status == dqt.DQT_E_BOUND
    # all 6,561 pairs and the all-2 worst case at q = 2^6 (the compile-time specialised kernel)
    elems = np.array(list(itertools.product(range(3), repeat=4)), dtype=np.uint8)
    ea, eb = np.repeat(elems, len(elems), axis=0), np.tile(elems, (len(elems), 1))
    assert (to_host(dqt.polymul_u8(to_dev(ea), to_dev(eb), 3, log2q=6)) == O.polymul(ea, eb, 3)).all()
    w = inputs.worst_case((1027, 4), 3)
    assert (to_host(dqt.polymul_u8(to_dev(w), to_dev(w), 3, log2q=6)) == O.polymul(w, w, 3)).all()
    plain = to_host(dqt.polymul_plain_u8(to_dev(a), to_dev(b), 3))
    assert (plain == ref).all()


@pytest.mark.parametrize("p,k", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_polymul_all_pairs(dqt, p, k):
    elems = np.array(list(itertools.product(range(p), repeat=k)), dtype=np.uint8)
    a = np.repeat(elems, len(elems), axis=0)
    b = np.tile(elems, (len(elems), 1))
    ref = O.polymul(a, b, p)
    assert (to_host(dqt.polymul_u8(to_dev(a), to_dev(b), p)) == ref).all()
    assert (to_host(dqt.polymul_plain_u8(to_dev(a), to_dev(b), p)) == ref).all()


def _supported_pairs():
    out = []
    for p in (2, 3, 5, 7, 11, 13, 17, 31, 61, 127, 251):
        for k in range(1, 10):
            if O.dqt_bounds_ok(p, k, 1, max(1, (k * (p - 1) ** 2).bit_length()), 53):
                out.append((p, k))
    return out


@pytest.mark.parametrize("p,k", _supported_pairs())
def test_polymul_fields_and_degrees(dqt, p, k):
    q = dqt.qadic_choose(p, k, 1)
    assert O.dqt_bounds_ok(p, k, 1, q.log2q, 53) and not O.dqt_bounds_ok(p, k, 1, q.log2q - 1, 53)
    for count in (1, 3, 4, 5, 1023, 4097):
        a, b = inputs.polymul_pairs(count, k, p, seed=count * 31 + p)
        ref = O.polymul(a, b, p)
        assert (to_host(dqt.polymul_u8(to_dev(a), to_dev(b), p)) == ref).all(), (p, k, count)
        assert (to_host(dqt.polymul_plain_u8(to_dev(a), to_dev(b), p)) == ref).all(), (p, k, count)
    w = inputs.worst_case((257, k), p)
    assert (to_host(dqt.polymul_u8(to_dev(w), to_dev(w), p)) == O.polymul(w, w, p)).all()


def test_polymul_unsupported_degree(dqt):
    # degree 9 over F_251 cannot fit one 53-bit word
    a = torch.zeros((4, 10), dtype=torch.uint8, device=device())
    with pytest.raises(dqt.DQTError) as e:
        dqt.polymul_u8(a, a, 251)
    assert e.value.status == dqt.DQT_E_UNSUPPORTED


def test_polymul_empty_and_unaligned(dqt):
    z = torch.zeros((0, 4), dtype=torch.uint8, device=device())
    assert dqt.polymul_u8(z, z, 3).shape == (0, 7)
    a, b = inputs.polymul_pairs(1001, 4, 3, seed=5)
    ref = O.polymul(a, b, 3)
    out = unaligned_empty((1001, 7), 3)
    dqt.polymul_u8(unaligned_like(a, 1), unaligned_like(b, 2), 3, out=out)
    assert (to_host(out) == ref).all()


def test_unfused_composition_matches(dqt):
    """pack -> packed product -> REDQ gives the same bytes as the fused kernel."""
    for p, k in [(3, 4), (2, 5), (5, 3), (7, 3), (11, 2), (3, 5)]:
        a, b = inputs.polymul_pairs(3000, k, p, seed=k + 100 * p)
        q = dqt.qadic_choose(p, k, 1)
        wa, wb = dqt.pack(to_dev(a), q), dqt.pack(to_dev(b), q)
        assert (to_host(wa).view(np.uint64) == O.dqt_eval(a, q.log2q)).all()
        assert (to_host(dqt.pack(to_dev(a), q, reverse=True)).view(np.uint64) == O.dqt_eval(a, q.log2q, True)).all()
        r = dqt.polymul_words(wa, wb, q)
        got = to_host(dqt.redq_unpack(r, q))
        assert (got == O.polymul(a, b, p)).all()
        assert (got == to_host(dqt.polymul_u8(to_dev(a), to_dev(b), p))).all()


@pytest.mark.parametrize("p,b,nres", [(3, 6, 7), (3, 13, 4), (2, 11, 4), (5, 7, 7), (7, 7, 7), (11, 9, 5),
                                      (13, 10, 5), (31, 11, 4), (251, 17, 3), (3, 4, 13), (3, 13, 1),
                                      (7, 3, 17), (5, 26, 2), (3, 5, 10), (3, 8, 6), (5, 17, 3), (3, 16, 3),
                                      (13, 17, 3), (7, 17, 3)])
def test_redq_unpack_words(dqt, p, b, nres):
    """REDQ of arbitrary words with digits < q (top digit free) vs radix conversion + mod p; the last
    four have correction windows of three residues spanning more than 32 bits of the word."""
    g = np.random.default_rng(p * 1000 + b * 10 + nres)
    n = 20000
    top_bits = 53 - b * (nres - 1)
    low = g.integers(0, 2 ** b, size=(n, nres - 1), dtype=np.uint64)
    top = g.integers(0, 2 ** min(top_bits, 62), size=n, dtype=np.uint64)
    r = top << np.uint64(b * (nres - 1))
    for i in range(nres - 1):
        r |= low[:, i] << np.uint64(b * i)
    # words right at the top of the range exercise the one-sided AFDIV test
    r[:8] = np.uint64(2 ** 53 - 1) - np.arange(8, dtype=np.uint64)
    for i in range(8):
        digits = [(int(r[i]) >> (b * j)) & (2 ** b - 1) for j in range(nres - 1)]
        assert all(d < 2 ** b for d in digits)
    rt = torch.from_numpy(r.view(np.int64)).to(device())
    got = to_host(dqt.redq_unpack(rt, dqt.Qadic(p, b, 1, nres, 1)))
    assert (got == O.radix_mod(r, p, b, nres)).all()


@pytest.mark.parametrize("p,k", [(3, 5), (7, 3)])
def test_gf_full_tables(dqt, p, k):
    """Every product of GF(3^5) (59,049) and GF(7^3) (117,649) with the seeded irreducible modulus."""
    P = inputs.irreducible(p, k)
    elems = np.array(list(O.all_elements(p, k)), dtype=np.uint8)
    a = np.repeat(elems, len(elems), axis=0)
    b = np.tile(elems, (len(elems), 1))
    ref = O.gf_mul(a, b, p, P)
    assert (to_host(dqt.gf_mul_u8(to_dev(a), to_dev(b), p, P)) == ref).all()
    assert (to_host(dqt.gf_mul_plain_u8(to_dev(a), to_dev(b), p, P)) == ref).all()
    q = dqt.qadic_choose(p, k, 1)
    r = dqt.polymul_words(dqt.pack(to_dev(a), q), dqt.pack(to_dev(b), q), q)
    assert (to_host(dqt.redq_unpack(r, q, modulus=P)) == ref).all()


@pytest.mark.parametrize("p,k", [(3, 5), (7, 3)])
def test_gf_workload_and_inverse(dqt, p, k):
    """2^24 products per field as in the GF(p^k) workload; a.b.b^-1 = a on 4,096 elements."""
    P = inputs.irreducible(p, k)
    n = 1 << 24
    a, b = inputs.gf_pairs(n, k, p)
    ref = O.gf_mul(a, b, p, P)
    da, db = to_dev(a), to_dev(b)
    got = dqt.gf_mul_u8(da, db, p, P)
    assert (to_host(got) == ref).all()
    # inverse check: b^-1 from the oracle's full table
    elems = np.array(list(O.all_elements(p, k)), dtype=np.uint8)
    m = len(elems)
    tab = O.gf_mul(np.repeat(elems, m, axis=0), np.tile(elems, (m, 1)), p, P).reshape(m, m, k)
    one = np.zeros(k, np.uint8)
    one[0] = 1
    inv = {}
    for i in range(1, m):
        j = int(np.nonzero((tab[i] == one).all(axis=1))[0][0])
        inv[i] = elems[j]
    weights = p ** np.arange(k)
    idx = (b[:4096].astype(np.int64) * weights).sum(axis=1)
    sel = np.nonzero(idx)[0]
    binv = np.stack([inv[int(i)] for i in idx[sel]])
    back = dqt.gf_mul_u8(got[:4096][sel].contiguous(), to_dev(binv), p, P)
    assert (to_host(back) == a[:4096][sel]).all()


def test_gf_ragged_and_unaligned(dqt):
    for p, k in [(3, 5), (7, 3), (2, 6), (5, 4), (3, 2), (13, 3), (2, 2)]:
        P = inputs.irreducible(p, k)
        for count in (1, 2, 3, 5, 4099):
            a, b = inputs.gf_pairs(count, k, p, seed=count)
            ref = O.gf_mul(a, b, p, P)
            assert (to_host(dqt.gf_mul_u8(to_dev(a), to_dev(b), p, P)) == ref).all(), (p, k, count)
            assert (to_host(dqt.gf_mul_plain_u8(to_dev(a), to_dev(b), p, P)) == ref).all(), (p, k, count)
            out = unaligned_empty((count, k), 1)
            dqt.gf_mul_u8(unaligned_like(a, 3), unaligned_like(b, 2), p, P, out=out)
            assert (to_host(out) == ref).all(), (p, k, count)
            out = unaligned_empty((count, k), 3)
            dqt.gf_mul_plain_u8(unaligned_like(a, 1), unaligned_like(b, 2), p, P, out=out)
            assert (to_host(out) == ref).all(), (p, k, count)


@pytest.mark.parametrize("p,k", [(251, 2), (251, 3), (127, 3)])
def test_gf_plain_large_prime(dqt, p, k):
    """The plain GF comparator's unreduced division steps at the largest primes (sums near their bound)."""
    P = inputs.irreducible(p, k)
    for count in (4096 + 3, 5):
        a, b = inputs.gf_pairs(count, k, p, seed=p + count)
        a[:64] = p - 1
        b[:64] = p - 1
        ref = O.gf_mul(a, b, p, P)
        assert (to_host(dqt.gf_mul_plain_u8(to_dev(a), to_dev(b), p, P)) == ref).all(), (p, k, count)


@pytest.mark.parametrize("p", [2, 3, 5, 7, 11])
def test_fqt_long_products(dqt, p):
    """Block (FQT) products for degrees 2..15 and unequal lengths, every admissible block size."""
    for na, nb in [(3, 3), (5, 5), (8, 8), (11, 11), (16, 16), (5, 13), (16, 2), (1, 9), (32, 32), (20, 7)]:
        for count in (1, 7, 1000):
            a, b = inputs.polymul_pairs(count, na, p, seed=na * 100 + nb + count, kb=nb)
            ref = O.polymul(a, b, p)
            got = to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p))
            assert (got == ref).all(), (p, na, nb, count)
        a, b = inputs.polymul_pairs(300, na, p, seed=na + nb, kb=nb)
        ref = O.polymul(a, b, p)
        for block in range(2, 7):
            try:
                got = to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p, block=block))
            except dqt.DQTError as e:
                assert e.status in (dqt.DQT_E_BOUND, dqt.DQT_E_UNSUPPORTED)
                continue
            assert (got == ref).all(), (p, na, nb, block)
        w = inputs.worst_case((64, na), p)
        wb = inputs.worst_case((64, nb), p)
        assert (to_host(dqt.polymul_fqt_u8(to_dev(w), to_dev(wb), p)) == O.polymul(w, wb, p)).all()


@pytest.mark.parametrize("levels", [-1, 0, 1, 2])
def test_fqt_tiles_unaligned_and_bounded(dqt, levels):
    """The FQT kernels (levels 0: schoolbook blocks, 1-2: Karatsuba) and the plain long-product
    comparator (levels -1, equal lengths from 9 coefficients) move 256 products at a time through
    LDS: operands and results at every byte offset (odd record lengths, so no tile is a whole
    number of words), partial last tiles, and not one byte written outside the result (sentinels
    on both sides)."""
    if levels == -1:
        run = lambda a, b, p, out: dqt.polymul_plain_u8(a, b, p, out=out)
        cases = ((3, 13, 13, 1000), (5, 9, 9, 257), (2, 31, 31, 513), (3, 47, 47, 300), (251, 64, 64, 77))
    else:
        run = (lambda a, b, p, out: dqt.polymul_fqt_u8(a, b, p, out=out)) if levels == 0 else \
              (lambda a, b, p, out: dqt.polymul_fqt_kara_u8(a, b, p, levels=levels, out=out))
        cases = ((3, 13, 7, 1000), (5, 9, 9, 257), (2, 31, 17, 513), (3, 48, 45, 300), (7, 20, 19, 77), (3, 1, 5, 3))
    dev = device()
    for (p, na, nb, count) in cases:
        a, b = inputs.polymul_pairs(count, na, p, seed=na * 7 + nb + levels, kb=nb)
        ref = O.polymul(a, b, p)
        nout = na + nb - 1
        for oa, ob, oo in ((1, 2, 3), (3, 0, 1), (2, 1, 2), (0, 3, 0)):
            flat = torch.full((count * nout + 64,), 0xAB, dtype=torch.uint8, device=dev)
            out = flat[oo:oo + count * nout].view(count, nout)
            run(unaligned_like(a, oa), unaligned_like(b, ob), p, out)
            host = to_host(flat)
            assert (host[oo:oo + count * nout].reshape(count, nout) == ref).all(), (p, na, nb, count, oa, ob, oo)
            assert (host[:oo] == 0xAB).all() and (host[oo + count * nout:] == 0xAB).all(), (p, na, nb, oo)


@pytest.mark.parametrize("levels", [0, 1])
def test_fqt_many_tiles_per_workgroup(dqt, levels):
    """More products than the grid has threads: each workgroup takes several tiles in turn."""
    count, na = 160_001, 12
    a, b = inputs.polymul_pairs(count, na, 3, seed=41 + levels)
    ref = O.polymul(a, b, 3)
    da, db = to_dev(a), to_dev(b)
    got = dqt.polymul_fqt_u8(da, db, 3) if levels == 0 else dqt.polymul_fqt_kara_u8(da, db, 3, levels=levels)
    assert (to_host(got) == ref).all()


@pytest.mark.parametrize("k", [9, 16, 33, 48, 64])
def test_polymul_plain_long(dqt, k):
    """The plain comparator at long degrees (operands staged in LDS by blocks of 256 products)."""
    for p in (2, 3, 251):
        for count in (1, 255, 256, 257, 3000):
            a, b = inputs.polymul_pairs(count, k, p, seed=k * 7 + count + p)
            got = to_host(dqt.polymul_plain_u8(to_dev(a), to_dev(b), p))
            assert (got == O.polymul(a, b, p)).all(), (p, k, count)


@pytest.mark.parametrize("p", [2, 3, 5, 7, 11])
def test_fqt_karatsuba_products(dqt, p):
    """Karatsuba block products (1 and 2 levels) give the oracle's bytes, also for unequal lengths,
    every admissible block size and the all-(p-1) worst case (digits at their bound)."""
    ran = 0
    for na, nb in [(3, 3), (8, 8), (16, 16), (5, 13), (16, 2), (1, 9), (32, 32), (20, 7), (48, 48), (45, 31)]:
        a, b = inputs.polymul_pairs(257, na, p, seed=na * 31 + nb, kb=nb)
        ref = O.polymul(a, b, p)
        da, db = to_dev(a), to_dev(b)
        for levels in (1, 2):
            for block in (0, 2, 3, 4, 5, 6):
                try:
                    got = to_host(dqt.polymul_fqt_kara_u8(da, db, p, levels=levels, block=block))
                except dqt.DQTError as e:
                    # refused exactly when the one-word-per-block FQT refuses (same block and q
                    # choice); with the block size left open the FQT entry then takes the
                    # chunked sums instead
                    assert e.status in (dqt.DQT_E_BOUND, dqt.DQT_E_UNSUPPORTED), e
                    if block == 0:
                        assert (to_host(dqt.polymul_fqt_u8(da, db, p)) == ref).all(), (p, na, nb)
                        continue
                    with pytest.raises(dqt.DQTError) as e2:
                        dqt.polymul_fqt_u8(da, db, p, block=block)
                    assert e2.value.status == e.status
                    continue
                assert (got == ref).all(), (p, na, nb, levels, block)
                ran += 1
        w, wb = inputs.worst_case((64, na), p), inputs.worst_case((64, nb), p)
        want = O.polymul(w, wb, p)
        for levels in (1, 2):
            try:
                got = to_host(dqt.polymul_fqt_kara_u8(to_dev(w), to_dev(wb), p, levels=levels))
            except dqt.DQTError:
                continue
            assert (got == want).all(), (p, na, nb, levels)
    assert ran >= 40
    with pytest.raises(dqt.DQTError):
        dqt.polymul_fqt_kara_u8(da, db, p, levels=3)


@pytest.mark.parametrize("p,k,n", [(3, 5, 1), (3, 5, 7), (7, 3, 1), (7, 3, 9), (7, 3, 10), (7, 3, 100), (3, 2, 1000),
                                   (3, 2, 20000), (2, 6, 33), (5, 4, 17), (13, 3, 5), (3, 5, 128), (7, 3, 129),
                                   (3, 5, 300)])
def test_gf_dot_products(dqt, p, k, n):
    """FGDP dot products: packed sums of n_q products, one REDQ and two lookups per word; lengths on
    each number of lanes per dot product (1 up to 16 elements, 4 up to 128, 16 up to 512, then 64)."""
    P = inputs.irreducible(p, k)
    g = np.random.default_rng(p * 100 + k * 10 + n)
    count = 257 if n < 1000 else 17
    a = g.integers(0, p, size=(count, n, k), dtype=np.uint8)
    b = g.integers(0, p, size=(count, n, k), dtype=np.uint8)
    ref = O.gf_dot(a, b, p, P)
    got = to_host(dqt.gf_dot_u8(to_dev(a), to_dev(b), p, P))
    assert (got == ref).all()
    w = inputs.worst_case((5, n, k), p)
    assert (to_host(dqt.gf_dot_u8(to_dev(w), to_dev(w), p, P)) == O.gf_dot(w, w, p, P)).all()


@pytest.mark.parametrize("p,k", [(3, 5), (7, 3), (2, 6), (13, 2)])
def test_gf_dot_unaligned_operands(dqt, p, k):
    """Operands starting at every byte offset (the kernel reads runs of eight records with 8-byte
    loads at any address), lengths that end inside a run of eight, and results against the oracle;
    the bytes around the output stay untouched."""
    import torch
    P = inputs.irreducible(p, k)
    g = np.random.default_rng(900 + p * 10 + k)
    dev = device()
    for n in (1, 7, 8, 9, 37, 64, 128, 301):
        count = 129
        a = g.integers(0, p, size=(count, n, k), dtype=np.uint8)
        b = g.integers(0, p, size=(count, n, k), dtype=np.uint8)
        a[0] = p - 1
        b[0] = p - 1
        ref = O.gf_dot(a, b, p, P)
        for off in (1, 3, 6):
            bufa = torch.zeros(a.size + 16, dtype=torch.uint8, device=dev)
            bufb = torch.zeros(b.size + 16, dtype=torch.uint8, device=dev)
            va = bufa[off:off + a.size].view(count, n, k)
            vb = bufb[off + 1:off + 1 + b.size].view(count, n, k)
            va.copy_(torch.from_numpy(a))
            vb.copy_(torch.from_numpy(b))
            out = torch.full((count * k + 8,), 0xAB, dtype=torch.uint8, device=dev)
            vo = out[off:off + count * k].view(count, k)
            dqt.gf_dot_u8(va, vb, p, P, out=vo)
            h = out.cpu().numpy()
            assert (h[off:off + count * k].reshape(count, k) == ref).all(), (p, k, n, off)
            assert (h[:off] == 0xAB).all() and (h[off + count * k:] == 0xAB).all()


@pytest.mark.parametrize("p,k", [(3, 5), (7, 3), (2, 6), (13, 2), (3, 2), (5, 3)])
def test_gf_matmul(dqt, p, k):
    """Matrix products over GF(p^k) against the oracle: ragged edges on every tile size a thread
    can take (4 x 2 outputs from 1024 tiles of 64 x 32 up, then 2 x 2, 2 x 1 and 1 x 1: the shapes
    of 2050, 1030 and 520 rows reach the first three, the rest the last), inner dimensions within
    one step of 16, across several, and long enough for several packed sums (n_q > 1) and folds,
    the all-(p-1) worst case, an empty inner dimension (zeros)."""
    import torch
    P = inputs.irreducible(p, k)
    g = np.random.default_rng(600 + p * 10 + k)
    dev = device()
    for m, kd, n in [(1, 1, 1), (64, 16, 32), (65, 17, 33), (130, 40, 70), (7, 300, 5), (3, 1000, 40),
                     (2050, 2, 1000), (1030, 17, 1000), (520, 3, 1000)]:
        a = g.integers(0, p, size=(m, kd, k), dtype=np.uint8)
        b = g.integers(0, p, size=(kd, n, k), dtype=np.uint8)
        a[0] = p - 1
        b[:, 0] = p - 1
        got = to_host(dqt.gf_matmul_u8(to_dev(a), to_dev(b), p, P))
        assert (got == O.gf_matmul(a, b, p, P)).all(), (p, k, m, kd, n)
    z = dqt.gf_matmul_u8(torch.zeros((5, 0, k), dtype=torch.uint8, device=dev),
                         torch.zeros((0, 9, k), dtype=torch.uint8, device=dev), p, P)
    assert z.shape == (5, 9, k) and not to_host(z).any()
    e = dqt.gf_matmul_u8(torch.zeros((0, 4, k), dtype=torch.uint8, device=dev),
                         torch.zeros((4, 9, k), dtype=torch.uint8, device=dev), p, P)
    assert e.shape == (0, 9, k)


def test_gf_matmul_limits(dqt):
    """Fields whose tables do not fit next to the tiles are refused; bad shapes are refused."""
    import torch
    dev = device()
    P = inputs.irreducible(5, 4)        # k w = 12
    x = torch.zeros((4, 4, 4), dtype=torch.uint8, device=dev)
    with pytest.raises(dqt.DQTError) as e:
        dqt.gf_matmul_u8(x, x, 5, P)
    assert e.value.status == dqt.DQT_E_UNSUPPORTED
    with pytest.raises(ValueError):
        dqt.gf_matmul_u8(x, torch.zeros((5, 4, 4), dtype=torch.uint8, device=dev), 5, P)


def test_gf_dot_many_long(dqt):
    """More long dot products than one pass of the grid holds (a wave per dot product, grid-stride),
    and a count that leaves the last pass partly empty."""
    p, k, n = 3, 5, 300
    P = inputs.irreducible(p, k)
    g = np.random.default_rng(4242)
    for count in (5003, 70):
        a = g.integers(0, p, size=(count, n, k), dtype=np.uint8)
        b = g.integers(0, p, size=(count, n, k), dtype=np.uint8)
        assert (to_host(dqt.gf_dot_u8(to_dev(a), to_dev(b), p, P)) == O.gf_dot(a, b, p, P)).all(), count


@pytest.mark.parametrize("p", [2, 3, 5, 7, 13, 31, 127])
def test_fqt_long_products(dqt, p):
    """Products of more than 64 coefficients (one workgroup per product, chunked packed sums) and the plain
    comparator at the same lengths, up to 4096 coefficients, the all-(p-1) case included; 512 and 520
    coefficients sit either side of the plain kernel's switch between its two walks (64 chunk pairs)."""
    g = np.random.default_rng(7000 + p)
    for na, nb, count in [(65, 65, 300), (100, 200, 100), (256, 255, 64), (500, 500, 40), (1000, 1024, 9),
                          (4096, 4096, 3), (65, 4096, 5), (3000, 70, 5),
                          (512, 512, 12), (520, 520, 12)]:
        a = g.integers(0, p, size=(count, na), dtype=np.uint8)
        b = g.integers(0, p, size=(count, nb), dtype=np.uint8)
        a[0] = p - 1
        b[0] = p - 1
        ref = O.polymul(a, b, p)
        got = to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p))
        assert (got == ref).all(), (p, na, nb)
        if na == nb:
            assert (to_host(dqt.polymul_plain_u8(to_dev(a), to_dev(b), p)) == ref).all(), (p, na)


@pytest.mark.parametrize("p", [3, 7, 127])
def test_long_products_several_per_workgroup(dqt, p):
    """Short long products share a wave (64 / pairs products, a group of lanes and an LDS slot each,
    lanes left over when the group size does not divide 64):
    batch sizes that leave the last workgroup partly empty, results between sentinel bytes, for the
    FQT and the plain comparator."""
    import torch
    dev = device()
    g = np.random.default_rng(7300 + p)
    for na, nb in [(65, 65), (70, 100), (129, 128), (200, 250), (300, 300), (65, 7)]:
        for count in (1, 3, 65, 130):
            a = g.integers(0, p, size=(count, na), dtype=np.uint8)
            b = g.integers(0, p, size=(count, nb), dtype=np.uint8)
            a[0] = p - 1
            b[0] = p - 1
            ref = O.polymul(a, b, p)
            nout = na + nb - 1
            runs = [lambda o: dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p, out=o)]
            if na == nb:
                runs.append(lambda o: dqt.polymul_plain_u8(to_dev(a), to_dev(b), p, out=o))
            for run in runs:
                buf = torch.full((count * nout + 64,), 0xCD, dtype=torch.uint8, device=dev)
                run(buf[32:32 + count * nout].view(count, nout))
                h = buf.cpu().numpy()
                assert (h[32:32 + count * nout].reshape(count, nout) == ref).all(), (p, na, nb, count)
                assert (h[:32] == 0xCD).all() and (h[32 + count * nout:] == 0xCD).all(), (p, na, nb, count)


@pytest.mark.parametrize("p", [3, 7])
def test_long_products_several_rounds(dqt, p):
    """Batches larger than what fits the device at once, so that every workgroup loops over several
    groups of products (short products several to a wave and four waves to a workgroup; long ones a
    workgroup each), for the FQT and the plain comparator: a sample of products against the oracle,
    the last products of the batch among them."""
    g = np.random.default_rng(7700 + p)
    for n, count in [(65, 200003), (200, 40001), (1000, 3001)]:
        a = g.integers(0, p, size=(count, n), dtype=np.uint8)
        b = g.integers(0, p, size=(count, n), dtype=np.uint8)
        pick = np.unique(np.concatenate([g.choice(count, size=150, replace=False), np.arange(count - 5, count)]))
        ref = O.polymul(a[pick], b[pick], p)
        da, db = to_dev(a), to_dev(b)
        for run in (dqt.polymul_fqt_u8, dqt.polymul_plain_u8):
            got = to_host(run(da, db, p))
            assert (got[pick] == ref).all(), (p, n, count, run.__name__)


def test_fqt_long_block_sizes_and_limits(dqt):
    """Every block size of the long path gives the oracle's bytes; the limits are refused."""
    p, na, nb, count = 3, 777, 500, 20
    a, b = inputs.polymul_pairs(count, na, p, seed=77, kb=nb)
    ref = O.polymul(a, b, p)
    for block in (2, 3, 4):
        got = to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p, block=block))
        assert (got == ref).all(), block
    with pytest.raises(dqt.DQTError) as e:
        dqt.polymul_fqt_u8(to_dev(a), to_dev(b), 131)
    assert e.value.status == dqt.DQT_E_UNSUPPORTED
    big = np.zeros((1, 4097), dtype=np.uint8)
    with pytest.raises(dqt.DQTError) as e:
        dqt.polymul_fqt_u8(to_dev(big), to_dev(big), 3)
    assert e.value.status == dqt.DQT_E_INVALID


def _kara_base(n, levels):
    h = n
    for _ in range(levels):
        h = (h + 1) // 2
    return h


@pytest.mark.parametrize("p", [7, 31, 127])
def test_fqt_short_operands_by_chunked_sums(dqt, p):
    """Up to 64 coefficients, where no block size keeps a whole output block's sum in one word
    (larger p), the FQT entry with the block size left open computes by chunked sums; an explicit
    block size is still refused there."""
    g = np.random.default_rng(7200 + p)
    lengths = [(na, nb) for na in (1, 2, 5, 16, 25, 33, 48, 64) for nb in (1, 3, 16, 33, 64)]
    chunked = 0
    for na, nb in lengths:
        a = g.integers(0, p, size=(37, na), dtype=np.uint8)
        b = g.integers(0, p, size=(37, nb), dtype=np.uint8)
        a[0] = p - 1
        b[0] = p - 1
        ref = O.polymul(a, b, p)
        assert (to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p)) == ref).all(), (p, na, nb)
        refused = 0
        for block in range(2, 7):
            try:
                got = to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), p, block=block))
            except dqt.DQTError as e:
                assert e.status in (dqt.DQT_E_BOUND, dqt.DQT_E_UNSUPPORTED)
                refused += 1
                continue
            assert (got == ref).all(), (p, na, nb, block)
        chunked += refused == 5
    assert chunked >= 1


@pytest.mark.parametrize("p", [2, 3, 7, 31, 127, 251])
def test_kara_long_products(dqt, p):
    """Karatsuba levels over F_p on top of the FQT (1..3 levels, odd lengths so every level pads a
    half, up to 4096 coefficients), the all-(p-1) operands in the first row; over 127 only base
    sizes the FQT takes (one word per output block) are computed, the others refused."""
    g = np.random.default_rng(7100 + p)
    for n, count, levels in [(3, 50, 1), (9, 100, 3), (65, 300, 1), (100, 50, 2), (128, 64, 3), (255, 20, 1),
                             (500, 20, 2), (1001, 9, 1), (2048, 4, 2), (4096, 3, 1), (4095, 2, 3)]:
        a = g.integers(0, p, size=(count, n), dtype=np.uint8)
        b = g.integers(0, p, size=(count, n), dtype=np.uint8)
        a[0] = p - 1
        b[0] = p - 1
        h = _kara_base(n, levels)
        try:   # the base size the FQT takes (an empty batch checks the parameters only)
            z = to_dev(np.zeros((0, h), dtype=np.uint8))
            dqt.polymul_fqt_u8(z, z, p)
        except dqt.DQTError as e0:
            assert p > 127, (p, n, levels)
            with pytest.raises(dqt.DQTError) as e:
                dqt.polymul_kara_long_u8(to_dev(a), to_dev(b), p, levels=levels)
            assert e.value.status == e0.status == dqt.DQT_E_UNSUPPORTED
            continue
        ref = O.polymul(a, b, p)
        got = to_host(dqt.polymul_kara_long_u8(to_dev(a), to_dev(b), p, levels=levels))
        assert (got == ref).all(), (p, n, levels)


def test_kara_long_limits_and_workspace(dqt):
    """Levels outside 1..3, lengths outside 2..4096, a base below 2 coefficients and a short
    workspace are refused; an empty batch is a no-op; the result does not depend on what the
    workspace held before."""
    import torch
    p, n, count = 5, 300, 11
    a, b = inputs.polymul_pairs(count, n, p, seed=5300)
    da, db = to_dev(a), to_dev(b)
    for levels, nn in ((0, 300), (4, 300), (1, 4097), (1, 2), (3, 7)):
        assert dqt.kara_long_workspace(count, nn, levels) == 0
        x = torch.zeros((count, nn), dtype=torch.uint8, device=da.device)
        with pytest.raises(dqt.DQTError) as e:
            dqt.polymul_kara_long_u8(x, x, p, levels=levels)
        assert e.value.status == dqt.DQT_E_INVALID, (levels, nn)
    need = dqt.kara_long_workspace(count, n, 2)
    short = torch.empty(need - 1, dtype=torch.uint8, device=da.device)
    with pytest.raises(dqt.DQTError) as e:
        dqt.polymul_kara_long_u8(da, db, p, levels=2, work=short)
    assert e.value.status == dqt.DQT_E_WORKSPACE
    work = torch.full((need,), 255, dtype=torch.uint8, device=da.device)
    ref = O.polymul(a, b, p)
    assert (to_host(dqt.polymul_kara_long_u8(da, db, p, levels=2, work=work)) == ref).all()
    assert (to_host(dqt.polymul_kara_long_u8(da, db, p, levels=2, work=work)) == ref).all()
    z = torch.zeros((0, n), dtype=torch.uint8, device=da.device)
    assert dqt.polymul_kara_long_u8(z, z, p, levels=1).shape == (0, 2 * n - 1)


def test_check_input_and_debug_mode(dqt):
    """An entry >= p is reported (DQT_E_INPUT); debug mode checks every call's inputs."""
    import torch
    a, b = inputs.polymul_pairs(1000, 4, 3)
    da, db = to_dev(a), to_dev(b)
    dqt.check_input(da, 3)
    bad = da.clone()
    bad.view(-1)[777] = 3
    with pytest.raises(dqt.DQTError) as e:
        dqt.check_input(bad, 3)
    assert e.value.status == dqt.DQT_E_INPUT
    dqt.check_input(bad, 5)
    try:
        dqt.debug_enable(True)     # the library's debug mode with a device status word
        assert (to_host(dqt.polymul_u8(da, db, 3)) == O.polymul(a, b, 3)).all()
        with pytest.raises(dqt.DQTError) as e:
            dqt.polymul_u8(bad, db, 3)
        assert e.value.status == dqt.DQT_E_INPUT
        A = torch.zeros((64, 64), dtype=torch.uint8, device=da.device)
        A[5, 7] = 200
        with pytest.raises(dqt.DQTError):
            dqt.fgemm(A, A, 7)
    finally:
        dqt.debug_enable(False)


def test_empty_batches_every_entry(dqt):
    """count = 0 is a no-op for every batched entry point (empty outputs of the right shape)."""
    import torch
    dev = device()
    z4, z10, z5 = (torch.zeros((0, k), dtype=torch.uint8, device=dev) for k in (4, 10, 5))
    assert dqt.polymul_plain_u8(z4, z4, 3).shape == (0, 7)
    assert dqt.polymul_fqt_u8(z10, z10, 3).shape == (0, 19)
    assert dqt.polymul_fqt_kara_u8(z10, z10, 3).shape == (0, 19)
    P = inputs.irreducible(3, 5)
    assert dqt.gf_mul_u8(z5, z5, 3, P).shape == (0, 5)
    assert dqt.gf_mul_plain_u8(z5, z5, 3, P).shape == (0, 5)
    zd = torch.zeros((0, 3, 5), dtype=torch.uint8, device=dev)
    assert dqt.gf_dot_u8(zd, zd, 3, P).shape == (0, 5)


@pytest.mark.parametrize("j", [1, 2, 3])
def test_table_windows_give_identical_bytes(dqt, j):
    """Section 3.5: every correction-table window (none, 2, 3 residues) gives the oracle's bytes."""
    try:
        dqt.set_table_window(j)
        for (p, k) in ((3, 4), (5, 3), (7, 3), (2, 6), (13, 2)):
            a, b = inputs.polymul_pairs(3001, k, p, seed=j * 100 + p)
            assert (to_host(dqt.polymul_u8(to_dev(a), to_dev(b), p)) == O.polymul(a, b, p)).all(), (j, p, k)
        for (p, k) in ((3, 5), (7, 3)):
            P = inputs.irreducible(p, k)
            x, y = inputs.gf_pairs(3001, k, p)
            assert (to_host(dqt.gf_mul_u8(to_dev(x), to_dev(y), p, P)) == O.gf_mul(x, y, p, P)).all(), (j, p, k)
        a, b = inputs.polymul_pairs(501, 30, 5, seed=j, kb=17)
        assert (to_host(dqt.polymul_fqt_u8(to_dev(a), to_dev(b), 5)) == O.polymul(a, b, 5)).all()
    finally:
        dqt.set_table_window(0)
