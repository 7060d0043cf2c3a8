"""GPU parity: F_p matrix products (packed CMM, plain, dot4, dot8, INT8 matrix cores) vs the oracle, bit-exact."""
import numpy as np
import pytest

import oracle as O
from paper_0809_0063_amd import inputs
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dqt():
    device()
    from paper_0809_0063_amd import dqt as D
    return D


def _all_algos(D):
    return [D.GemmPlan(algo=D.GEMM_CMM), D.GemmPlan(algo=D.GEMM_CMM, epilogue=D.EPI_REDQ),
            D.GemmPlan(algo=D.GEMM_PLAIN), D.GemmPlan(algo=D.GEMM_DOT4), D.GemmPlan(algo=D.GEMM_DOT8),
            D.GemmPlan(algo=D.GEMM_MFMA)]


def test_fgemm_1024_p3(dqt):
    """C = A.B mod 3 with m = n = k = 1024 (uniform entries) and the all-2 worst case."""
    A, B = inputs.gemm_pair(1024, 1024, 1024, 3)
    ref = O.fgemm(A, B, 3)
    dA, dB = to_dev(A), to_dev(B)
    for plan in [None] + _all_algos(dqt):
        got = to_host(dqt.fgemm(dA, dB, 3, plan=plan))
        assert (got == ref).all(), plan
    W = to_dev(inputs.worst_case((1024, 1024), 3))
    for plan in [None] + _all_algos(dqt):
        got = to_host(dqt.fgemm(W, W, 3, plan=plan))
        assert (got == (1024 * 4) % 3).all(), plan


@pytest.mark.parametrize("p,m,n,k", [(3, 3000, 3000, 200), (7, 2900, 3100, 333), (127, 2945, 2817, 64),
                                     (2, 2944, 2944, 1)])
def test_fgemm_mfma_large_ragged(dqt, p, m, n, k):
    """The INT8 matrix-core comparator on products of about 3000^2 outputs: uniform entries vs the
    oracle with ragged m, n, k (k = 1 gives each workgroup one wave on k); and all entries p - 1."""
    A, B = inputs.gemm_pair(m, n, k, p, seed=m + n + k)
    plan = dqt.GemmPlan(algo=dqt.GEMM_MFMA)
    got = to_host(dqt.fgemm(to_dev(A), to_dev(B), p, plan=plan))
    assert (got == O.fgemm(A, B, p)).all()
    W = inputs.worst_case((m, k), p)
    V = inputs.worst_case((k, n), p)
    got = to_host(dqt.fgemm(to_dev(W), to_dev(V), p, plan=plan))
    assert (got == (k * (p - 1) ** 2) % p).all()


@pytest.mark.parametrize("p", [2, 3, 5, 7, 11, 13])
def test_fgemm_bound_edges_worst_case(dqt, p):
    """All entries p-1 at inner dimensions around the interval limits (digits at their maximum)."""
    for k in (1, 3, 4, 5, 63, 64, 65, 227, 228, 229, 511, 512, 513, 1020, 1021, 2047, 2048, 2049, 4095, 4096, 4097):
        A = to_dev(inputs.worst_case((33, k), p))
        B = to_dev(inputs.worst_case((k, 65), p))
        want = (k * (p - 1) ** 2) % p
        for plan in [None, dqt.GemmPlan(algo=dqt.GEMM_PLAIN), dqt.GemmPlan(algo=dqt.GEMM_CMM, epilogue=dqt.EPI_REDQ),
                     dqt.GemmPlan(algo=dqt.GEMM_DOT8)]:
            got = to_host(dqt.fgemm(A, B, p, plan=plan))
            assert (got == want).all(), (p, k, plan)


@pytest.mark.parametrize("p", [2, 3, 5, 7, 11])
def test_fgemm_ragged_shapes(dqt, p):
    g = np.random.default_rng(p)
    for _ in range(12):
        m, n, k = (int(x) for x in g.integers(1, 300, size=3))
        A, B = inputs.gemm_pair(m, n, k, p, seed=int(g.integers(1 << 30)))
        ref = O.fgemm(A, B, p)
        dA, dB = to_dev(A), to_dev(B)
        for plan in [None] + _all_algos(dqt):
            got = to_host(dqt.fgemm(dA, dB, p, plan=plan))
            assert (got == ref).all(), (m, n, k, plan)


def test_fgemm_plans(dqt):
    """Every tile/split/interval choice gives the same bytes."""
    p = 5
    A, B = inputs.gemm_pair(200, 300, 1000, p, seed=11)
    ref = O.fgemm(A, B, p)
    dA, dB = to_dev(A), to_dev(B)
    for tm, tn in ((8, 2), (8, 4), (16, 2), (16, 4), (32, 2)):
        for ks in (1, 2, 4, 8):
            if ks * tm * tn * 256 > 65536:
                with pytest.raises(dqt.DQTError):
                    dqt.fgemm(dA, dB, p, plan=dqt.GemmPlan(algo=dqt.GEMM_CMM, tile_rows=tm, tile_cols=tn, ksplit=ks))
                continue
            for interval in (0, 4, 64, 500, 508):
                for epi in (dqt.EPI_REDC, dqt.EPI_REDQ):
                    plan = dqt.GemmPlan(algo=dqt.GEMM_CMM, interval=interval, tile_rows=tm, tile_cols=tn, ksplit=ks,
                                        epilogue=epi)
                    got = to_host(dqt.fgemm(dA, dB, p, plan=plan))
                    assert (got == ref).all(), plan
            for algo in (dqt.GEMM_PLAIN, dqt.GEMM_DOT4, dqt.GEMM_DOT8):
                got = to_host(dqt.fgemm(dA, dB, p, plan=dqt.GemmPlan(algo=algo, tile_rows=tm, tile_cols=tn, ksplit=ks)))
                assert (got == ref).all(), (algo, tm, tn, ks)


def test_fgemm_large_prime_routes_plain(dqt):
    for p in (31, 127, 251):
        A, B = inputs.gemm_pair(70, 90, 300, p, seed=p)
        ref = O.fgemm(A, B, p)
        got = to_host(dqt.fgemm(to_dev(A), to_dev(B), p))
        assert (got == ref).all()
    with pytest.raises(dqt.DQTError) as e:
        dqt.fgemm(to_dev(A), to_dev(B), 251, plan=dqt.GemmPlan(algo=dqt.GEMM_CMM))
    assert e.value.status in (dqt.DQT_E_UNSUPPORTED, dqt.DQT_E_BOUND)
    # four-bit entries stop at p = 16
    with pytest.raises(dqt.DQTError) as e:
        dqt.fgemm(to_dev(A), to_dev(B), 251, plan=dqt.GemmPlan(algo=dqt.GEMM_DOT8))
    assert e.value.status == dqt.DQT_E_UNSUPPORTED


@pytest.mark.parametrize("p", [2, 13, 16])
def test_fgemm_dot8_edges(dqt, p):
    """The eight-entry words at every k mod 8 (partial last word), unaligned leading dimensions and
    the all-(p-1) case; p = 16 (entries 15, a full nibble) included."""
    g = np.random.default_rng(900 + p)
    plan = dqt.GemmPlan(algo=dqt.GEMM_DOT8)
    for k in (1, 7, 8, 9, 15, 16, 17, 1023, 1024, 1025, 4097):
        m, n = int(g.integers(1, 70)), int(g.integers(1, 300))
        A = inputs.uniform_residues((m, k), p, int(g.integers(1 << 30)))
        B = inputs.uniform_residues((k, n), p, int(g.integers(1 << 30)))
        assert (to_host(dqt.fgemm(to_dev(A), to_dev(B), p, plan=plan)) == O.fgemm(A, B, p)).all(), (k, m, n)
        W = to_dev(inputs.worst_case((m, k), p))
        V = to_dev(inputs.worst_case((k, n), p))
        assert (to_host(dqt.fgemm(W, V, p, plan=plan)) == (k * (p - 1) ** 2) % p).all(), k
    # rows that start off 4-byte boundaries take the byte-wise packing
    A = inputs.uniform_residues((45, 203), p, 1)
    B = inputs.uniform_residues((203, 77), p, 2)
    got = to_host(dqt.fgemm(to_dev(A), to_dev(B), p, plan=plan))
    assert (got == O.fgemm(A, B, p)).all()


def test_fgemm_identity_permutation(dqt):
    p = 7
    g = np.random.default_rng(3)
    A = inputs.uniform_residues((129, 129), p, 5)
    I = np.eye(129, dtype=np.uint8)
    P = I[g.permutation(129)]
    dA = to_dev(A)
    assert (to_host(dqt.fgemm(dA, to_dev(I), p)) == A).all()
    assert (to_host(dqt.fgemm(to_dev(P), dA, p)) == (P.astype(np.int64) @ A) % p).all()


def test_fgemm_workspace_errors(dqt):
    import torch
    A = torch.zeros((64, 64), dtype=torch.uint8, device=device())
    ws = dqt.fgemm_workspace_size(3, 64, 64, 64)
    assert ws > 0
    small = torch.zeros(ws - 1, dtype=torch.uint8, device=device())
    C = torch.zeros((64, 64), dtype=torch.uint8, device=device())
    from paper_0809_0063_amd.dqt import _load, _stream
    import ctypes
    st = _load().dqt_fgemm(3, 64, 64, 64, ctypes.c_void_p(A.data_ptr()), 64, ctypes.c_void_p(A.data_ptr()), 64,
                           ctypes.c_void_p(C.data_ptr()), 64, None, ctypes.c_void_p(small.data_ptr()), ws - 1,
                           _stream(None))
    assert st == dqt.DQT_E_WORKSPACE
    # a workspace that is not 16-byte aligned is refused before any launch
    big = torch.zeros(ws + 64, dtype=torch.uint8, device=device())
    st = _load().dqt_fgemm(3, 64, 64, 64, ctypes.c_void_p(A.data_ptr()), 64, ctypes.c_void_p(A.data_ptr()), 64,
                           ctypes.c_void_p(C.data_ptr()), 64, None, ctypes.c_void_p(big.data_ptr() + 4), ws,
                           _stream(None))
    assert st == dqt.DQT_E_INVALID


@pytest.mark.parametrize("p", [2, 3, 7])
def test_fgemm_packed_operands_reused(dqt, p):
    """A packed B kept in its own buffer times several packed A (different m, ragged), and one packed A
    times two packed B: every product equals the oracle (section 7.1, reuse of compressed matrices)."""
    g = np.random.default_rng(100 + p)
    k, n = 333, 257
    _, B = inputs.gemm_pair(1, n, k, p, seed=int(g.integers(1 << 30)))
    dB = to_dev(B)
    for plan in [None] + _all_algos(dqt):
        CB = dqt.fgemm_pack_side(dB, p, 1, plan=plan)
        assert CB.numel() == dqt.fgemm_packed_bytes(p, n, k, 1, plan)
        for m in (1, 17, 130):
            A, _ = inputs.gemm_pair(m, 1, k, p, seed=int(g.integers(1 << 30)))
            dA = to_dev(A)
            CA = dqt.fgemm_pack_side(dA, p, 0, plan=plan)
            got = to_host(dqt.fgemm_packed(CA, CB, p, m, n, k, plan=plan))
            assert (got == O.fgemm(A, B, p)).all(), (plan, m)
            # the same packed A against a second B with fewer columns
            _, B2 = inputs.gemm_pair(1, 65, k, p, seed=int(g.integers(1 << 30)))
            CB2 = dqt.fgemm_pack_side(to_dev(B2), p, 1, plan=plan)
            got2 = to_host(dqt.fgemm_packed(CA, CB2, p, m, 65, k, plan=plan))
            assert (got2 == O.fgemm(A, B2, p)).all(), (plan, m)


def test_fgemm_packed_argument_errors(dqt):
    import torch
    dA = to_dev(inputs.gemm_pair(8, 8, 8, 3)[0])
    assert dqt.fgemm_packed_bytes(3, 8, 8, 2, None) == 0
    with pytest.raises(dqt.DQTError):
        dqt.fgemm_pack_side(dA, 3, 2)
    CA = dqt.fgemm_pack_side(dA, 3, 0)
    with pytest.raises(ValueError):
        dqt.fgemm_pack_side(dA, 3, 0, out=torch.empty(4, dtype=torch.uint8, device=dA.device))
    with pytest.raises(ValueError):
        dqt.fgemm_packed(CA, CA, 3, 8, 8, 8, out=torch.empty((8, 9), dtype=torch.uint8, device=dA.device))


def test_fgemm_call_object_matches(dqt):
    """The prepared-argument launcher gives the same bytes as fgemm."""
    import torch
    A, B = inputs.gemm_pair(200, 300, 500, 5)
    dA, dB = to_dev(A), to_dev(B)
    C = torch.empty((200, 300), dtype=torch.uint8, device=dA.device)
    call = dqt.FgemmCall(dA, dB, C, 5, plan=dqt.GemmPlan(algo=dqt.GEMM_CMM))
    call.pack()
    call.compute()
    assert (to_host(C) == O.fgemm(A, B, 5)).all()


def _f64_digits(p, k):
    """Digits per binary64 word of the matrix-core compressed products: floor(52 / log2 Q) with
    Q the smallest power of two above k (p-1)^2 (eq:lower, eq:upper)."""
    b = max(1, (k * (p - 1) ** 2).bit_length())
    return 52 // b


def _f64_plans(dqt, p, k):
    d = _f64_digits(p, k)
    out = []
    if d >= 2:
        out += [dqt.GemmPlan(algo=dqt.GEMM_RIGHT), dqt.GemmPlan(algo=dqt.GEMM_LEFT)]
    if d >= 4:
        out.append(dqt.GemmPlan(algo=dqt.GEMM_FULL))
    return out


def test_compressed_f64_1024_p3(dqt):
    """Right, Left and Full compression on the FP64 matrix cores, 1024^3 over F_3, uniform and all-2."""
    A, B = inputs.gemm_pair(1024, 1024, 1024, 3)
    ref = O.fgemm(A, B, 3)
    dA, dB = to_dev(A), to_dev(B)
    plans = _f64_plans(dqt, 3, 1024)
    assert len(plans) == 3
    for plan in plans:
        got = to_host(dqt.fgemm(dA, dB, 3, plan=plan))
        assert (got == ref).all(), plan
    W = to_dev(inputs.worst_case((1024, 1024), 3))
    for plan in plans:
        got = to_host(dqt.fgemm(W, W, 3, plan=plan))
        assert (got == (1024 * 4) % 3).all(), plan


@pytest.mark.parametrize("p", [2, 3, 5, 7, 11, 13, 31, 251])
def test_compressed_f64_ragged_and_bounds(dqt, p):
    """Ragged shapes (rows or columns not a multiple of the words' e) and the worst case at inner
    dimensions whose bound k (p-1)^2 sits just below and at a power of two."""
    g = np.random.default_rng(500 + p)
    for _ in range(6):
        m, n, k = (int(x) for x in g.integers(1, 260, size=3))
        A, B = inputs.gemm_pair(m, n, k, p, seed=int(g.integers(1 << 30)))
        ref = O.fgemm(A, B, p)
        dA, dB = to_dev(A), to_dev(B)
        for plan in _f64_plans(dqt, p, k):
            for ks in (0, 1, 8, 16):
                if ks == 16 and plan.algo == dqt.GEMM_FULL:
                    continue
                pl = dqt.GemmPlan(algo=plan.algo, ksplit=ks)
                got = to_host(dqt.fgemm(dA, dB, p, plan=pl))
                assert (got == ref).all(), (m, n, k, pl)
    e2 = (p - 1) ** 2
    for k in sorted({1, 3, 4, 5, max(1, (1 << 12) // e2), (1 << 12) // e2 + 1, 1023, 1024, 1025, 2048}):
        A = to_dev(inputs.worst_case((37, k), p))
        B = to_dev(inputs.worst_case((k, 70), p))
        want = (k * e2) % p
        plans = _f64_plans(dqt, p, k)
        for plan in plans:
            got = to_host(dqt.fgemm(A, B, p, plan=plan))
            assert (got == want).all(), (p, k, plan)
        if not plans:
            with pytest.raises(dqt.DQTError) as e:
                dqt.fgemm(A, B, p, plan=dqt.GemmPlan(algo=dqt.GEMM_RIGHT))
            assert e.value.status == dqt.DQT_E_UNSUPPORTED


def test_compressed_f64_larger_q_and_reuse(dqt):
    """A larger Q than needed (log2Q) still gives the same bytes; packed sides reused."""
    p, m, n, k = 5, 130, 257, 200
    A, B = inputs.gemm_pair(m, n, k, p, seed=77)
    ref = O.fgemm(A, B, p)
    dA, dB = to_dev(A), to_dev(B)
    for algo in (dqt.GEMM_RIGHT, dqt.GEMM_LEFT, dqt.GEMM_FULL):
        for b in (0, 13):
            plan = dqt.GemmPlan(algo=algo, log2Q=b)
            assert (to_host(dqt.fgemm(dA, dB, p, plan=plan)) == ref).all(), plan
        plan = dqt.GemmPlan(algo=algo)
        CB = dqt.fgemm_pack_side(dB, p, 1, plan=plan)
        for rows in (1, 64, 130):
            CA = dqt.fgemm_pack_side(dA[:rows].contiguous(), p, 0, plan=plan)
            got = to_host(dqt.fgemm_packed(CA, CB, p, rows, n, k, plan=plan))
            assert (got == ref[:rows]).all(), (algo, rows)
    with pytest.raises(dqt.DQTError) as e:
        dqt.fgemm(dA, dB, p, plan=dqt.GemmPlan(algo=dqt.GEMM_RIGHT, log2Q=5))   # below k (p-1)^2
    assert e.value.status == dqt.DQT_E_BOUND


def test_fgemm_empty_dimensions(dqt):
    """m = 0 or n = 0: nothing is written; k = 0: C = 0 (empty sums), for every algorithm and through
    the two-phase and resident-operand calls."""
    import torch
    dev = device()
    for plan in [None] + _all_algos(dqt) + _f64_plans(dqt, 3, 64):
        for m, n in ((0, 5), (5, 0), (0, 0)):
            A = torch.zeros((m, 7), dtype=torch.uint8, device=dev)
            B = torch.zeros((7, n), dtype=torch.uint8, device=dev)
            assert tuple(dqt.fgemm(A, B, 3, plan=plan).shape) == (m, n)
        A = torch.zeros((33, 0), dtype=torch.uint8, device=dev)
        B = torch.zeros((0, 130), dtype=torch.uint8, device=dev)
        C = torch.full((33, 130), 9, dtype=torch.uint8, device=dev)
        dqt.fgemm(A, B, 3, plan=plan, out=C)
        assert (to_host(C) == 0).all(), plan
        C.fill_(9)
        CA, CB = dqt.fgemm_pack_side(A, 3, 0, plan=plan), dqt.fgemm_pack_side(B, 3, 1, plan=plan)
        dqt.fgemm_packed(CA, CB, 3, 33, 130, 0, plan=plan, out=C)
        assert (to_host(C) == 0).all(), plan


def test_shape_rule_products(dqt):
    """The shape rule's choice on rectangular products gives the oracle's bytes."""
    for (m, n, k, p) in ((40, 700, 130, 3), (700, 40, 130, 5), (50, 60, 900, 7), (33, 513, 64, 2)):
        A, B = inputs.gemm_pair(m, n, k, p, seed=m + n + k)
        got = to_host(dqt.fgemm(to_dev(A), to_dev(B), p, plan=dqt.GemmPlan(algo=dqt.GEMM_BY_SHAPE)))
        assert (got == O.fgemm(A, B, p)).all(), (m, n, k, p)
