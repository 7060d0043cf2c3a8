"""The C ABI without a GPU: the library loads, exports every declared symbol, and
its host-only logic (a priori bounds, plans, argument checks) is right."""
import ctypes
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dqt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:dqt_status|size_t|uint32_t|const char\s*\*|char\s*\*|void)\s*\*?\s*(\w+)\s*\(",
                       text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def D():
    from paper_0809_0063_amd import build, dqt
    build.ensure_built()
    return dqt


def test_header_parses():
    names = declared_functions()
    for must in ("dqt_pack", "dqt_polymul", "redq_unpack", "dqt_fgemm", "dqt_qadic_check", "dqt_qadic_choose",
                 "dqt_fgemm_batched", "dqt_polymul_u8", "dqt_gf_mul_u8", "dqt_debug_enable", "dqt_sync_status"):
        assert must in names


def test_every_declared_symbol_is_exported(D):
    lib = D.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(D):
    lib = D.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.dqt_status_str(s)
    assert b"gfx950" in lib.dqt_version()


@pytest.mark.parametrize("p", [2, 3, 5, 7, 11, 13, 31, 127, 251])
def test_qadic_choose_matches_eq_bounds(D, p):
    for k in range(1, 10):
        for n in (1, 2, 3, 7, 100):
            want = None
            for b in range(1, 33):
                if O.dqt_bounds_ok(p, k, n, b, 53):
                    want = b
                    break
            if want is None:
                with pytest.raises(D.DQTError) as e:
                    D.qadic_choose(p, k, n)
                assert e.value.status == D.DQT_E_BOUND
            else:
                q = D.qadic_choose(p, k, n)
                assert (q.log2q, q.nres, q.k_coeffs, q.n_accum) == (want, 2 * k - 1, k, n)


def test_qadic_check_grid(D):
    for p in (2, 3, 5, 7, 251):
        for k in (1, 2, 4, 7):
            for n in (1, 3, 1000):
                for b in range(1, 33):
                    st = D.qadic_check(D.Qadic(p, b, k, 2 * k - 1, n))
                    assert (st == 0) == O.dqt_bounds_ok(p, k, n, b, 53), (p, k, n, b)
    # the degree-3 polynomials over F_3 at q = 2^6 admit up to 3 accumulated products
    assert D.qadic_check(D.Qadic(3, 6, 4, 7, 3)) == 0
    assert D.qadic_check(D.Qadic(3, 6, 4, 7, 4)) == D.DQT_E_BOUND
    assert D.qadic_check(D.Qadic(1, 6, 4, 7, 1)) == D.DQT_E_INVALID


def test_argument_errors_before_any_device_call(D):
    lib = D.lib()
    # p out of range, k too large for one word, bounds violated: refused on the host
    assert lib.dqt_polymul_u8(None, None, 10, 4, 1, 0, None, None) == D.DQT_E_INVALID
    assert lib.dqt_polymul_u8(None, None, 10, 10, 251, 0, None, None) == D.DQT_E_UNSUPPORTED
    assert lib.dqt_polymul_u8(None, None, 10, 4, 3, 4, None, None) == D.DQT_E_BOUND
    assert lib.dqt_polymul_u8(None, None, 0, 4, 3, 6, None, None) == D.DQT_OK   # empty: no-op
    mod_bad = (ctypes.c_uint8 * 6)(1, 2, 0, 0, 0, 2)  # not monic
    assert lib.dqt_gf_mul_u8(None, None, 10, 5, 3, 0, mod_bad, None, None) == D.DQT_E_INVALID
    assert lib.dqt_gf_mul_u8(None, None, 10, 5, 3, 0, None, None, None) == D.DQT_E_INVALID
    q = D.Qadic(3, 13, 1, 5, 1)._c()  # 5 * 13 > 53
    assert lib.redq_unpack(None, 10, ctypes.byref(q), None, None, None) == D.DQT_E_BOUND
    assert lib.dqt_fgemm(300, 4, 4, 4, None, 4, None, 4, None, 4, None, None, 0, None) == D.DQT_E_INVALID
    assert lib.dqt_fgemm(3, 0, 4, 4, None, 4, None, 4, None, 4, None, None, 0, None) == D.DQT_OK
    assert lib.dqt_polymul_fqt_u8(None, 0, None, 4, 10, 3, 0, None, None) == D.DQT_E_INVALID


def test_long_products_planned_without_device(D):
    """An empty batch of long products is planned (block size, q, chunk size and launch shape from
    the cost estimate, whose register counts fall back to a fixed value without a device) and
    accepted; a forced block size whose sums cannot hold four block products is refused."""
    lib = D.lib()
    for p in (2, 3, 7, 31, 127):
        for na, nb in ((65, 65), (70, 500), (500, 500), (1000, 1024), (4096, 4096), (3000, 70)):
            assert lib.dqt_polymul_fqt_u8(None, na, None, nb, 0, p, 0, None, None) == D.DQT_OK, (p, na, nb)
    for block in (2, 3, 4):
        assert lib.dqt_polymul_fqt_u8(None, 500, None, 500, 0, 3, block, None, None) == D.DQT_OK, block
    # blocks of four over F_31: q = 2^7 holds no block product of 4 (p - 1)^2 = 3600
    assert lib.dqt_polymul_fqt_u8(None, 500, None, 500, 0, 31, 4, None, None) == D.DQT_E_BOUND
    assert lib.dqt_polymul_fqt_u8(None, 500, None, 500, 0, 131, 0, None, None) == D.DQT_E_UNSUPPORTED


def test_fgemm_workspace_sizes(D):
    # packed path: words of four entries for the rows of A and the columns of B
    ws = D.fgemm_workspace_size(3, 1024, 1024, 1024)
    assert ws == 256 * (1024 + 1024) * 4
    assert D.fgemm_workspace_size(3, 1024, 1024, 1024, D.GemmPlan(algo=D.GEMM_PLAIN)) == 1024 * 2048 * 4
    assert D.fgemm_workspace_size(3, 100, 100, 100, D.GemmPlan(algo=D.GEMM_MFMA)) == 128 * (128 + 128)
    # packing bounds: a Kronecker pair must fit a 16-bit lane, the interval must fit Q
    assert D.fgemm_workspace_size(251, 64, 64, 64, D.GemmPlan(algo=D.GEMM_CMM)) == 0
    assert D.fgemm_workspace_size(3, 64, 64, 64, D.GemmPlan(algo=D.GEMM_CMM, interval=8192)) == 0


def test_kara_long_workspace_sizes(D):
    """Per level: the 3^l operand pairs of h_l coefficients and their 3^l products of 2 h_l - 1
    coefficients, each region rounded up to 256 bytes; 0 where the arguments are refused."""
    r = lambda x: (x + 255) // 256 * 256
    assert D.kara_long_workspace(10, 100, 1) == r(2 * 30 * 50) + r(30 * 99)
    assert D.kara_long_workspace(10, 100, 2) == r(2 * 30 * 50) + r(30 * 99) + r(2 * 90 * 25) + r(90 * 49)
    assert D.kara_long_workspace(1, 4096, 3) == r(2 * 3 * 2048) + r(3 * 4095) + r(2 * 9 * 1024) + r(9 * 2047) + \
        r(2 * 27 * 512) + r(27 * 1023)
    assert D.kara_long_workspace(0, 100, 1) == 0
    for count, n, levels in ((10, 100, 0), (10, 100, 4), (10, 4097, 1), (10, 2, 1), (10, 7, 3)):
        assert D.kara_long_workspace(count, n, levels) == 0


def test_packed_side_sizes_add_up_to_the_workspace(D):
    """Host logic of the resident-operand calls: the two packed sides are the two halves of the workspace."""
    for p in (2, 3, 7, 13):
        for (m, n, k) in ((1, 1, 1), (17, 130, 333), (1024, 1024, 1024), (64, 5, 4097)):
            for plan in (None, D.GemmPlan(algo=D.GEMM_CMM), D.GemmPlan(algo=D.GEMM_PLAIN),
                         D.GemmPlan(algo=D.GEMM_DOT4), D.GemmPlan(algo=D.GEMM_MFMA),
                         D.GemmPlan(algo=D.GEMM_CMM, tile_rows=8), D.GemmPlan(algo=D.GEMM_RIGHT),
                         D.GemmPlan(algo=D.GEMM_LEFT), D.GemmPlan(algo=D.GEMM_FULL)):
                ws = D.fgemm_workspace_size(p, m, n, k, plan)
                a = D.fgemm_packed_bytes(p, m, k, 0, plan)
                b = D.fgemm_packed_bytes(p, n, k, 1, plan)
                assert a + b == ws, (p, m, n, k, plan, a, b, ws)
    assert D.fgemm_packed_bytes(3, 8, 8, 5, None) == 0
    assert D.fgemm_packed_bytes(1, 8, 8, 0, None) == 0
    lib = D.lib()
    # null operand or packed buffer, bad side: refused before any launch
    assert lib.dqt_fgemm_pack_side(3, 8, 8, None, 8, 0, None, None, None) == D.DQT_E_INVALID
    assert lib.dqt_fgemm_pack_side(3, 8, 8, None, 8, 3, None, None, None) == D.DQT_E_INVALID
    assert lib.dqt_fgemm_packed(3, 8, 8, 8, None, None, None, 8, None, None) == D.DQT_E_INVALID


def test_compressed_f64_plan_sizes(D):
    """Matrix-core compressed products: digits per word from eq:lower and the 52-bit budget."""
    # p = 3, k = 1024: Q = 2^13, four digits per word
    m = n = k = 1024
    ws = D.fgemm_workspace_size(3, m, n, k, D.GemmPlan(algo=D.GEMM_RIGHT))
    assert ws == 1024 * 1024 + 256 * 1024 * 8     # A uncompressed (uint8), B four columns per binary64 word
    ws = D.fgemm_workspace_size(3, m, n, k, D.GemmPlan(algo=D.GEMM_LEFT))
    assert ws == 256 * 1024 * 8 + 1024 * 1024     # A four rows per binary64 word, B^T uncompressed (uint8)
    ws = D.fgemm_workspace_size(3, m, n, k, D.GemmPlan(algo=D.GEMM_FULL))
    assert ws == (512 + 512) * 1024 * 8           # two rows and two columns per word
    # fewer than two digits per word: unsupported (size 0); FULL needs four
    assert D.fgemm_workspace_size(251, 64, 64, 1 << 20, D.GemmPlan(algo=D.GEMM_RIGHT)) == 0
    assert D.fgemm_workspace_size(13, 64, 64, 1024, D.GemmPlan(algo=D.GEMM_FULL)) == 0
    assert D.fgemm_workspace_size(13, 64, 64, 1024, D.GemmPlan(algo=D.GEMM_RIGHT)) > 0
    # a Q below the bound is refused
    assert D.fgemm_workspace_size(3, 64, 64, 1024, D.GemmPlan(algo=D.GEMM_RIGHT, log2Q=12)) == 0


def test_input_status(D):
    lib = D.lib()
    assert lib.dqt_status_str(D.DQT_E_INPUT).startswith(b"input check failed")
    # argument checks before any device call
    assert lib.dqt_check_input_u8(None, 10, 3, None, None) == D.DQT_E_INVALID
    assert lib.dqt_check_input_u8(None, 0, 3, None, None) == D.DQT_E_INVALID
    assert lib.dqt_check_input_u8(None, 10, 1, None, None) == D.DQT_E_INVALID


def test_shape_rule_picks_by_largest_dimension(D):
    """Section 7.6.2: middle product when k is the largest dimension, Right when n is, Left when m is."""
    ws = lambda m, n, k, a: D.fgemm_workspace_size(3, m, n, k, D.GemmPlan(algo=a))
    for (m, n, k, want) in ((64, 1024, 256, D.GEMM_RIGHT), (1024, 64, 256, D.GEMM_LEFT),
                            (64, 64, 1024, D.GEMM_AUTO), (300, 300, 300, D.GEMM_AUTO)):
        assert ws(m, n, k, D.GEMM_BY_SHAPE) == ws(m, n, k, want), (m, n, k)
    # no two digits fit a binary64 word: the middle product (or plain) path instead
    assert D.fgemm_workspace_size(251, 8, 4096, 1 << 20, D.GemmPlan(algo=D.GEMM_BY_SHAPE)) == \
        D.fgemm_workspace_size(251, 8, 4096, 1 << 20, D.GemmPlan(algo=D.GEMM_AUTO))


def test_table_window_setting(D):
    assert D.get_table_window() == 0
    for j in (1, 2, 3, 0):
        D.set_table_window(j)
        assert D.get_table_window() == j
    with pytest.raises(D.DQTError) as e:
        D.set_table_window(4)
    assert e.value.status == D.DQT_E_INVALID
    assert D.get_table_window() == 0
    assert "dqt_get_table_window" in declared_functions()


def test_word_bits_bound_the_packed_result(D):
    """eq:bounds with beta = word_bits: nres log2 q <= beta; 0 means 53, more than 53 is unsupported."""
    for beta in (0, 53, 40, 24):
        b_eff = beta or 53
        for p in (2, 3, 7):
            for k in (1, 2, 3, 4):
                want = None
                for b in range(1, 33):
                    if O.dqt_bounds_ok(p, k, 1, b, b_eff):
                        want = b
                        break
                if want is None:
                    with pytest.raises(D.DQTError) as e:
                        D.qadic_choose(p, k, 1, word_bits=beta)
                    assert e.value.status == D.DQT_E_BOUND
                else:
                    q = D.qadic_choose(p, k, 1, word_bits=beta)
                    assert (q.log2q, q.word_bits) == (want, beta)
    # degree 3 over F_3 at q = 2^6 needs 42 bits: fits beta = 42, not 41
    assert D.qadic_check(D.Qadic(3, 6, 4, 7, 1, 42)) == 0
    assert D.qadic_check(D.Qadic(3, 6, 4, 7, 1, 41)) == D.DQT_E_BOUND
    assert D.qadic_check(D.Qadic(3, 6, 4, 7, 1, 60)) == D.DQT_E_UNSUPPORTED
    with pytest.raises(D.DQTError) as e:
        D.qadic_choose(3, 4, 1, word_bits=64)
    assert e.value.status == D.DQT_E_UNSUPPORTED
    lib = D.lib()
    q = D.Qadic(3, 6, 4, 7, 1, 60)._c()
    assert lib.redq_unpack(None, 10, ctypes.byref(q), None, None, None) == D.DQT_E_UNSUPPORTED


def test_uint32_sums_bound_every_word_gemm(D):
    """CMM, PLAIN and DOT4 add whole dot products in uint32: kdim (p-1)^2 < 2^32 or the plan is refused."""
    for p in (23, 13, 3):
        e2 = (p - 1) ** 2
        k_ok = (2 ** 32 - 1) // e2
        for algo in (D.GEMM_CMM, D.GEMM_AUTO, D.GEMM_PLAIN, D.GEMM_DOT4):
            pl = D.GemmPlan(algo=algo)
            assert D.fgemm_workspace_size(p, 1, 1, k_ok + 1, pl) == 0, (p, algo)
            if k_ok < 2 ** 31:
                assert D.fgemm_workspace_size(p, 1, 1, k_ok, pl) > 0, (p, algo)
    # the example of a 23-residue product with 9,000,000 terms
    assert D.fgemm_workspace_size(23, 1, 1, 9_000_000, D.GemmPlan(algo=D.GEMM_CMM)) == 0
    assert D.fgemm_workspace_size(23, 1, 1, 9_000_000, None) == 0
    lib = D.lib()
    assert lib.dqt_fgemm(23, 1, 1, 9_000_000, None, 9_000_000, None, 1, None, 1, None, None, 0, None) == \
        D.DQT_E_UNSUPPORTED


def test_shape_rule_refused_for_one_packed_side(D):
    """A side packed on its own cannot know the algorithm the shape rule would pick for the product."""
    pl = D.GemmPlan(algo=D.GEMM_BY_SHAPE)
    for side in (0, 1):
        assert D.fgemm_packed_bytes(3, 1500, 1800, side, pl) == 0
    lib = D.lib()
    cp = pl._c()
    assert lib.dqt_fgemm_pack_side(3, 8, 8, None, 8, 0, ctypes.byref(cp), None, None) == D.DQT_E_INVALID
    assert lib.dqt_fgemm_packed(3, 8, 8, 8, None, None, None, 8, ctypes.byref(cp), None) == D.DQT_E_INVALID


def test_batched_launch_shapes(D):
    """Workspace sizes of a batch for every accepted launch shape (rows, k-split, columns); the shape
    whose LDS partial sums would exceed the workgroup's share (16 rows, 4 columns, 8 waves) and
    unknown shapes get 0."""
    descs = (D._GemmDesc * 2)()
    for i, (m, n, k, p) in enumerate([(100, 70, 300, 3), (1024, 1024, 1024, 7)]):
        descs[i] = D._GemmDesc(0x1000, 0x2000, 0x3000, m, n, k, k, n, n, p, D.GEMM_CMM, 0, 0, 0)
    ok = [(8, 2, 2), (8, 4, 2), (8, 8, 2), (16, 2, 2), (16, 4, 2), (16, 8, 2), (8, 2, 4), (8, 4, 4), (8, 8, 4),
          (16, 2, 4), (16, 4, 4)]
    for shape in ok:
        assert D.fgemm_batched_workspace_size(descs, *shape) > 0, shape
    for shape in [(16, 8, 4), (4, 2, 2), (8, 3, 2), (8, 2, 3)]:
        assert D.fgemm_batched_workspace_size(descs, *shape) == 0, shape
