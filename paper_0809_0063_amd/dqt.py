"""Python binding of libdqt (ctypes): argument marshalling only.

Every function forwards torch device tensors (as raw device pointers) and the
current HIP stream to the C ABI declared in include/dqt.h; every step of the
path runs in the library's HIP kernels.  There is no CPU fallback: if the
library is missing or the device is not a GPU the call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdqt.so")

DQT_OK, DQT_E_INVALID, DQT_E_BOUND, DQT_E_UNSUPPORTED, DQT_E_DEVICE, DQT_E_WORKSPACE, DQT_E_INPUT = 0, -1, -2, -3, -4, -5, -6
# DQT_DEBUG=1: the library's debug mode is turned on at load (dqt_debug_enable with a device status
# word): every call then checks its data on the device first and fails with DQT_E_INPUT (blocking)
DEBUG = os.environ.get("DQT_DEBUG", "") not in ("", "0")

GEMM_AUTO, GEMM_CMM, GEMM_PLAIN, GEMM_DOT4, GEMM_MFMA, GEMM_RIGHT, GEMM_LEFT, GEMM_FULL = 0, 1, 2, 3, 4, 5, 6, 7
GEMM_BY_SHAPE = 8
GEMM_DOT8 = 9
EPI_REDC, EPI_REDQ = 0, 1


class DQTError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {_status_str(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class _Qadic(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint32), ("log2q", ctypes.c_uint32), ("k_coeffs", ctypes.c_uint32),
                ("nres", ctypes.c_uint32), ("n_accum", ctypes.c_uint64), ("word_bits", ctypes.c_uint32)]


class _GemmPlan(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("log2Q", ctypes.c_uint32), ("interval", ctypes.c_uint32),
                ("tile_rows", ctypes.c_uint32), ("ksplit", ctypes.c_uint32), ("epilogue", ctypes.c_uint32),
                ("tile_cols", ctypes.c_uint32)]


class _GemmDesc(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("m", ctypes.c_uint32), ("n", ctypes.c_uint32), ("kdim", ctypes.c_uint32),
                ("lda", ctypes.c_uint32), ("ldb", ctypes.c_uint32), ("ldc", ctypes.c_uint32),
                ("p", ctypes.c_uint32), ("algo", ctypes.c_uint32), ("interval", ctypes.c_uint32),
                ("log2Q", ctypes.c_uint32), ("epilogue", ctypes.c_uint32)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_uint32), ("ksplit", ctypes.c_uint32), ("tile_cols", ctypes.c_uint32)]


@dataclass(frozen=True)
class Qadic:
    """q-adic packing parameters (p, q = 2^log2q, k coefficients, nres digits, n accumulated products,
    word width beta; 0 = 53)."""
    p: int
    log2q: int
    k_coeffs: int
    nres: int
    n_accum: int = 1
    word_bits: int = 0

    def _c(self) -> _Qadic:
        return _Qadic(self.p, self.log2q, self.k_coeffs, self.nres, self.n_accum, self.word_bits)


@dataclass(frozen=True)
class GemmPlan:
    algo: int = GEMM_AUTO
    log2Q: int = 0
    interval: int = 0
    tile_rows: int = 0
    ksplit: int = 0
    epilogue: int = EPI_REDC
    tile_cols: int = 0

    def _c(self) -> _GemmPlan:
        return _GemmPlan(self.algo, self.log2Q, self.interval, self.tile_rows, self.ksplit, self.epilogue,
                         self.tile_cols)


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdqt.so not found at {LIB_PATH}; build it with "
                          f"`python -m paper_0809_0063_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    V, U32, U64, I, SZ = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
    QP = ctypes.POINTER(_Qadic)
    sigs = {
        "dqt_qadic_check": [QP],
        "dqt_qadic_choose": [U32, U32, U64, U32, QP],
        "dqt_debug_enable": [V],
        "dqt_sync_status": [V],
        "dqt_pack": [V, U64, QP, I, V, V],
        "dqt_polymul": [V, V, U64, QP, V, V],
        "redq_unpack": [V, U64, QP, V, V, V],
        "dqt_polymul_u8": [V, V, U64, U32, U32, U32, V, V],
        "dqt_gf_mul_u8": [V, V, U64, U32, U32, U32, V, V, V],
        "dqt_polymul_plain_u8": [V, V, U64, U32, U32, V, V],
        "dqt_gf_mul_plain_u8": [V, V, U64, U32, U32, V, V, V],
        "dqt_gf_dot_u8": [V, V, U64, U32, U32, U32, V, V, V],
        "dqt_polymul_fqt_u8": [V, U32, V, U32, U64, U32, U32, V, V],
        "dqt_polymul_fqt_kara_u8": [V, U32, V, U32, U64, U32, U32, U32, V, V],
        "dqt_polymul_kara_long_u8": [V, V, U64, U32, U32, U32, V, V, SZ, V],
        "dqt_gf_matmul_u8": [V, V, U64, U64, U64, U32, U32, V, V, V],
        "dqt_check_input_u8": [V, U64, U32, V, V],
        "dqt_fgemm": [U32, U64, U64, U64, V, U64, V, U64, V, U64, ctypes.POINTER(_GemmPlan), V, SZ, V],
        "dqt_fgemm_batched": [ctypes.POINTER(_GemmDesc), U32, ctypes.POINTER(_BatchOpts), V, SZ, V],
        "dqt_fgemm_batched_prepare": [ctypes.POINTER(_GemmDesc), U32, ctypes.POINTER(_BatchOpts), V, SZ, V,
                                      ctypes.POINTER(ctypes.c_void_p)],
        "dqt_fgemm_batched_run": [V, V],
        "dqt_fgemm_batched_pack": [V, V],
        "dqt_fgemm_batched_compute": [V, V],
        "dqt_fgemm_pack": [U32, U64, U64, U64, V, U64, V, U64, ctypes.POINTER(_GemmPlan), V, SZ, V],
        "dqt_fgemm_compute": [U32, U64, U64, U64, V, U64, ctypes.POINTER(_GemmPlan), V, SZ, V],
        "dqt_fgemm_compute_timed": [U32, U64, U64, U64, V, U64, ctypes.POINTER(_GemmPlan), V, SZ, V, V, V],
        "dqt_fgemm_timed": [U32, U64, U64, U64, V, U64, V, U64, V, U64, ctypes.POINTER(_GemmPlan), V, SZ, V, V, V],
        "dqt_fgemm_pack_side": [U32, U64, U64, V, U64, I, ctypes.POINTER(_GemmPlan), V, V],
        "dqt_fgemm_packed": [U32, U64, U64, U64, V, V, V, U64, ctypes.POINTER(_GemmPlan), V],
        "dqt_fgemm_noalloc": [U32, U64, U64, U64, V, U64, V, U64, V, U64, ctypes.POINTER(_GemmPlan), V],
    }
    for name, args in sigs.items():
        if not hasattr(lib, name):
            continue  # reported by the ABI export test
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    if hasattr(lib, "dqt_fgemm_workspace_size"):
        lib.dqt_fgemm_workspace_size.argtypes = [U32, U64, U64, U64, ctypes.POINTER(_GemmPlan)]
        lib.dqt_fgemm_workspace_size.restype = SZ
    if hasattr(lib, "dqt_fgemm_batched_workspace_size"):
        lib.dqt_fgemm_batched_workspace_size.argtypes = [ctypes.POINTER(_GemmDesc), U32, ctypes.POINTER(_BatchOpts)]
        lib.dqt_fgemm_batched_workspace_size.restype = SZ
    if hasattr(lib, "dqt_fgemm_packed_bytes"):
        lib.dqt_fgemm_packed_bytes.argtypes = [U32, U64, U64, I, ctypes.POINTER(_GemmPlan)]
        lib.dqt_fgemm_packed_bytes.restype = SZ
    if hasattr(lib, "dqt_polymul_kara_long_workspace"):
        lib.dqt_polymul_kara_long_workspace.argtypes = [U64, U32, U32]
        lib.dqt_polymul_kara_long_workspace.restype = SZ
    if hasattr(lib, "dqt_fgemm_noalloc_max_bytes"):
        lib.dqt_fgemm_noalloc_max_bytes.argtypes = []
        lib.dqt_fgemm_noalloc_max_bytes.restype = SZ
    if hasattr(lib, "dqt_set_table_window"):
        lib.dqt_set_table_window.argtypes = [U32]
        lib.dqt_set_table_window.restype = ctypes.c_int
        lib.dqt_get_table_window.argtypes = []
        lib.dqt_get_table_window.restype = U32
    if hasattr(lib, "dqt_batch_free"):
        lib.dqt_batch_free.argtypes = [V]
        lib.dqt_batch_free.restype = None
    for name in ("dqt_status_str",):
        getattr(lib, name).argtypes = [ctypes.c_int]
        getattr(lib, name).restype = ctypes.c_char_p
    lib.dqt_last_error.argtypes = []
    lib.dqt_last_error.restype = ctypes.c_char_p
    lib.dqt_version.argtypes = []
    lib.dqt_version.restype = ctypes.c_char_p
    _lib = lib
    if DEBUG:
        debug_enable(True)
    return lib


def lib():
    """The loaded ctypes library (raises ImportError if it was not built)."""
    return _load()


def _status_str(s: int) -> str:
    try:
        return _load().dqt_status_str(s).decode()
    except Exception:
        return "status"


def _check(status: int, where: str):
    if status != DQT_OK:
        detail = _load().dqt_last_error().decode() if status in (DQT_E_DEVICE, DQT_E_INPUT) else ""
        raise DQTError(status, where, detail)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def set_table_window(j: int) -> None:
    """REDQ correction-table window for the calls that follow (0 auto, 1 none, 2, 3)."""
    _check(_load().dqt_set_table_window(j), "dqt_set_table_window")


def get_table_window() -> int:
    return int(_load().dqt_get_table_window())


_FLAG = {}


def check_input(t: torch.Tensor, p: int, stream=None) -> None:
    """Raise DQTError(DQT_E_INPUT) if some entry of the uint8 device tensor t is >= p (blocking)."""
    dev = t.device
    if dev not in _FLAG:
        _FLAG[dev] = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(_load().dqt_check_input_u8(_dev(t, "input", torch.uint8), t.numel(), p, _dev(_FLAG[dev], "flag"),
                                      _stream(stream)), "dqt_check_input_u8")


_STATUS = {}


def debug_enable(on: bool = True, device=None) -> None:
    """Turn the library's debug mode on (with a device status word on `device`) or off."""
    if not on:
        _check(_load().dqt_debug_enable(None), "dqt_debug_enable")
        return
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if dev not in _STATUS:
        _STATUS[dev] = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(_load().dqt_debug_enable(_dev(_STATUS[dev], "status")), "dqt_debug_enable")


def sync_status(stream=None) -> None:
    """dqt_sync_status: wait for the stream; raise DQTError(DQT_E_INPUT) if a debug check failed."""
    _check(_load().dqt_sync_status(_stream(stream)), "dqt_sync_status")


def _host_modulus(modulus: Sequence[int]):
    arr = (ctypes.c_uint8 * len(modulus))(*[int(x) for x in modulus])
    return arr


def version() -> str:
    return _load().dqt_version().decode()


# --- parameters --------------------------------------------------------------

def qadic_check(q: Qadic) -> int:
    """Status of dqt_qadic_check (0 = the parameters satisfy eq:bounds with beta = 53)."""
    c = q._c()
    return _load().dqt_qadic_check(ctypes.byref(c))


def qadic_choose(p: int, k_coeffs: int, n_accum: int = 1, word_bits: int = 0) -> Qadic:
    c = _Qadic()
    _check(_load().dqt_qadic_choose(p, k_coeffs, n_accum, word_bits, ctypes.byref(c)), "dqt_qadic_choose")
    return Qadic(c.p, c.log2q, c.k_coeffs, c.nres, c.n_accum, c.word_bits)


# --- one-word path -------------------------------------------------------------

def pack(coeffs: torch.Tensor, q: Qadic, reverse: bool = False, out: Optional[torch.Tensor] = None, stream=None):
    """DQT words (int64 bit patterns) of coeffs uint8 [N, k]."""
    n = coeffs.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=coeffs.device)
    c = q._c()
    _check(_load().dqt_pack(_dev(coeffs, "coeffs", torch.uint8), n, ctypes.byref(c), int(reverse),
                            _dev(out, "out", torch.int64), _stream(stream)), "dqt_pack")
    return out


def polymul_words(a: torch.Tensor, b: torch.Tensor, q: Qadic, out: Optional[torch.Tensor] = None, stream=None):
    n = a.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=a.device)
    c = q._c()
    _check(_load().dqt_polymul(_dev(a, "a", torch.int64), _dev(b, "b", torch.int64), n, ctypes.byref(c),
                               _dev(out, "out", torch.int64), _stream(stream)), "dqt_polymul")
    return out


def redq_unpack(r: torch.Tensor, q: Qadic, modulus: Optional[Sequence[int]] = None,
                out: Optional[torch.Tensor] = None, stream=None):
    """REDQ of packed words r (int64 [N]) -> uint8 [N, nres] (or [N, k] with a GF modulus)."""
    n = r.shape[0]
    width = q.nres if modulus is None else q.k_coeffs
    if out is None:
        out = torch.empty((n, width), dtype=torch.uint8, device=r.device)
    c = q._c()
    mod = _host_modulus(modulus) if modulus is not None else None
    _check(_load().redq_unpack(_dev(r, "r", torch.int64), n, ctypes.byref(c),
                               ctypes.cast(mod, ctypes.c_void_p) if mod is not None else None,
                               _dev(out, "out", torch.uint8), _stream(stream)), "redq_unpack")
    return out


def _u8_pair(a, b):
    if a.dim() != 2 or b.dim() != 2 or a.shape[0] != b.shape[0]:
        raise ValueError("a and b must be [N, k] with the same N")


def polymul_u8(a: torch.Tensor, b: torch.Tensor, p: int, out: Optional[torch.Tensor] = None, stream=None,
               log2q: int = 0):
    """Packed fused product: uint8 [N, k] x uint8 [N, k] -> uint8 [N, 2k-1] over F_p (q = 2^log2q, 0 = smallest)."""
    _u8_pair(a, b)
    n, k = a.shape
    if b.shape[1] != k:
        raise ValueError("a and b must have the same k")
    if out is None:
        out = torch.empty((n, 2 * k - 1), dtype=torch.uint8, device=a.device)
    _check(_load().dqt_polymul_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), n, k, p, log2q,
                                  _dev(out, "out", torch.uint8), _stream(stream)), "dqt_polymul_u8")
    return out


def polymul_plain_u8(a: torch.Tensor, b: torch.Tensor, p: int, out: Optional[torch.Tensor] = None, stream=None):
    _u8_pair(a, b)
    n, k = a.shape
    if out is None:
        out = torch.empty((n, 2 * k - 1), dtype=torch.uint8, device=a.device)
    _check(_load().dqt_polymul_plain_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), n, k, p,
                                        _dev(out, "out", torch.uint8), _stream(stream)), "dqt_polymul_plain_u8")
    return out


def polymul_fqt_u8(a: torch.Tensor, b: torch.Tensor, p: int, block: int = 0, out: Optional[torch.Tensor] = None,
                   stream=None):
    """Long products by blocks (FQT): uint8 [N, na] x uint8 [N, nb] -> uint8 [N, na+nb-1]."""
    _u8_pair(a, b)
    n, na = a.shape
    nb = b.shape[1]
    if out is None:
        out = torch.empty((n, na + nb - 1), dtype=torch.uint8, device=a.device)
    _check(_load().dqt_polymul_fqt_u8(_dev(a, "a", torch.uint8), na, _dev(b, "b", torch.uint8), nb, n, p, block,
                                      _dev(out, "out", torch.uint8), _stream(stream)), "dqt_polymul_fqt_u8")
    return out


def polymul_fqt_kara_u8(a: torch.Tensor, b: torch.Tensor, p: int, levels: int = 1, block: int = 0,
                        out: Optional[torch.Tensor] = None, stream=None):
    """FQT products with Karatsuba block products (levels 1 or 2): same shapes and bytes as polymul_fqt_u8."""
    _u8_pair(a, b)
    n, na = a.shape
    nb = b.shape[1]
    if out is None:
        out = torch.empty((n, na + nb - 1), dtype=torch.uint8, device=a.device)
    _check(_load().dqt_polymul_fqt_kara_u8(_dev(a, "a", torch.uint8), na, _dev(b, "b", torch.uint8), nb, n, p, block,
                                           levels, _dev(out, "out", torch.uint8), _stream(stream)),
           "dqt_polymul_fqt_kara_u8")
    return out


def kara_long_workspace(count: int, n: int, levels: int) -> int:
    """Workspace bytes dqt_polymul_kara_long_u8 needs (0 for invalid arguments)."""
    return int(_load().dqt_polymul_kara_long_workspace(count, n, levels))


def polymul_kara_long_u8(a: torch.Tensor, b: torch.Tensor, p: int, levels: int = 1,
                         out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None, stream=None):
    """Products of equal-length polynomials by `levels` Karatsuba levels over F_p with FQT base products."""
    _u8_pair(a, b)
    count, n = a.shape
    if b.shape[1] != n:
        raise ValueError(f"polymul_kara_long_u8 takes equal lengths, got {n} and {b.shape[1]}")
    if out is None:
        out = torch.empty((count, 2 * n - 1), dtype=torch.uint8, device=a.device)
    need = kara_long_workspace(count, n, levels)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=a.device)
    _check(_load().dqt_polymul_kara_long_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), count, n, p,
                                            levels, _dev(out, "out", torch.uint8), _dev(work, "work", torch.uint8),
                                            work.numel(), _stream(stream)),
           "dqt_polymul_kara_long_u8")
    return out


def gf_mul_u8(a: torch.Tensor, b: torch.Tensor, p: int, modulus: Sequence[int],
              out: Optional[torch.Tensor] = None, stream=None, log2q: int = 0):
    """Packed GF(p^k) products: uint8 [N, k] each, modulus = k+1 monic coefficients (low first)."""
    _u8_pair(a, b)
    n, k = a.shape
    if out is None:
        out = torch.empty((n, k), dtype=torch.uint8, device=a.device)
    mod = _host_modulus(modulus)
    _check(_load().dqt_gf_mul_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), n, k, p, log2q,
                                 ctypes.cast(mod, ctypes.c_void_p), _dev(out, "out", torch.uint8), _stream(stream)),
           "dqt_gf_mul_u8")
    return out


def gf_matmul_u8(a: torch.Tensor, b: torch.Tensor, p: int, modulus: Sequence[int],
                 out: Optional[torch.Tensor] = None, stream=None):
    """Matrix products over GF(p^k) by FGDP: uint8 [m, kd, k] x uint8 [kd, n, k] -> uint8 [m, n, k]."""
    if a.dim() != 3 or b.dim() != 3 or a.shape[1] != b.shape[0] or a.shape[2] != b.shape[2]:
        raise ValueError("a must be [m, kd, k] and b [kd, n, k]")
    m, kd, k = a.shape
    n = b.shape[1]
    if out is None:
        out = torch.empty((m, n, k), dtype=torch.uint8, device=a.device)
    mod = _host_modulus(modulus)
    _check(_load().dqt_gf_matmul_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), m, n, kd, k, p,
                                    ctypes.cast(mod, ctypes.c_void_p), _dev(out, "out", torch.uint8), _stream(stream)),
           "dqt_gf_matmul_u8")
    return out


def gf_dot_u8(a: torch.Tensor, b: torch.Tensor, p: int, modulus: Sequence[int],
              out: Optional[torch.Tensor] = None, stream=None):
    """Dot products over GF(p^k) by FGDP: uint8 [N, n, k] x uint8 [N, n, k] -> uint8 [N, k]."""
    if a.dim() != 3 or a.shape != b.shape:
        raise ValueError("a and b must be [N, n, k] with the same shape")
    N, n, k = a.shape
    if out is None:
        out = torch.empty((N, k), dtype=torch.uint8, device=a.device)
    mod = _host_modulus(modulus)
    _check(_load().dqt_gf_dot_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), N, n, k, p,
                                 ctypes.cast(mod, ctypes.c_void_p), _dev(out, "out", torch.uint8), _stream(stream)),
           "dqt_gf_dot_u8")
    return out


def gf_mul_plain_u8(a: torch.Tensor, b: torch.Tensor, p: int, modulus: Sequence[int],
                    out: Optional[torch.Tensor] = None, stream=None):
    _u8_pair(a, b)
    n, k = a.shape
    if out is None:
        out = torch.empty((n, k), dtype=torch.uint8, device=a.device)
    mod = _host_modulus(modulus)
    _check(_load().dqt_gf_mul_plain_u8(_dev(a, "a", torch.uint8), _dev(b, "b", torch.uint8), n, k, p,
                                       ctypes.cast(mod, ctypes.c_void_p), _dev(out, "out", torch.uint8),
                                       _stream(stream)), "dqt_gf_mul_plain_u8")
    return out


# --- matrix products -----------------------------------------------------------

def fgemm_workspace_size(p: int, m: int, n: int, kdim: int, plan: Optional[GemmPlan] = None) -> int:
    pc = plan._c() if plan is not None else None
    return int(_load().dqt_fgemm_workspace_size(p, m, n, kdim, ctypes.byref(pc) if pc is not None else None))


def fgemm(A: torch.Tensor, B: torch.Tensor, p: int, plan: Optional[GemmPlan] = None,
          out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None, stream=None):
    """C = A.B mod p for uint8 A [m, k], B [k, n] (row-major, contiguous)."""
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("A [m,k] and B [k,n] required")
    m, kdim = A.shape
    n = B.shape[1]
    if out is None:
        out = torch.empty((m, n), dtype=torch.uint8, device=A.device)
    ws = fgemm_workspace_size(p, m, n, kdim, plan)
    if ws and (workspace is None or workspace.numel() * workspace.element_size() < ws):
        workspace = torch.empty(ws, dtype=torch.uint8, device=A.device)
    pc = plan._c() if plan is not None else None
    wptr = _dev(workspace, "workspace") if ws else None
    wbytes = workspace.numel() * workspace.element_size() if ws else 0
    _check(_load().dqt_fgemm(p, m, n, kdim, _dev(A, "A", torch.uint8), kdim, _dev(B, "B", torch.uint8), n,
                             _dev(out, "C", torch.uint8), n, ctypes.byref(pc) if pc is not None else None,
                             wptr, wbytes, _stream(stream)), "dqt_fgemm")
    return out


def fgemm_noalloc(A: torch.Tensor, B: torch.Tensor, p: int, out: torch.Tensor, plan: Optional[GemmPlan] = None,
                  stream=None):
    """dqt_fgemm_noalloc: C = A.B mod p into the caller's `out`, packed operands in the library's
    static device array (no workspace, no allocation)."""
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("A [m,k] and B [k,n] required")
    m, kdim = A.shape
    n = B.shape[1]
    if tuple(out.shape) != (m, n):
        raise ValueError("out must be [m, n]")
    pc = plan._c() if plan is not None else None
    _check(_load().dqt_fgemm_noalloc(p, m, n, kdim, _dev(A, "A", torch.uint8), kdim, _dev(B, "B", torch.uint8), n,
                                     _dev(out, "C", torch.uint8), n, ctypes.byref(pc) if pc is not None else None,
                                     _stream(stream)), "dqt_fgemm_noalloc")
    return out


def fgemm_pack(A: Optional[torch.Tensor], B: Optional[torch.Tensor], p: int, plan: Optional[GemmPlan] = None,
               workspace: Optional[torch.Tensor] = None, shape=None, stream=None):
    """Packing phase of fgemm into `workspace` (A or B may be None to keep a packed copy)."""
    if shape is None:
        m, kdim = A.shape
        n = B.shape[1]
    else:
        m, n, kdim = shape
    pc = plan._c() if plan is not None else None
    _check(_load().dqt_fgemm_pack(p, m, n, kdim, _dev(A, "A", torch.uint8) if A is not None else None, kdim,
                                  _dev(B, "B", torch.uint8) if B is not None else None, n,
                                  ctypes.byref(pc) if pc is not None else None, _dev(workspace, "workspace"),
                                  workspace.numel() * workspace.element_size(), _stream(stream)), "dqt_fgemm_pack")


def fgemm_compute(C: torch.Tensor, p: int, kdim: int, plan: Optional[GemmPlan] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None):
    """Multiplication phase of fgemm on the packed operands in `workspace`; writes C [m, n]."""
    m, n = C.shape
    pc = plan._c() if plan is not None else None
    _check(_load().dqt_fgemm_compute(p, m, n, kdim, _dev(C, "C", torch.uint8), n,
                                     ctypes.byref(pc) if pc is not None else None, _dev(workspace, "workspace"),
                                     workspace.numel() * workspace.element_size(), _stream(stream)),
           "dqt_fgemm_compute")
    return C


def fgemm_compute_timed(C: torch.Tensor, p: int, kdim: int, start, stop, plan: Optional[GemmPlan] = None,
                        workspace: Optional[torch.Tensor] = None, stream=None):
    """fgemm_compute whose multiply kernel records its own start/end into torch.cuda.Event start/stop."""
    m, n = C.shape
    pc = plan._c() if plan is not None else None
    _check(_load().dqt_fgemm_compute_timed(p, m, n, kdim, _dev(C, "C", torch.uint8), n,
                                           ctypes.byref(pc) if pc is not None else None,
                                           _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                                           ctypes.c_void_p(start.cuda_event), ctypes.c_void_p(stop.cuda_event),
                                           _stream(stream)), "dqt_fgemm_compute_timed")
    return C


def fgemm_packed_bytes(p: int, rows_or_cols: int, kdim: int, side: int, plan: Optional[GemmPlan] = None) -> int:
    """Bytes of one packed operand (side 0: the m rows of A; side 1: the n columns of B)."""
    pc = plan._c() if plan is not None else None
    return int(_load().dqt_fgemm_packed_bytes(p, rows_or_cols, kdim, side, ctypes.byref(pc) if pc is not None else None))


def fgemm_pack_side(X: torch.Tensor, p: int, side: int, plan: Optional[GemmPlan] = None,
                    out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Packed copy of A [m, k] (side 0) or B [k, n] (side 1) in a buffer of its own (uint8 tensor)."""
    if X.dim() != 2:
        raise ValueError("a matrix is required")
    rows_or_cols, kdim = (X.shape[0], X.shape[1]) if side == 0 else (X.shape[1], X.shape[0])
    if kdim == 0 or rows_or_cols == 0:
        return torch.empty(0, dtype=torch.uint8, device=X.device) if out is None else out
    nb = fgemm_packed_bytes(p, rows_or_cols, kdim, side, plan)
    if nb == 0:
        raise DQTError(DQT_E_UNSUPPORTED, "dqt_fgemm_packed_bytes", "no packed layout for these arguments")
    if out is None:
        out = torch.empty(nb, dtype=torch.uint8, device=X.device)
    elif out.numel() * out.element_size() < nb:
        raise ValueError("packed buffer too small")
    pc = plan._c() if plan is not None else None
    _check(_load().dqt_fgemm_pack_side(p, rows_or_cols, kdim, _dev(X, "X", torch.uint8), X.shape[1], side,
                                       ctypes.byref(pc) if pc is not None else None, _dev(out, "packed"),
                                       _stream(stream)), "dqt_fgemm_pack_side")
    return out


def fgemm_packed(CA: torch.Tensor, CB: torch.Tensor, p: int, m: int, n: int, kdim: int,
                 plan: Optional[GemmPlan] = None, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """C = A.B mod p from a packed A (m rows) and a packed B (n columns) made by fgemm_pack_side."""
    if out is None:
        out = torch.empty((m, n), dtype=torch.uint8, device=CA.device)
    if tuple(out.shape) != (m, n):
        raise ValueError("C must be [m, n]")
    pc = plan._c() if plan is not None else None
    _check(_load().dqt_fgemm_packed(p, m, n, kdim, _dev(CA, "CA"), _dev(CB, "CB"), _dev(out, "C", torch.uint8),
                                    out.stride(0), ctypes.byref(pc) if pc is not None else None, _stream(stream)),
           "dqt_fgemm_packed")
    return out


class FgemmCall:
    """One F_p product with its arguments marshalled once, for repeated launches.

    pack() and compute() / compute_timed() enqueue the same two phases as
    fgemm on the stream given at construction; the operands, output and
    workspace must stay alive and unchanged in shape while the object is used.
    """

    def __init__(self, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, p: int, plan: Optional[GemmPlan] = None,
                 workspace: Optional[torch.Tensor] = None, stream=None):
        m, kdim = A.shape
        n = B.shape[1]
        if B.shape[0] != kdim or tuple(C.shape) != (m, n):
            raise ValueError("shapes do not match")
        ws = fgemm_workspace_size(p, m, n, kdim, plan)
        if ws and (workspace is None or workspace.numel() * workspace.element_size() < ws):
            workspace = torch.empty(ws, dtype=torch.uint8, device=A.device)
        self._keep = (A, B, C, workspace)
        self._pc = plan._c() if plan is not None else None
        pcp = ctypes.byref(self._pc) if self._pc is not None else None
        wptr = _dev(workspace, "workspace") if ws else None
        wbytes = workspace.numel() * workspace.element_size() if ws else 0
        st = _stream(stream)
        self._lib = _load()
        self._pack_args = (p, m, n, kdim, _dev(A, "A", torch.uint8), kdim, _dev(B, "B", torch.uint8), n, pcp,
                           wptr, wbytes, st)
        self._comp_args = (p, m, n, kdim, _dev(C, "C", torch.uint8), n, pcp, wptr, wbytes)
        self._full_args = (p, m, n, kdim, _dev(A, "A", torch.uint8), kdim, _dev(B, "B", torch.uint8), n,
                           _dev(C, "C", torch.uint8), n, pcp, wptr, wbytes, st)
        self._st = st

    def run(self):
        """Both phases in one call (dqt_fgemm)."""
        _check(self._lib.dqt_fgemm(*self._full_args), "dqt_fgemm")

    def run_timed(self, start, stop):
        """Both phases in one call, the multiply kernel recording its own start and end (dqt_fgemm_timed)."""
        _check(self._lib.dqt_fgemm_timed(*self._full_args[:-1], ctypes.c_void_p(start.cuda_event),
                                         ctypes.c_void_p(stop.cuda_event), self._st), "dqt_fgemm_timed")

    def pack(self):
        _check(self._lib.dqt_fgemm_pack(*self._pack_args), "dqt_fgemm_pack")

    def compute(self):
        _check(self._lib.dqt_fgemm_compute(*self._comp_args, self._st), "dqt_fgemm_compute")

    def compute_timed(self, start, stop):
        _check(self._lib.dqt_fgemm_compute_timed(*self._comp_args, ctypes.c_void_p(start.cuda_event),
                                                 ctypes.c_void_p(stop.cuda_event), self._st),
               "dqt_fgemm_compute_timed")


def make_descs(items):
    """ctypes descriptor array from dicts (or tuples) describing each product.

    Each item: (A, B, C, p) or (A, B, C, p, algo) or a dict with keys A, B, C, p
    and optional algo, interval, log2Q, epilogue.  A [m, k], B [k, n], C [m, n]
    are contiguous uint8 device tensors.
    """
    arr = (_GemmDesc * len(items))()
    for i, it in enumerate(items):
        if isinstance(it, dict):
            A, B, C, p = it["A"], it["B"], it["C"], it["p"]
            algo, interval, log2Q, epi = it.get("algo", 0), it.get("interval", 0), it.get("log2Q", 0), it.get("epilogue", 0)
        else:
            A, B, C, p = it[:4]
            algo = it[4] if len(it) > 4 else 0
            interval = log2Q = epi = 0
        m, kdim = A.shape
        n = B.shape[1]
        if B.shape[0] != kdim or tuple(C.shape) != (m, n):
            raise ValueError("descriptor shapes do not match")
        for t in (A, B, C):
            _dev(t, "operand", torch.uint8)
        arr[i] = _GemmDesc(A.data_ptr(), B.data_ptr(), C.data_ptr(), m, n, kdim, kdim, n, n, p, algo, interval,
                           log2Q, epi)
    return arr


def _opts(tile_rows: int, ksplit: int, tile_cols: int = 0) -> _BatchOpts:
    return _BatchOpts(tile_rows, ksplit, tile_cols)


def fgemm_batched_workspace_size(descs, tile_rows: int = 0, ksplit: int = 0, tile_cols: int = 0) -> int:
    o = _opts(tile_rows, ksplit, tile_cols)
    return int(_load().dqt_fgemm_batched_workspace_size(descs, len(descs), ctypes.byref(o)))


class Batch:
    """A prepared batch (device-resident plan in `workspace`); run() enqueues pack + persistent compute."""

    def __init__(self, descs, workspace: torch.Tensor, tile_rows: int = 0, ksplit: int = 0, tile_cols: int = 0,
                 stream=None):
        self._descs = descs
        self.workspace = workspace
        self._handle = ctypes.c_void_p()
        o = _opts(tile_rows, ksplit, tile_cols)
        _check(_load().dqt_fgemm_batched_prepare(descs, len(descs), ctypes.byref(o), _dev(workspace, "workspace"),
                                                 workspace.numel() * workspace.element_size(), _stream(stream),
                                                 ctypes.byref(self._handle)), "dqt_fgemm_batched_prepare")

    def run(self, stream=None):
        _check(_load().dqt_fgemm_batched_run(self._handle, _stream(stream)), "dqt_fgemm_batched_run")

    def pack(self, stream=None):
        """Only the packing launch: the packed copies of every operand in the workspace."""
        _check(_load().dqt_fgemm_batched_pack(self._handle, _stream(stream)), "dqt_fgemm_batched_pack")

    def compute(self, stream=None):
        """Only the persistent launch, on the packed copies left by the last run() or pack()."""
        _check(_load().dqt_fgemm_batched_compute(self._handle, _stream(stream)), "dqt_fgemm_batched_compute")

    def close(self):
        if self._handle:
            _load().dqt_batch_free(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fgemm_batched(descs, workspace: torch.Tensor, tile_rows: int = 0, ksplit: int = 0, tile_cols: int = 0,
                  stream=None):
    """Run every descriptor (from make_descs) in one packing launch and one persistent launch."""
    o = _opts(tile_rows, ksplit, tile_cols)
    ws = fgemm_batched_workspace_size(descs, tile_rows, ksplit, tile_cols)
    if workspace.numel() * workspace.element_size() < ws:
        raise ValueError(f"workspace needs {ws} bytes")
    _check(_load().dqt_fgemm_batched(descs, len(descs), ctypes.byref(o), _dev(workspace, "workspace"),
                                     workspace.numel() * workspace.element_size(), _stream(stream)),
           "dqt_fgemm_batched")
