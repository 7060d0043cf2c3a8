"""Benchmark of the packed DQT + REDQ hot path on one MI355X.

Workload (one step): C = A.B mod 3 with m = n = k = 1024, uniform uint8 entries
in [0, 3): DQT packing of the rows of A and the columns of B (reversed
Kronecker pairs, four entries per 32-bit word), the packed multiply-accumulate
(middle product, delayed reduction, one v_dot2_u32_u16 per four F_p
multiply-adds), middle-digit extraction and one reduction per output, uint8
store.  Inputs are resident in HBM before the timed region.

Printed: one JSON line.  `value` is F_p Gop/s (2 m n k per step) of the
packed path; `roofline` is the packed multiply kernel against the VALU issue
rate; `cpu_baseline` is the CPU oracle on a bounded sample; `extra` holds the
other measured paths, by section (--sections): the plain per-entry, dot4, dot8,
INT8 matrix-core and FP64 matrix-core compressed products with their own
roofline fractions (gemm), one-word polynomial products against HBM, the
four-call composition and the small workload in graph replays (polymul),
long products by blocks (fqt), GF(p^k) products and dot products (gf), the
batched workload of 10,000 products and the serving loop at three loads
(workloads), and the CPU oracle on every workload (cpu).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "F_p GEMM Gop/s + polymul/s, packed DQT+REDQ vs plain modular; p99 latency"
PEAK_LANE_OPS = 256 * 64 * 2.4e9          # VALU lane-instructions per second (256 CUs, wave64, 2.4 GHz)
PEAK_HBM = 8.0e12                          # bytes per second
PEAK_INT8_MFMA = 5.0e15                    # dense INT8 matrix-core ops per second
PEAK_F64_FMA = 78.6e12 / 2                 # binary64 multiply-adds per second (78.6 TFLOP/s)
MNK = 1024
MIN_EVENT_SAMPLES = 8                      # kernel-timed steps in the timed region, at least
SECTIONS = ("gemm", "polymul", "fqt", "gf", "workloads", "cpu")


# HBM bytes per launch of the timed multiply kernel, from two rocprofv3 counter
# runs (FETCH_SIZE, WRITE_SIZE; the summary and its commands are in profiles/),
# valid only for the device code they were taken on: the tile and REDQ device
# headers and the kernel's definition, identified by their SHA-256.
TRAFFIC_SOURCES = ("paper_0809_0063_amd/csrc/dqt_gemm_tile.h", "paper_0809_0063_amd/csrc/dqt_device.h")
TRAFFIC_KERNEL = ("paper_0809_0063_amd/csrc/dqt_gemm.hip", "__device__ __forceinline__ void tile_of(",
                  "// Pack A (rows")
TRAFFIC = {"sha256": "754243f159153713bf45f7bbef26d13e548facff839856d52514705724516662", "bytes": 11725786}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    rel, begin, end = TRAFFIC_KERNEL
    with open(os.path.join(ROOT, rel)) as f:
        text = f.read()
    i = text.index(begin)
    h.update(text[i:text.index(end, i)].encode())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sections", default="", help="comma-separated subset of " + ",".join(SECTIONS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-extra", action="store_true", help="skip the comparator and other-path measurements")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the batched (10,000 products) and serving measurements")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device-to-device copy (reference kernel for counter scaling)")
    return ap.parse_args()


def hip_elapsed_ms(start, stop) -> float:
    """hipEventElapsedTime of two torch events recorded by the HIP runtime itself."""
    import ctypes
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so.7")
        _HIP.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _HIP.hipEventElapsedTime.restype = ctypes.c_int
    ms = ctypes.c_float()
    if not start.cuda_event or not stop.cuda_event:
        raise RuntimeError("event not created")
    st = _HIP.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(start.cuda_event), ctypes.c_void_p(stop.cuda_event))
    if st != 0:
        raise RuntimeError(f"hipEventElapsedTime failed ({st})")
    return ms.value


_HIP = None


_T0 = time.perf_counter()


def log(msg):
    """Progress on stderr (the result line alone goes to stdout)."""
    print(f"bench [{time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def timed_loop(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps   # seconds per call


def kernel_us(call, torch, reps):
    """Average duration of the multiply kernel of a prepared product (HIP events recorded by the launch)."""
    evs = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    for a, b in evs:
        call.pack()
        call.compute_timed(a, b)
    torch.cuda.synchronize()
    return sum(hip_elapsed_ms(a, b) for a, b in evs) / len(evs) * 1e3


def f64_digits(p, k):
    """Digits per binary64 word of the matrix-core compressed products (eq:lower, eq:upper with 52 bits)."""
    return 52 // max(1, (k * (p - 1) ** 2).bit_length())


def bench_gemm_comparators(D, torch, dA, dB, dC, p, row0, stream, reps):
    """Every F_p product of the 1024^3 workload: step (pack + multiply) and multiply kernel alone, with
    the kernel's fraction of the roofline of the unit it runs on."""
    n = MNK
    macs = float(n) ** 3
    e = f64_digits(p, n)
    cases = (
        ("cmm_redq_epilogue", D.GemmPlan(algo=D.GEMM_CMM, epilogue=D.EPI_REDQ), "alu", macs / 4),
        ("plain_mad", D.GemmPlan(algo=D.GEMM_PLAIN), "alu", macs),
        ("plain_dot4", D.GemmPlan(algo=D.GEMM_DOT4), "alu", macs / 4),
        ("plain_dot8", D.GemmPlan(algo=D.GEMM_DOT8), "alu", macs / 8),
        ("mfma_int8", D.GemmPlan(algo=D.GEMM_MFMA), "mfma_int8", 2 * macs),
        ("right_compressed_f64mfma", D.GemmPlan(algo=D.GEMM_RIGHT), "mfma_f64", macs / e),
        ("left_compressed_f64mfma", D.GemmPlan(algo=D.GEMM_LEFT), "mfma_f64", macs / e),
        ("full_compressed_f64mfma", D.GemmPlan(algo=D.GEMM_FULL), "mfma_f64", macs / e),
    )
    peak = {"alu": PEAK_LANE_OPS, "mfma_int8": PEAK_INT8_MFMA, "mfma_f64": PEAK_F64_FMA}
    unit = {"alu": "lane-instructions", "mfma_int8": "int8 ops", "mfma_f64": "binary64 FMAs"}
    out = {}
    for name, pl, bound, work in cases:
        w2 = torch.empty(max(1, D.fgemm_workspace_size(p, n, n, n, pl)), dtype=torch.uint8, device=dA.device)
        c2 = D.FgemmCall(dA, dB, dC, p, plan=pl, workspace=w2, stream=stream)
        s = timed_loop(c2.run, reps, 3, torch)
        assert (dC[:1].cpu().numpy() == row0).all(), name
        kus = kernel_us(c2, torch, max(8, reps // 4))
        out["fgemm_" + name] = {"gop_s": round(2 * macs / s / 1e9, 1), "us_per_step": round(s * 1e6, 2),
                                "kernel_us": round(kus, 3), "kernel_fp_top_s": round(2 * macs / kus / 1e6, 1),
                                "bound": bound, "work_per_launch": work, "work_unit": unit[bound],
                                "kernel_frac": round(work / (kus * 1e-6) / peak[bound], 4)}
    out.update(bench_library_int8(torch, p, n, dA.cpu().numpy(), dB.cpu().numpy()))
    out.update(bench_gemm_4096(D, torch, p, stream, peak, unit))
    return out


def bench_gemm_4096(D, torch, p, stream, peak, unit):
    """The multiply kernels at 4096^3 over F_3 (64 times the work of the headline product), where launch
    and start-up latency no longer dominate: kernel time and fraction of each kernel's own roofline."""
    import numpy as np
    from paper_0809_0063_amd import inputs
    n = 4096
    macs = float(n) ** 3
    A, B = inputs.gemm_pair(n, n, n, p, seed=inputs.SEED_FGEMM + 4096)
    dA, dB = torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda")
    dC = torch.empty((n, n), dtype=torch.uint8, device="cuda")
    row0 = (A[:1].astype(np.int64) @ B.astype(np.int64)) % p
    out = {}
    for name, pl, bound, work in (("packed_cmm", D.GemmPlan(algo=D.GEMM_CMM), "alu", macs / 4),
                                  ("plain_dot4", D.GemmPlan(algo=D.GEMM_DOT4), "alu", macs / 4),
                                  ("plain_dot8", D.GemmPlan(algo=D.GEMM_DOT8), "alu", macs / 8),
                                  ("mfma_int8", D.GemmPlan(algo=D.GEMM_MFMA), "mfma_int8", 2 * macs),
                                  ("right_compressed_f64mfma", D.GemmPlan(algo=D.GEMM_RIGHT), "mfma_f64",
                                   macs / f64_digits(p, n))):
        c2 = D.FgemmCall(dA, dB, dC, p, plan=pl, stream=stream)
        c2.run()
        torch.cuda.synchronize()
        assert (dC[:1].cpu().numpy() == row0).all(), name
        kus = kernel_us(c2, torch, 6)
        out["fgemm4096_" + name] = {"kernel_us": round(kus, 1), "kernel_fp_top_s": round(2 * macs / kus / 1e6, 1),
                                    "bound": bound, "work_per_launch": work, "work_unit": unit[bound],
                                    "kernel_frac": round(work / (kus * 1e-6) / peak[bound], 4)}
        del c2
    out.update(bench_library_int8(torch, p, 4096, A, B))
    return out


def bench_library_int8(torch, p, n, A, B):
    """The vendor library's int8 matrix product (torch._int_mm: int8 x int8 -> int32 on the matrix cores)
    followed by one reduction mod p per output: the machine's best dense routine as a plain comparator
    (section 7.3 compares with the machine's dgemm).  Not part of the library; timed with events around
    each call on the current stream."""
    import numpy as np
    out = {}
    try:
        dA = torch.from_numpy(A.astype(np.int8)).to("cuda")
        dB = torch.from_numpy(B.astype(np.int8)).to("cuda")
        row0 = (A[:1].astype(np.int64) @ B.astype(np.int64)) % p
        for _ in range(3):
            C32 = torch._int_mm(dA, dB)
        torch.cuda.synchronize()
        reps = 10
        e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in e:
            a.record()
            C32 = torch._int_mm(dA, dB)
            b.record()
        torch.cuda.synchronize()
        mm_s = sum(a.elapsed_time(b) for a, b in e) / reps / 1e3
        C = (C32 % p).to(torch.uint8)
        s = timed_loop(lambda: (torch._int_mm(dA, dB) % p).to(torch.uint8), reps, 2, torch)
        assert (C[:1].cpu().numpy() == row0).all()
        ops = 2.0 * n ** 3
        out[f"fgemm{n}_library_int8_mm"] = {"matmul_us": round(mm_s * 1e6, 1), "us_per_step_with_mod_p": round(s * 1e6, 1),
                                           "matmul_top_s": round(ops / mm_s / 1e12, 1),
                                           "matmul_frac": round(ops / mm_s / PEAK_INT8_MFMA, 4),
                                           "bound": "mfma_int8"}
    except Exception as ex:  # reported, not hidden
        out[f"fgemm{n}_library_int8_mm"] = {"error": f"{type(ex).__name__}: {ex}"}
    return out


def polymul_graph_replays(D, torch, dev, inputs, count, sets, replays):
    """One-word products on `sets` rotating buffer sets captured in one graph, replayed: time per launch."""
    bufs = []
    for i in range(sets):
        a, b = inputs.polymul_pairs(count, 4, 3, seed=inputs.SEED_POLYMUL + 100 + i)
        bufs.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev),
                     torch.empty((count, 7), dtype=torch.uint8, device=dev)))
    for a, b, o in bufs:      # outside capture first (device set-up)
        D.polymul_u8(a, b, 3, out=o, log2q=6)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for a, b, o in bufs:
                D.polymul_u8(a, b, 3, out=o, log2q=6)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / (replays * sets)


def ref_polymul_f3(a, b):
    """Products of a few degree-3 polynomials over F_3 by integer numpy (a spot check of timed output)."""
    import numpy as np
    out = np.zeros((a.shape[0], 7), dtype=np.int64)
    for i in range(4):
        for j in range(4):
            out[:, i + j] += a[:, i].astype(np.int64) * b[:, j]
    return out % 3


def bench_polymul(D, inputs, torch, dev, reps_big, reps_small):
    out = {}
    # one-word polynomial products: degree 3 over F_3, q = 2^6, 2^26 products (beyond the MALL)
    n = 1 << 26
    a, b = inputs.polymul_pairs(n, 4, 3)
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    o = torch.empty((n, 7), dtype=torch.uint8, device=dev)
    for name, fn in (("packed", lambda: D.polymul_u8(da, db, 3, out=o, log2q=6)),
                     ("plain", lambda: D.polymul_plain_u8(da, db, 3, out=o))):
        s = timed_loop(fn, reps_big, 2, torch)
        out["polymul_deg3_f3_" + name] = {"polymul_s": round(n / s, 1), "GB_s": round(15 * n / s / 1e9, 1),
                                          "hbm_frac": round(15 * n / s / PEAK_HBM, 4)}
    # the four-call composition (pack a, pack b, packed product, REDQ unpack) on the same products;
    # its own traffic is 4 + 8 bytes per pack (twice), 16 + 8 for the product, 8 + 7 for the unpack
    q = D.Qadic(3, 6, 4, 7, 1)
    wa = torch.empty(n, dtype=torch.int64, device=dev)
    wb = torch.empty(n, dtype=torch.int64, device=dev)
    wr = torch.empty(n, dtype=torch.int64, device=dev)

    def four():
        D.pack(da, q, out=wa)
        D.pack(db, q, out=wb)
        D.polymul_words(wa, wb, q, out=wr)
        D.redq_unpack(wr, q, out=o)
    s = timed_loop(four, reps_big, 2, torch)
    assert (o[:4].cpu().numpy() == ref_polymul_f3(a[:4], b[:4])).all()
    out["polymul_deg3_f3_four_calls"] = {"polymul_s": round(n / s, 1), "GB_s": round(63 * n / s / 1e9, 1),
                                         "hbm_frac": round(63 * n / s / PEAK_HBM, 4),
                                         "fused_bytes_GB_s": round(15 * n / s / 1e9, 1)}
    del wa, wb, wr
    # the correction-table window (section 3.5): none, two or three residues per lookup
    try:
        for j in (1, 2, 3):
            D.set_table_window(j)
            s = timed_loop(lambda: D.polymul_u8(da, db, 3, out=o, log2q=6), reps_big, 2, torch)
            out[f"polymul_deg3_f3_table_window_{j}"] = {"GB_s": round(15 * n / s / 1e9, 1),
                                                        "hbm_frac": round(15 * n / s / PEAK_HBM, 4)}
    finally:
        D.set_table_window(0)
    del da, db, o
    # the small workload itself: 65,536 products per launch, 8 rotating buffer sets in one graph
    s = polymul_graph_replays(D, torch, dev, inputs, 65536, 8, max(20, reps_small))
    out["polymul_65536_graph"] = {"us_per_launch": round(s * 1e6, 3), "polymul_s": round(65536 / s, 1),
                                  "GB_s": round(15 * 65536 / s / 1e9, 1), "buffer_sets": 8}
    return out


def bench_fqt(D, inputs, torch, dev, reps_big):
    out = {}
    # long products by blocks (FQT): degree 47 over F_3, 2^20 products, schoolbook and Karatsuba blocks
    nl = 1 << 20
    al, bl = inputs.polymul_pairs(nl, 48, 3)
    dal, dbl = torch.from_numpy(al).to(dev), torch.from_numpy(bl).to(dev)
    ol = torch.empty((nl, 95), dtype=torch.uint8, device=dev)
    for name, fn in (("fqt", lambda: D.polymul_fqt_u8(dal, dbl, 3, out=ol)),
                     ("fqt_karatsuba1", lambda: D.polymul_fqt_kara_u8(dal, dbl, 3, levels=1, out=ol)),
                     ("fqt_karatsuba2", lambda: D.polymul_fqt_kara_u8(dal, dbl, 3, levels=2, out=ol)),
                     ("plain", lambda: D.polymul_plain_u8(dal, dbl, 3, out=ol))):
        try:
            s = timed_loop(fn, reps_big, 2, torch)
            out["polymul_deg47_f3_" + name] = {"polymul_s": round(nl / s, 1), "us_per_call": round(s * 1e6, 1)}
        except D.DQTError as e:
            out["polymul_deg47_f3_" + name] = {"error": str(e)}
    del dal, dbl, ol
    out.update(bench_fqt_long(D, inputs, torch, dev))
    return out


def fqt_long_model(p, n, bs):
    """Operation counts of section 5.3's model for a product of two n-coefficient polynomials: block products
    and REDQ_{2bs-1} of a bs-block FQT (sums of at most n_q block products, q = 2^b, (2bs-1) b <= 51), against
    the n^2 coefficient products and 2n-1 reductions of the plain delayed product."""
    b = 51 // (2 * bs - 1)
    nq = ((1 << b) - 1) // (bs * (p - 1) ** 2)
    nb = -(-n // bs)
    nw = 2 * nb - 1
    reds = sum(-(-(min(u, nb - 1) - max(0, u - nb + 1) + 1) // nq) for u in range(nw))
    return {"block": bs, "q": 1 << b, "n_q": nq, "block_products": nb * nb, "redq": reds,
            "plain_products": n * n, "plain_reductions": 2 * n - 1,
            "model_op_ratio": round((n * n + 2 * n - 1) / (nb * nb + reds), 2)}


def bench_fqt_long(D, inputs, torch, dev):
    """Long products over F_3 (n = 65 .. 4096 coefficients, n = 500 the example of section 5.3): FQT by
    blocks, Karatsuba levels over FQT base products (from n = 500), and the plain per-coefficient
    product, same batch."""
    out = {}
    p = 3
    for n in (65, 96, 128, 192, 256, 384, 500, 1024, 2048, 4096):
        count = max(2048, (1 << 34) // (n * n))
        a, b = inputs.polymul_pairs(count, n, p, seed=inputs.SEED_POLYMUL + n)
        da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
        o = torch.empty((count, 2 * n - 1), dtype=torch.uint8, device=dev)
        row = {"count": count}
        blocks = (0, 2, 3, 4) if n in (500, 1024, 2048) else (0, 2, 3)
        for blk in blocks:
            s = timed_loop(lambda: D.polymul_fqt_u8(da, db, p, block=blk, out=o), 5, 2, torch)
            key = "fqt" if blk == 0 else f"fqt_block{blk}"
            row[key] = {"products_s": round(count / s, 1), "us_per_call": round(s * 1e6, 1),
                        "coeff_products_s": round(count * n * n / s, 1)}
            if blk:
                # block products (one binary64 FMA each) per second over the FP64 vector peak
                nblk = -(-n // blk)
                row[key]["fma_frac"] = round(count * nblk * nblk / s / PEAK_F64_FMA, 4)
        if n >= 500:
            # Karatsuba levels over F_p with FQT base products (workspace allocated once, outside the loop)
            for lv in ((1, 2) if n < 4096 else (1, 2, 3)):
                work = torch.empty(D.kara_long_workspace(count, n, lv), dtype=torch.uint8, device=dev)
                s = timed_loop(lambda: D.polymul_kara_long_u8(da, db, p, levels=lv, out=o, work=work), 5, 2, torch)
                row[f"kara{lv}"] = {"products_s": round(count / s, 1), "us_per_call": round(s * 1e6, 1)}
                del work
        s = timed_loop(lambda: D.polymul_plain_u8(da, db, p, out=o), 5, 2, torch)
        row["plain"] = {"products_s": round(count / s, 1), "us_per_call": round(s * 1e6, 1),
                        "lane_op_frac": round(count * n * n / s / PEAK_LANE_OPS, 4)}
        row["fqt_over_plain"] = round(row["fqt"]["products_s"] / row["plain"]["products_s"], 2)
        row["model"] = [fqt_long_model(p, n, bs) for bs in (2, 3, 4)]
        out[f"polymul_n{n}_f3_long"] = row
        del da, db, o
    return out


def bench_gf(D, inputs, torch, dev, reps_big):
    out = {}
    n = 1 << 26
    for (pp, k) in ((3, 5), (7, 3)):
        P = inputs.irreducible(pp, k)
        x, y = inputs.gf_pairs(n, k, pp)
        dx, dy = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        oz = torch.empty((n, k), dtype=torch.uint8, device=dev)
        for name, fn in (("packed", lambda: D.gf_mul_u8(dx, dy, pp, P, out=oz)),
                         ("plain", lambda: D.gf_mul_plain_u8(dx, dy, pp, P, out=oz))):
            s = timed_loop(fn, reps_big, 2, torch)
            out[f"gf_{pp}^{k}_{name}"] = {"mul_s": round(n / s, 1), "GB_s": round(3 * k * n / s / 1e9, 1),
                                         "hbm_frac": round(3 * k * n / s / PEAK_HBM, 4)}
        del dx, dy, oz
    # dot products over GF(3^5): 65,536 dot products of length 128 (2 n k + k bytes each)
    pp, k, cnt, ln = 3, 5, 65536, 128
    P = inputs.irreducible(pp, k)
    g = inputs.rng(inputs.SEED_GF + 99)
    xa = torch.from_numpy(g.integers(0, pp, size=(cnt, ln, k), dtype="uint8")).to(dev)
    xb = torch.from_numpy(g.integers(0, pp, size=(cnt, ln, k), dtype="uint8")).to(dev)
    od = torch.empty((cnt, k), dtype=torch.uint8, device=dev)
    s = timed_loop(lambda: D.gf_dot_u8(xa, xb, pp, P, out=od), max(4, reps_big), 2, torch)
    byts = cnt * (2 * ln * k + k)
    # q = 2^floor(53/9) = 2^5 admits n_q = floor(31 / (5 * 2^2)) = 1 product per packed word, so every
    # product has its own REDQ and two table lookups: the kernel is bound by instruction issue
    out["gf_3^5_dot_n128"] = {"dot_s": round(cnt / s, 1), "GB_s": round(byts / s / 1e9, 1),
                              "hbm_frac": round(byts / s / PEAK_HBM, 4), "us_per_call": round(s * 1e6, 1),
                              "n_q": 1, "bound": "valu"}
    # matrix product over GF(3^5): 512 x 512 x 512 field elements (FGDP dot products, n_q = 1)
    mm = 512
    xa = torch.from_numpy(g.integers(0, pp, size=(mm, mm, k), dtype="uint8")).to(dev)
    xb = torch.from_numpy(g.integers(0, pp, size=(mm, mm, k), dtype="uint8")).to(dev)
    om = torch.empty((mm, mm, k), dtype=torch.uint8, device=dev)
    s = timed_loop(lambda: D.gf_matmul_u8(xa, xb, pp, P, out=om), 4, 2, torch)
    out["gf_3^5_matmul_512"] = {"field_products_s": round(mm ** 3 / s, 1), "us_per_call": round(s * 1e6, 1),
                                "n_q": 1, "bound": "valu"}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baselines(A, B, p, row0, fp_ops, inputs):
    """The CPU oracle (reduce after every operation) on bounded samples of each workload, with one
    thread and with all cores.  Returns the headline entry (the 1024^3 product, all cores) and the table."""
    import oracle as O
    cores = O.max_threads()

    def rate(fn, work, min_s):
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_s:
                return reps * work / dt, reps, dt

    table = {"cpu_model": cpu_model(), "cores": cores}
    # the F_p product: the whole of it with all cores; 64 of its rows on one thread
    v_all, reps, dt = rate(lambda: O.fgemm(A, B, p), fp_ops, 6.0)
    assert (O.fgemm(A[:1], B, p) == row0).all()
    v_one, _, _ = rate(lambda: O.fgemm(A[:64], B, p, threads=1), 2.0 * 64 * MNK * MNK, 2.0)
    log("cpu: F_p product done")
    table["fgemm_1024_p3"] = {"unit": "Gop/s", "all_cores": round(v_all / 1e9, 3), "one_thread": round(v_one / 1e9, 3)}
    headline = {"value": round(v_all / 1e9, 3), "unit": "Gop/s", "cores": cores, "kind": "oracle",
                "sample": f"the whole 1024^3 mod-3 product, {reps} times ({dt:.1f} s), reduce after every op",
                "cpu_model": table["cpu_model"], "one_thread_value": round(v_one / 1e9, 3)}
    # 65,536 products of degree 3 over F_3
    a, b = inputs.polymul_pairs(65536, 4, 3)
    table["polymul_65536_deg3_f3"] = {
        "unit": "polymul/s", "all_cores": round(rate(lambda: O.polymul(a, b, 3), 65536, 1.0)[0], 1),
        "one_thread": round(rate(lambda: O.polymul(a, b, 3, threads=1), 65536, 1.0)[0], 1)}
    # GF(3^5) and GF(7^3) products (a 2^20 sample of the 2^24)
    for pp, k in ((3, 5), (7, 3)):
        P = inputs.irreducible(pp, k)
        x, y = inputs.gf_pairs(1 << 20, k, pp)
        table[f"gf_{pp}^{k}_mul"] = {
            "unit": "mul/s", "sample": "2^20 products",
            "all_cores": round(rate(lambda: O.gf_mul(x, y, pp, P), 1 << 20, 1.0)[0], 1),
            "one_thread": round(rate(lambda: O.gf_mul(x, y, pp, P, threads=1), 1 << 20, 1.0)[0], 1)}
    # the first 300 products of the batched workload
    items = inputs.batch_items(10000)[:100]
    ops = [inputs.item_operands(it) + (it.p,) for it in items]
    work = sum(2.0 * it.n ** 3 for it in items)
    work20 = sum(2.0 * it.n ** 3 for it in items[:20])

    def batch(th, count):
        for Ai, Bi, pi in ops[:count]:
            O.fgemm(Ai, Bi, pi, threads=th)
    table["batched_sample"] = {"unit": "Gop/s",
                               "sample": "all cores: the first 100 of the 10,000 products; one thread: the first 20",
                               "all_cores": round(rate(lambda: batch(0, 100), work, 1.0)[0] / 1e9, 3),
                               "one_thread": round(rate(lambda: batch(1, 20), work20, 1.0)[0] / 1e9, 3)}
    log("cpu: batched sample done")
    # the first 100 polynomial-product payloads of the serving pool (its products are like the above)
    pool = [pl for pl in inputs.serve_pool() if pl.kind == "polymul"][:100]
    pops = [inputs.payload_operands(pl) + (pl.p,) for pl in pool]
    pwork = float(sum(pl.n for pl in pool))

    def serve(th):
        for ai, bi, pi in pops:
            O.polymul(ai, bi, pi, threads=th)
    table["serving_polymul_payloads_first100"] = {
        "unit": "polymul/s", "all_cores": round(rate(lambda: serve(0), pwork, 1.0)[0], 1),
        "one_thread": round(rate(lambda: serve(1), pwork, 1.0)[0], 1)}
    return headline, table


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU layout is a design, not run here", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0809_0063_amd import dqt as D
    from paper_0809_0063_amd import inputs

    dev = torch.device("cuda:0")
    p = 3
    A, B = inputs.gemm_pair(MNK, MNK, MNK, p)
    dA, dB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    dC = torch.empty((MNK, MNK), dtype=torch.uint8, device=dev)
    plan = D.GemmPlan(algo=D.GEMM_CMM)
    ws = torch.empty(D.fgemm_workspace_size(p, MNK, MNK, MNK, plan), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    # warmup: both launch forms of the timed loop (the plain one and the one recording events), so
    # that no first-call cost of either falls into the timed region
    wcall = D.FgemmCall(dA, dB, dC, p, plan=plan, workspace=ws, stream=stream)
    w_a, w_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w_a.record(stream)           # torch creates the HIP event at its first record
    w_b.record(stream)
    for i in range(max(2, args.warmup)):
        if i % 2:
            wcall.run_timed(w_a, w_b)
        else:
            wcall.run()
    torch.cuda.synchronize()

    # timed region: K whole steps; the packed multiply kernel of the last n_ev steps records its
    # own start and end (a launch that records events costs the host about twice as much as a
    # plain one; the plain steps before them let the host run ahead of the device, so that the
    # sampled steps do not leave the device idle): at least 8 samples, every eighth step's worth
    # beyond 64 steps
    n_ev = min(args.steps, max(MIN_EVENT_SAMPLES, args.steps // 8))
    first_sampled = args.steps - n_ev
    ev_a = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    ev_b = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    for e in ev_a + ev_b:        # torch creates the HIP event at its first record
        e.record(stream)
    # arguments marshalled once, so that the host issues the launches faster than the device runs them
    call = D.FgemmCall(dA, dB, dC, p, plan=plan, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t_start.record(stream)
    host_t0 = time.perf_counter()
    for i in range(args.steps):
        if i >= first_sampled:
            # pack + multiply in one call; the multiply kernel records its own start and end
            call.run_timed(ev_a[i - first_sampled], ev_b[i - first_sampled])
        else:
            call.run()      # pack + multiply in one call
    t_end.record(stream)
    host_s = time.perf_counter() - host_t0
    torch.cuda.synchronize()
    total_s = t_start.elapsed_time(t_end) / 1e3
    step_s = total_s / args.steps
    # the HIP runtime recorded ev_a/ev_b at the kernel's own start and end
    kern_s = sum(hip_elapsed_ms(a, b) for a, b in zip(ev_a, ev_b)) / 1e3 / n_ev
    fp_ops = 2.0 * MNK ** 3
    value = fp_ops / step_s / 1e9

    # correctness of the timed output against a cheap property (full parity is in the tests):
    # row 0 of C equals row 0 of A times B mod 3 computed with integer numpy on the host
    row0 = (A[:1].astype(np.int64) @ B.astype(np.int64)) % p
    assert (dC[:1].cpu().numpy() == row0).all(), "bench output mismatch"

    # roofline of the packed multiply kernel: algorithmic dot2 lane-instructions per launch
    lane_ops = MNK * MNK * (MNK // 4)
    achieved = lane_ops / kern_s
    roofline = {
        "bound": "alu",
        "achieved": round(achieved / 1e12, 3),
        "peak": round(PEAK_LANE_OPS / 1e12, 3),
        "unit": "Tlane-op/s",
        "frac": round(achieved / PEAK_LANE_OPS, 4),
        "traffic": TRAFFIC["bytes"] if TRAFFIC["sha256"] == kernel_sources_sha256() else None,
        "kernel": "k_gemm_words<DOT2> (packed multiply-accumulate + epilogue)",
        "kernel_us": round(kern_s * 1e6, 3),
        "kernel_samples": n_ev,
        "host_issue_us_per_step": round(host_s / args.steps * 1e6, 2),
        "fp_top_s": round(fp_ops / kern_s / 1e12, 2),
    }

    if args.copy_probe:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    sections = set(args.sections.split(",")) if args.sections else set(SECTIONS)
    if args.no_extra:
        sections -= {"gemm", "polymul", "fqt", "gf"}
    if args.no_workloads:
        sections.discard("workloads")
    if args.no_cpu:
        sections.discard("cpu")
    log(f"headline done: {step_s * 1e6:.2f} us per step")
    extra = {}
    reps_gemm = max(4, args.steps // 2)
    reps_big = max(2, args.steps // 20)
    if "gemm" in sections:
        extra.update(bench_gemm_comparators(D, torch, dA, dB, dC, p, row0, stream, reps_gemm))
        log("gemm comparators done")
    if "polymul" in sections:
        extra.update(bench_polymul(D, inputs, torch, dev, reps_big, reps_gemm))
        log("polymul done")
    if "fqt" in sections:
        extra.update(bench_fqt(D, inputs, torch, dev, reps_big))
        log("fqt done")
    if "gf" in sections:
        extra.update(bench_gf(D, inputs, torch, dev, reps_big))
        log("gf done")
    if "workloads" in sections:
        from paper_0809_0063_amd import workloads as W
        from paper_0809_0063_amd import tune as T
        for name, fn in (("batched_10000_tuned", lambda: W.batched(10000, replays=3, tuner=T.Tuner())),
                         ("batched_10000_packed_cmm", lambda: W.batched(10000, replays=3, tuner=T.Tuner(),
                                                                         algo=D.GEMM_CMM)),
                         ("batched_10000_by_bucket", lambda: W.batched_buckets(10000, tuner=T.Tuner())),
                         ("serving", lambda: W.serving(n_requests=5000, warmup=500, loads=(0.5, 0.8, 1.2)))):
            try:
                extra[name] = fn()
            except Exception as e:  # reported in the output line, not hidden
                extra[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.synchronize()
            log(f"{name} done")

    cpu = None
    if "cpu" in sections:
        cpu, table = cpu_baselines(A, B, p, row0, fp_ops, inputs)
        log("cpu baselines done")
        extra["cpu_oracle"] = table

    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "F_p matrix product C = A.B mod 3, m = n = k = 1024, uint8 entries, packed DQT (CMM) + REDC",
                   "p": p, "m": MNK, "n": MNK, "k": MNK},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
