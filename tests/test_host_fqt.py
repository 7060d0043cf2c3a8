"""The FQT block-word reduction of the long-product kernels, built from the same source for the
host under UBSan and ASan, against the oracle's products (no GPU).

Three forms of the reduction: block words formed first (the compile-time instance the kernels
use over F_3 at q = 2^8), block words formed on demand inside the reduction loop (that
instance is not built for the device: it gave wrong bytes there), and the run-time form."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_0809_0063_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "host", "fqt_host.hip")
PKG = os.path.join(ROOT, "paper_0809_0063_amd")


@pytest.fixture(scope="module")
def fqt_host(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_0809_0063_amd import build
    build.ensure_built()
    exe = str(tmp_path_factory.mktemp("fqt") / "fqt_host")
    cmd = [hipcc, "-O2", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fno-sanitize-recover=all", SRC, f"-L{PKG}", "-ldqt", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.parametrize("na,nb", [(48, 48), (47, 48), (10, 37), (33, 31), (1, 48)])
def test_fqt_forms_on_host(fqt_host, tmp_path, na, nb):
    count = 20000
    a, b = inputs.polymul_pairs(count, na, 3, seed=na * 1000 + nb, kb=nb)
    a[::7] = 2            # every seventh product at the worst case (all entries p - 1)
    b[::7] = 2
    pa, pb = tmp_path / "a.bin", tmp_path / "b.bin"
    a.tofile(pa)
    b.tofile(pb)
    outs = [tmp_path / f"o{i}.bin" for i in range(3)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([fqt_host, str(count), str(pa), str(pb), *map(str, outs), str(na), str(nb)],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    ref = O.polymul(a, b, 3)
    for name, o in zip(("words first", "on demand", "run-time"), outs):
        got = np.fromfile(o, dtype=np.uint8).reshape(count, na + nb - 1)
        assert (got == ref).all(), name


@pytest.fixture(scope="module")
def redq_host(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_0809_0063_amd import build
    build.ensure_built()
    exe = str(tmp_path_factory.mktemp("redq") / "redq_host")
    src = os.path.join(HERE, "host", "redq_host.hip")
    cmd = [hipcc, "-O2", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fno-sanitize-recover=all", src, f"-L{PKG}", "-ldqt", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


# (p, b, residues, word bits): the long-product blocks (2, 3, 4 coefficients: 3, 5, 7 residues at
# q = 2^17, 2^10, 2^7) and windows of the correction wider than 32 bits of the word
@pytest.mark.parametrize("p,b,nres,bits", [(5, 17, 3, 51), (7, 17, 3, 51), (13, 17, 3, 51), (31, 17, 3, 51),
                                           (127, 17, 3, 51), (3, 10, 5, 50), (5, 10, 5, 50), (2, 10, 5, 50),
                                           (3, 7, 7, 49), (7, 7, 7, 49), (5, 16, 3, 48), (3, 13, 4, 52),
                                           (5, 26, 2, 52), (7, 24, 2, 52), (11, 12, 4, 48)])
@pytest.mark.parametrize("window", [0, 1, 2])
def test_redq_on_host(redq_host, p, b, nres, bits, window):
    """REDQ of words with uniform (and all-maximal) q-adic digits gives every digit mod p, for every
    table window (0 = the default, 1 = no table, 2 = pairs)."""
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([redq_host, str(p), str(b), str(nres), str(bits), str(window), "200000", str(p * 1000 + b)],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-500:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
