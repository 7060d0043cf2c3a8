"""Shared helpers for the GPU parity tests."""
import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(device())


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def unaligned_like(x: np.ndarray, offset: int = 1) -> torch.Tensor:
    """A contiguous device copy of x whose data pointer is `offset` bytes past an aligned address."""
    flat = torch.zeros(x.size + 64, dtype=torch.uint8, device=device())
    view = flat[offset:offset + x.size].view(x.shape)
    view.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return view


def unaligned_empty(shape, offset: int = 1) -> torch.Tensor:
    n = int(np.prod(shape))
    flat = torch.zeros(n + 64, dtype=torch.uint8, device=device())
    return flat[offset:offset + n].view(shape)


GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)), "golden")


def load_digests(name: str):
    """Rows of a digest file under tests/golden/ (written by tests/golden/make_digests.py from the oracle)."""
    import os
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def digest(x: np.ndarray) -> str:
    """128-bit prefix of SHA-256 over the bytes of x in C order (the digest the golden files hold)."""
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()[:32]
