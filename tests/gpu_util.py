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
