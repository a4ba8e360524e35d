"""Host <-> device marshalling of uint32/uint64 coefficient arrays.

torch has no full uint64 arithmetic; the library only needs the bits, so words
travel as torch.int64 / torch.int32 tensors with identical bit patterns.
"""
from __future__ import annotations

import numpy as np


def to_device(a: np.ndarray, word_bits: int, device="cuda"):
    import torch
    if word_bits == 64:
        host = np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)
    elif word_bits == 32:
        host = np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)
    else:
        raise ValueError("word_bits must be 32 or 64")
    return torch.from_numpy(host.copy()).to(device)


def to_host(t, word_bits: int) -> np.ndarray:
    h = t.detach().cpu().contiguous().numpy()
    return h.view(np.uint64) if word_bits == 64 else h.view(np.uint32)


def empty_device(shape, word_bits: int, device="cuda"):
    import torch
    dt = torch.int64 if word_bits == 64 else torch.int32
    return torch.empty(tuple(shape), dtype=dt, device=device)
