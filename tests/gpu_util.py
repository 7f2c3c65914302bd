"""Helpers shared by the GPU tests: host <-> device bit strings."""

import numpy as np


def to_dev(words, device="cuda"):
    import torch
    a = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_dev_u32(vals, device="cuda"):
    import torch
    a = np.ascontiguousarray(np.asarray(vals, dtype=np.uint32))
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def bit(words: np.ndarray, k: int) -> int:
    return int((int(words[k >> 6]) >> (k & 63)) & 1)


def first_diff(a: np.ndarray, b: np.ndarray) -> str:
    d = np.nonzero(a != b)[0]
    if d.size == 0:
        return "equal"
    w = int(d[0])
    x = int(a[w]) ^ int(b[w])
    return f"{d.size} words differ; first word {w} bit {(x & -x).bit_length() - 1}"
