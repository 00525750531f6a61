"""Helpers of the GPU tests: host <-> device transfers of uint64 residue arrays."""
import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    """uint64 numpy array -> int64 device tensor with the same bits."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def empty(shape) -> torch.Tensor:
    return torch.empty(shape, dtype=torch.int64, device="cuda")


def first_mismatch(a: np.ndarray, b: np.ndarray):
    """Index and values of the first differing element, or None."""
    if a.shape != b.shape:
        return ("shape", a.shape, b.shape)
    diff = np.argwhere(a != b)
    if len(diff) == 0:
        return None
    idx = tuple(int(v) for v in diff[0])
    return (idx, int(a[idx]), int(b[idx]), int(len(diff)))
