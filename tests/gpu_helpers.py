"""Shared helpers for the GPU tests: host <-> device transfer of uint32 residues."""
import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def empty(*shape) -> torch.Tensor:
    return torch.full(shape, -1, dtype=torch.int32, device="cuda")


def first_mismatch(got: np.ndarray, want: np.ndarray) -> str:
    if got.shape != want.shape:
        return f"shape {got.shape} != {want.shape}"
    bad = np.argwhere(got != want)
    if len(bad) == 0:
        return ""
    i = tuple(bad[0])
    return f"{len(bad)} mismatches, first at {i}: got {got[i]} want {want[i]}"
