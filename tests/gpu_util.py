"""Helpers shared by the GPU parity tests."""
from __future__ import annotations

import sys

import numpy as np
import torch


def dev(a, dtype=torch.float64) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu").numpy()


def fwd_err(x, ref) -> float:
    """max over columns of ||x - ref||_inf / ||ref||_inf."""
    x = np.asarray(x, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    num = np.abs(x - ref).max(axis=0)
    den = np.maximum(np.abs(ref).max(axis=0), 1e-300)
    return float((num / den).max())


def case(msg: str):
    """Name the case on stdout before a GPU step (flushed)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()
