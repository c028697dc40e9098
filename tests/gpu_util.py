"""Comparison helpers for the GPU tests (plain torch on the device; no library code)."""
from __future__ import annotations

import math

import numpy as np
import torch


def separable_rel(w_gpu: torch.Tensor, bx: np.ndarray, by: np.ndarray) -> float:
    """Relative L2 distance between a device CSD W[i1, j1, i2, j2] and bx[i1, i2] by[j1, j2], one
    first-point row i1 at a time (the reference is never materialised whole)."""
    n = w_gpu.shape[0]
    bxt = torch.from_numpy(bx).cuda()
    byt = torch.from_numpy(by).cuda()
    num = 0.0
    den = 0.0
    for m1 in range(n):
        blk = w_gpu[m1].to(torch.complex128)                     # [n1][m2][n2]
        exp = bxt[m1][None, :, None] * byt[:, None, :]           # [n1][m2][n2] = bx[m1,m2] by[n1,n2]
        num += torch.sum(torch.abs(blk - exp) ** 2).item()
        den += torch.sum(torch.abs(exp) ** 2).item()
    return math.sqrt(num / den)
