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


def separable_mu_check(mu_gpu: torch.Tensor, bx: np.ndarray, by: np.ndarray, floor: float, band: float):
    """The full mu[p1; p2] of W = bx (x) by, masked where S = Re diag(bx) (x) Re diag(by) is at or below
    floor * max S on either point (Algorithm 5, floor reading), against the device result, one
    first-point row at a time in float64.

    Points whose S lies within a relative `band` of the floor are left out (the device's S carries its
    own rounding there). Returns (relative L2 error over the compared entries, number of compared entries
    where the device's mask disagrees: a nonzero mu outside the mask, or zero where |mu| > 1e-3 inside)."""
    n = mu_gpu.shape[0]
    sx = np.real(np.diag(bx))
    sy = np.real(np.diag(by))
    s = sx[:, None] * sy[None, :]
    tau = floor * s.max()
    ok = s > tau
    clear = np.abs(s / tau - 1) > band
    okt = torch.from_numpy(ok).cuda()
    cleart = torch.from_numpy(clear).cuda()
    rsx = torch.from_numpy(np.sqrt(np.where(sx > 0, sx, 1.0))).cuda()
    rsy = torch.from_numpy(np.sqrt(np.where(sy > 0, sy, 1.0))).cuda()
    bxt = torch.from_numpy(bx).cuda()
    byt = torch.from_numpy(by).cuda()
    mux = bxt / (rsx[:, None] * rsx[None, :])                   # [m1, m2]
    muy = byt / (rsy[:, None] * rsy[None, :])                   # [n1, n2]
    num = den = 0.0
    bad = 0
    for m1 in range(n):
        got = mu_gpu[m1].to(torch.complex128)                   # [n1][m2][n2]
        exp = mux[m1][None, :, None] * muy[:, None, :]
        mask = okt[m1][:, None, None] & okt[None, :, :]         # both points above the floor
        use = cleart[m1][:, None, None] & cleart[None, :, :]
        exp = torch.where(mask, exp, torch.zeros_like(exp))
        d = (got - exp)[use]
        num += torch.sum(torch.abs(d) ** 2).item()
        den += torch.sum(torch.abs(exp[use]) ** 2).item()
        bad += int(torch.sum(use & ~mask & (got != 0)).item())
        bad += int(torch.sum(use & mask & (got == 0) & (torch.abs(exp) > 1e-3)).item())
    return math.sqrt(num / den), bad
