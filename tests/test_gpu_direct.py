"""Parity of the exact-kernel direct sum (eq. h_free; the validity check of the Fresnel
approximation) with the FP64 oracle."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle as O
import wolf_inputs as WI

pytestmark = pytest.mark.gpu

LAM = WI.LAMBDA_HENE
U32 = 2.0 ** -24


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def fp32_bound(w, n, p, z, kind):
    """Rounding bound of the complex64 path: the entries of H rounded once, then two products with
    inner dimension K = N^2 accumulated in FP32, |error| <= (2K + 4) u |conj(H)| |W| |H|^T (entrywise;
    the standard bound for a product chain), taken relative to the L2 norm of the exact result."""
    h = O.rs_kernel_matrix(n, p, LAM, z, kind)
    wm = w.reshape(n * n, n * n)
    k = n * n
    mag = p ** 4 * (np.abs(h) @ np.abs(wm) @ np.abs(h).T)
    ref = p ** 4 * (np.conj(h) @ wm @ h.T)
    return (2 * k + 4) * U32 * np.linalg.norm(mag) / np.linalg.norm(ref)


@pytest.mark.parametrize("kind", [O.KIND_SECONDARY, O.KIND_PRIMARY])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("n", [2, 4, 8, 16, 32])
def test_direct_vs_oracle(gpu_lib, n, dtype, kind):
    p, z = 20e-6, 4e-3
    w = WI.random_hermitian_psd(n, seed=80 + n)
    ref, dxr = O.propagate_direct(w, n, p, LAM, z, kind)
    got, dx = gpu_lib.propagate_direct(dev(w, dtype), p, LAM, z, kind)
    assert abs(dx / dxr - 1) < 1e-15
    tol = 1e-12 if dtype == torch.complex128 else fp32_bound(w, n, p, z, kind)
    assert rel(host(got), ref) < tol


def test_direct_in_place_and_repeatable(gpu_lib):
    n, p, z = 8, 20e-6, 4e-3
    w = dev(WI.random_hermitian_psd(n, seed=85), torch.complex128)
    a, _ = gpu_lib.propagate_direct(w, p, LAM, z)
    b = w.clone()
    gpu_lib.propagate_direct(b, p, LAM, z, out=b)
    c, _ = gpu_lib.propagate_direct(w, p, LAM, z)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_direct_n64_sampled(gpu_lib):
    """N = 64 complex128 (the size the check is meant for): every output is a sum over 2^24 source
    pairs; 24 sampled outputs and the S row through the centre are computed one by one by the oracle."""
    n, p, z = 64, 20e-6, 0.02
    sp = WI.gsm_small()[0].source
    w = gpu_lib.build_source(sp, n, p, torch.complex128)
    got, _ = gpu_lib.propagate_direct(w, p, LAM, z)
    g = host(got).reshape(n * n, n * n)
    del got
    wa = O.build_source(sp, n, p).reshape(n * n, n * n)
    h = O.rs_kernel_matrix(n, p, LAM, z)
    rng = WI.rng(86)
    rows = rng.integers(0, n * n, 24)
    cols = rng.integers(0, n * n, 24)
    scale = np.abs(g).max()
    for m1, m2 in zip(rows, cols):
        ref = p ** 4 * (np.conj(h[m1]) @ wa @ h[m2])
        assert abs(g[m1, m2] - ref) < 1e-12 * scale
    centre = [(n // 2) * n + j for j in range(n)]
    s_ref = np.array([p ** 4 * np.real(np.conj(h[m]) @ wa @ h[m]) for m in centre])
    assert rel(np.real(g[centre, centre]), s_ref) < 1e-12


def test_fresnel_validity_report(gpu_lib):
    """The error report of the Fresnel approximation equals the oracle's difference of the two sums."""
    n, p, z = 16, 20e-6, 3e-3
    w = WI.random_hermitian_psd(n, seed=87)
    d = gpu_lib.fresnel_validity(dev(w, torch.complex128), p, LAM, z)
    wd, _ = O.propagate_direct(w, n, p, LAM, z)
    wf, _ = O.propagate(w, n, p, LAM, z)
    assert abs(d["rel_l2_w"] / rel(wf, wd) - 1) < 1e-9
    sd, sf = O.spectral_density(wd), O.spectral_density(wf)
    assert abs(d["rel_l2_s"] / rel(sf, sd) - 1) < 1e-9
    assert abs(d["max_s_rel"] / (np.abs(sf - sd).max() / np.abs(sd).max()) - 1) < 1e-9


def test_direct_rejects(gpu_lib):
    w = torch.zeros((4, 4, 4, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_direct(w, 20e-6, LAM, -1.0)
    with pytest.raises(gpu_lib.WolfError):                      # work overlaps the input
        gpu_lib.propagate_direct(w, 20e-6, LAM, 1e-3, work=w)
    assert gpu_lib.load().wolf_direct_work_bytes(256, 0) == -1
