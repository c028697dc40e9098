"""Parity of the thin-lens propagation and of two-stage imaging (Sec. 2.2) with the FP64 oracle."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle as O
import wolf_inputs as WI
from tests.gpu_util import separable_rel

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}
LAM = WI.LAMBDA_HENE
DT = [torch.complex64, torch.complex128]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


PUPILS = [(O.GEO_NONE, 0.0), (O.GEO_CIRCLE, 0.35), (O.GEO_SQUARE, 0.3)]   # radius as a fraction of N pitch


@pytest.mark.parametrize("pupil", PUPILS)
@pytest.mark.parametrize("focal", [0.1, -0.4, 0.0])
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n", [4, 16, 32])
def test_lens_vs_oracle(gpu_lib, n, dtype, focal, pupil):
    p, z = 20e-6, 0.15
    geo, frac = pupil
    r = frac * n * p
    w = WI.random_hermitian_psd(n, seed=70 + n)
    ref, pref = O.propagate_lens(w, n, p, LAM, focal, z, geo, r)
    got, pc = gpu_lib.propagate_lens(dev(w, dtype), p, LAM, focal, z, geo, r)
    assert abs(pc / pref - 1) < 1e-15
    assert rel(host(got), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", DT)
def test_lens_all_schedules_agree(gpu_lib, dtype):
    """The pupil is applied inside the slab pass (fused_slab 1, 2) or by its own pass first (0)."""
    n, p, z, f = 32, 20e-6, 0.1, 0.07
    r = 0.3 * n * p
    w = WI.random_complex((n, n, n, n), seed=72)
    ref, _ = O.propagate_lens(w, n, p, LAM, f, z, O.GEO_CIRCLE, r)
    nn = n * n
    try:
        for plan in [(1, 0, 0, 0, 1), (2, 0, 0, 0, 1), (0, 0, 0, 0, 1), (0, nn // 4, 64, 0, 1), (3, 4 * n, 0, 0, 1),
                     (1, 8 * n, 0, 0, 1)]:
            gpu_lib.set_plan(n, dtype, *plan)
            got, _ = gpu_lib.propagate_lens(dev(w, dtype), p, LAM, f, z, O.GEO_CIRCLE, r)
            assert rel(host(got), ref) < TOL[dtype], plan
            x = dev(w, dtype)
            gpu_lib.propagate_lens(x, p, LAM, f, z, O.GEO_CIRCLE, r, out=x)   # in place
            assert rel(host(x), ref) < TOL[dtype], plan
    finally:
        gpu_lib.set_plan(n, dtype)


@pytest.mark.parametrize("n,r1,r2", [(16, 0.2, 0.2), (32, 0.15, 0.45)])
@pytest.mark.parametrize("dtype", DT)
def test_imaging_vs_oracle(gpu_lib, n, r1, r2, dtype):
    p = 20e-6
    f = r1 * r2 / (r1 + r2) * 1.05
    w = WI.random_hermitian_psd(n, seed=74)
    pb = O.output_pitch(n, p, LAM, r1)
    ref, pcr = O.image_through_lens(w, n, p, LAM, r1, f, r2, O.GEO_CIRCLE, 0.4 * n * pb)
    got, pc = gpu_lib.image_through_lens(dev(w, dtype), p, LAM, r1, f, r2, O.GEO_CIRCLE, 0.4 * n * pb)
    assert abs(pc / pcr - 1) < 1e-15
    assert rel(host(got), ref) < TOL[dtype]


def _separable_imaging(wx, wy, n, p, r1, f, r2, half_side):
    """Two-stage imaging of a separable source with a square pupil (also separable), from the
    oracle's separable propagation and the per-axis factor of T = P q*(f) on the lens plane."""
    bx, by = O.propagate_separable(wx, wy, n, p, LAM, r1)
    pb = O.output_pitch(n, p, LAM, r1)
    c = np.arange(n) - n / 2
    keep = (c ** 2 <= (half_side / pb) ** 2 * (1 + 1e-9)) if half_side > 0 else np.ones(n, bool)
    t = keep * np.exp(-1j * math.pi * (pb * c) ** 2 / (LAM * f))
    bx = np.conj(t)[:, None] * bx * t[None, :]
    by = np.conj(t)[:, None] * by * t[None, :]
    return O.propagate_separable(bx, by, n, pb, LAM, r2)


@pytest.mark.parametrize("half_side", [0.0, 0.25])
def test_imaging_full_size_gsm128(gpu_lib, half_side):
    """N = 128 complex64 GSM source through a 2f-2f system (R1 = R2 = 0.4 m, f = 0.2 m), without
    and with a square pupil, against the separable oracle. Without a pupil the image S is the
    mirrored source S (exact on the grid)."""
    wl = WI.gsm128()
    n, p, sp = wl.n, wl.pitch_m, wl.source
    r1 = r2 = 0.4
    f = 0.2
    pb = O.output_pitch(n, p, LAM, r1)
    w = gpu_lib.build_source(sp, n, p, torch.complex64)
    gpu_lib.image_through_lens(w, p, LAM, r1, f, r2, O.GEO_SQUARE if half_side else O.GEO_NONE,
                               half_side * n * pb, out=w)
    wx = O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x")
    wy = O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y")
    bx, by = _separable_imaging(wx, wy, n, p, r1, f, r2, half_side * n * pb)
    assert separable_rel(w, bx, by) < TOL[torch.complex64]
    if half_side == 0.0:
        s = host(gpu_lib.spectral_density(w)).astype(np.float64)
        rev = (n - np.arange(n)) % n
        sa = np.real(np.diag(wx)[:, None] * np.diag(wy)[None, :])
        assert rel(s, sa[np.ix_(rev, rev)]) < TOL[torch.complex64]
    del w
    torch.cuda.empty_cache()


def test_lens_rejects_bad_arguments(gpu_lib):
    w = torch.zeros((4, 4, 4, 4), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_lens(w, 20e-6, LAM, 0.1, 0.2, O.GEO_ANNULUS, 1e-5)
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_lens(w, 20e-6, LAM, 0.1, 0.2, O.GEO_CIRCLE, 0.0)
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_lens(w, 20e-6, LAM, math.inf, 0.2)
