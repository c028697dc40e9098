"""Parity of the propagation for any even N with zero padding (Sec. 3.3) with the FP64 oracle."""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np
import pytest
import torch

import oracle as O
import wolf_inputs as WI
from tests.gpu_util import separable_rel

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


def fp32_bound(w, n, p, z, farfield, nz):
    """Rounding bound of the complex64 dense passes: four chained products with inner dimension N
    (tables rounded once), |error| <= (4N + 8) u |K*| |K*| |W| |K| |K| entrywise, relative to the
    L2 norm of the exact result."""
    kx = np.abs(O.kernel_1d(n, p, LAM, z, farfield, "x", nz))
    ky = np.abs(O.kernel_1d(n, p, LAM, z, farfield, "y", nz))
    mag = np.abs(w)
    for ax, k in ((2, kx), (3, ky), (0, kx), (1, ky)):
        mag = np.moveaxis(np.tensordot(k, mag, axes=([1], [ax])), 0, ax)
    ref, _ = O.propagate(w, n, p, LAM, z, farfield, n_fft=nz)
    s = O.coupling_constant(LAM, z) * p ** 4
    return (4 * n + 8) * U32 * s * np.linalg.norm(mag) / np.linalg.norm(ref)


# (N, N_z): zero-padded FFT passes for powers of two and for the mixed lengths 6, 10, 12, 20, 24, 36,
# 48 (N_z = Q L2^2 with odd factors 3 and 5); dense passes for 14, 22, 40 (no such split in the list).
# N_z = 8, 32, 128 with 2N <= N_z take the folded first stage, with the padding offset s = 3, 2, 10, 9, 8,
# 61 (s mod L2 = 1, 0, 2, 1, 0, 5 at L2 = 2, 4, 8); (18, 32) is past the fold (2N > N_z).
CASES = [(2, 2), (4, 8), (6, 6), (6, 10), (10, 16), (12, 12), (16, 40), (24, 64), (10, 20), (20, 24), (12, 36),
         (24, 48), (6, 14), (10, 22), (2, 8), (12, 32), (14, 32), (16, 32), (18, 32), (6, 128)]


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("n,nz", CASES)
def test_padded_vs_oracle(gpu_lib, n, nz, dtype, farfield):
    p, z = 20e-6, 0.05
    w = WI.random_hermitian_psd(n, seed=90 + n)
    ref, dxr = O.propagate(w, n, p, LAM, z, farfield, n_fft=nz)
    got, dx = gpu_lib.propagate_padded(dev(w, dtype), p, LAM, z, nz, farfield)
    assert abs(dx / dxr - 1) < 1e-15
    tol = 1e-12 if dtype == torch.complex128 else fp32_bound(w, n, p, z, farfield, nz)
    assert rel(host(got), ref) < tol


def test_padded_in_place(gpu_lib):
    n, nz, p, z = 10, 16, 20e-6, 0.05
    w = dev(WI.random_hermitian_psd(n, seed=95), torch.complex128)
    a, _ = gpu_lib.propagate_padded(w, p, LAM, z, nz)
    b = w.clone()
    gpu_lib.propagate_padded(b, p, LAM, z, nz, out=b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("n", [8, 32])
def test_padded_without_padding_matches_fft_path(gpu_lib, n):
    """For a power-of-two N and n_fft = N the dense passes and the FFT passes compute the same operator."""
    p, z = 20e-6, 0.05
    w = dev(WI.random_complex((n, n, n, n), seed=96), torch.complex128)
    a, _ = gpu_lib.propagate_padded(w, p, LAM, z)
    b, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
    assert rel(host(a), host(b)) < 1e-12


@pytest.mark.parametrize("model", [WI.MODEL_GSM, WI.MODEL_COHERENT, WI.MODEL_INCOHERENT])
def test_source_builder_even_n(gpu_lib, model):
    n, p = 10, 20e-6
    sp = SimpleNamespace(model=model, amplitude=1.3, sigma_s_m=0.05e-3, sigma_g_m=0.04e-3, geometry=WI.GEO_CIRCLE,
                         geo_r0_m=3.5 * p, geo_r1_m=0.0, intensity_map=None, mask=None, lens_focal_m=0.0,
                         wavelength_m=0.0)
    got = host(gpu_lib.build_source(sp, n, p, torch.complex128))
    assert rel(got, O.build_source(sp, n, p)) < 1e-14


@pytest.mark.parametrize("n,nz,dtype", [(200, 512, torch.complex64), (96, 192, torch.complex128),
                                        (100, 256, torch.complex128), (200, 200, torch.complex64),
                                        (100, 100, torch.complex128), (144, 144, torch.complex64),
                                        (200, 210, torch.complex64), (60, 128, torch.complex64),
                                        (120, 512, torch.complex128), (256, 512, torch.complex64),
                                        (136, 512, torch.complex64), (196, 512, torch.complex128),
                                        (100, 512, torch.complex64), (32, 128, torch.complex64),
                                        (64, 128, torch.complex128), (160, 512, torch.complex128),
                                        (40, 128, torch.complex128)])
def test_padded_full_size_gsm(gpu_lib, n, nz, dtype):
    """The paper's example sizes: N = 200 padded to N_z = 512 and N = 200 unpadded (complex64, 1.6e9
    elements; power-of-two and 20 x 10 mixed-radix FFT passes), with N = 96 padded to 192, N = 100
    padded to 256, N = 100 unpadded (complex128), N = 144 unpadded (FFT passes) and N = 200 padded to
    210 (dense passes), GSM source, against the separable oracle with the same padding; N = 60 padded
    to 128, N = 120 padded to 512 (complex128) and N = 256 padded to 512 (the largest N, 2N = N_z) take
    the folded first stage. At N_z = 512 the bands of N in [64, 256] take compile-time row ranges:
    N = 100 (complex64, band 64-127, ragged 16-line tiles), 136 (band 128-191, ragged), 200 (band
    192-255) and 256, and N = 120 and 196 (complex128, bands 64-127 and 192-255, 196 with ragged 8-line
    tiles), and N = 160 (complex128, band 128-191); at N_z = 128 the bands 32-63 (N = 32 and 60 in complex64,
    60 with ragged 32-line tiles; N = 40 in complex128) and 64 (complex128)."""
    p, z, ss, sg = 20e-6, 0.5, 0.1e-3, 0.05e-3
    sp = SimpleNamespace(model=WI.MODEL_GSM, amplitude=1.0, sigma_s_m=ss, sigma_g_m=sg, geometry=WI.GEO_NONE,
                         geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=None, mask=None, lens_focal_m=0.0,
                         wavelength_m=0.0)
    w = gpu_lib.build_source(sp, n, p, dtype)
    gpu_lib.propagate_padded(w, p, LAM, z, nz, out=w)
    wx, wy = O.gsm_axis_factor(n, p, ss, sg, "x"), O.gsm_axis_factor(n, p, ss, sg, "y")
    bx, by = O.propagate_separable(wx, wy, n, p, LAM, z, n_fft=nz)
    if dtype == torch.complex128:
        tol = 1e-12
    else:
        kx = np.abs(O.kernel_1d(n, p, LAM, z, False, "x", nz))
        ky = np.abs(O.kernel_1d(n, p, LAM, z, False, "y", nz))
        s = O.coupling_constant(LAM, z) * p ** 4
        mx = s * kx @ np.abs(wx) @ kx.T
        my = ky @ np.abs(wy) @ ky.T
        tol = (4 * n + 8) * U32 * np.linalg.norm(mx) * np.linalg.norm(my) / (np.linalg.norm(bx) * np.linalg.norm(by))
    assert separable_rel(w, bx, by) < tol
    del w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,nz,dtype", [(136, 512, torch.complex64), (200, 512, torch.complex128),
                                        (200, 200, torch.complex64), (144, 144, torch.complex128)])
def test_padded_plane_groups_out_of_place(gpu_lib, n, nz, dtype):
    """The passes run over groups of i1 planes (12, 2, 4 and 5 planes here; 136 and 144 leave a ragged last
    group), padded and unpadded; out of place each group's first pass reads its planes of the input. The
    result equals the in-place one bit for bit and the input is left unchanged."""
    sp = SimpleNamespace(model=WI.MODEL_GSM, amplitude=1.0, sigma_s_m=0.1e-3, sigma_g_m=0.05e-3, geometry=WI.GEO_NONE,
                         geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=None, mask=None, lens_focal_m=0.0, wavelength_m=0.0)
    w = gpu_lib.build_source(sp, n, 20e-6, dtype)
    w0 = w.clone()
    out, _ = gpu_lib.propagate_padded(w, 20e-6, LAM, 0.5, nz)
    torch.cuda.synchronize()
    assert torch.equal(w, w0)
    gpu_lib.propagate_padded(w, 20e-6, LAM, 0.5, nz, out=w)
    torch.cuda.synchronize()
    assert torch.equal(out, w)
    del w, w0, out
    torch.cuda.empty_cache()


def test_padded_rejects(gpu_lib):
    w = torch.zeros((6, 6, 6, 6), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_padded(w, 20e-6, LAM, 0.1, 4)         # n_fft < N
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_padded(w, 20e-6, LAM, 0.1, 4096)      # n_fft > 2048
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_padded(w, 20e-6, LAM, 0.1, 8, work=w)  # work overlaps the input
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_fresnel(w, 20e-6, LAM, 0.1)            # the FFT path needs a power of two
    odd = torch.zeros((5, 5, 5, 5), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_padded(odd, 20e-6, LAM, 0.1, 8)
