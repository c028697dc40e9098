"""Parity of the polychromatic sum on a common output grid (R17) with the FP64 oracle."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle as O
import wolf_inputs as WI
from tests import closed_forms as CF

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("n", [2, 8, 16])
def test_polychromatic_vs_oracle(gpu_lib, n, dtype, farfield):
    """Random Hermitian source (not separable), five pairs of different wavelengths and distances, on
    a grid that is no pair's FFT grid, probe off-centre."""
    p = 20e-6
    w = WI.random_hermitian_psd(n, seed=70 + n)
    lam = np.array([500e-9, 560e-9, 633e-9, 700e-9, 610e-9])
    zs = np.array([0.05, 0.05, 0.08, 0.05, 0.12])
    ws = np.array([0.4, 1.0, 0.0, 0.7, 1.3])
    dxp = 0.83 * O.output_pitch(n, p, 600e-9, 0.06)
    ip, jp = n - 1, n // 2
    floor = 1e-4 if dtype == torch.complex64 else 1e-8
    s, mu = gpu_lib.propagate_polychromatic(torch.from_numpy(w).to(dtype).cuda(), p, lam, zs, ws, dxp,
                                            farfield=farfield, ip=ip, jp=jp, floor_rel=floor)
    sr, mur = O.polychromatic(w, n, p, lam, zs, ws, dxp, farfield, ip=ip, jp=jp, floor_rel=floor)
    assert rel(host(s), sr) < TOL[dtype]
    assert rel(host(mu), mur) < TOL[dtype] / math.sqrt(floor)


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("n", [2, 8, 32])
def test_polychromatic_single_pair_vs_oracle(gpu_lib, n, dtype, farfield):
    """One pair (the one-pass sums of a group of one) on a grid that is not its FFT grid, random Hermitian
    source, probe off-centre."""
    p = 20e-6
    w = WI.random_hermitian_psd(n, seed=80 + n)
    dxp = 1.17 * O.output_pitch(n, p, 560e-9, 0.07)
    ip, jp = n // 2 - 1, n - 1
    floor = 1e-4 if dtype == torch.complex64 else 1e-8
    s, mu = gpu_lib.propagate_polychromatic(torch.from_numpy(w).to(dtype).cuda(), p, [560e-9], [0.07], [0.8], dxp,
                                            farfield=farfield, ip=ip, jp=jp, floor_rel=floor)
    sr, mur = O.polychromatic(w, n, p, [560e-9], [0.07], [0.8], dxp, farfield, ip=ip, jp=jp, floor_rel=floor)
    assert rel(host(s), sr) < TOL[dtype]
    assert rel(host(mu), mur) < TOL[dtype] / math.sqrt(floor)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_polychromatic_two_groups_vs_oracle(gpu_lib, dtype):
    """70 pairs (a group of 64, then 6 whose sums add to the first group's in FP64), random Hermitian
    source at N = 8, random wavelengths, distances and weights, a common grid of no pair's pitch."""
    n, p = 8, 20e-6
    w = WI.random_hermitian_psd(n, seed=93)
    g = WI.rng(94)
    lam = g.uniform(450e-9, 750e-9, 70)
    zs = g.uniform(0.05, 0.2, 70)
    ws = g.uniform(0.0, 1.0, 70)
    dxp = 0.9 * O.output_pitch(n, p, 600e-9, 0.1)
    ip, jp = 2, 5
    floor = 1e-4 if dtype == torch.complex64 else 1e-8
    s, mu = gpu_lib.propagate_polychromatic(torch.from_numpy(w).to(dtype).cuda(), p, lam, zs, ws, dxp, ip=ip,
                                            jp=jp, floor_rel=floor)
    sr, mur = O.polychromatic(w, n, p, lam, zs, ws, dxp, False, ip=ip, jp=jp, floor_rel=floor)
    assert rel(host(s), sr) < TOL[dtype]
    assert rel(host(mu), mur) < TOL[dtype] / math.sqrt(floor)


@pytest.mark.parametrize("farfield", [False, True])
def test_single_pair_on_its_fft_grid_equals_batch(gpu_lib, farfield):
    """One pair on its own FFT grid (pitch lambda z / (N pitch)): the chirp-z transforms reduce to
    DFTs and the result equals the batch's (and the propagation's) S and mu."""
    n, p, lam, z = 16, 20e-6, 633e-9, 0.1
    w = torch.from_numpy(WI.random_hermitian_psd(n, seed=77)).to(torch.complex128).cuda()
    dx = O.output_pitch(n, p, lam, z)
    s1, mu1 = gpu_lib.propagate_polychromatic(w, p, [lam], [z], [0.6], dx, farfield=farfield, ip=3, jp=9,
                                              floor_rel=1e-8)
    s2, mu2 = gpu_lib.propagate_batch(w, p, [lam], [z], [0.6], farfield=farfield, ip=3, jp=9, floor_rel=1e-8)
    assert rel(host(s1), host(s2[0])) < 1e-12
    assert rel(host(mu1), host(mu2[0])) < 1e-10


def test_polychromatic_full_size_gsm(gpu_lib):
    """N = 128 complex64 GSM source, 16 wavelengths over 500-700 nm at z = 0.5 m with the Gaussian
    spectral weights, on the FFT grid of 500 nm: S and the mu row against the weighted sum of the
    closed-form GSM CSDs on that grid."""
    wl = WI.gsm128()
    n, p, sp = wl.n, wl.pitch_m, wl.source
    pairs = WI.polychromatic_pairs()
    sel = pairs["z"] == 0.5
    lam, zs, ws = pairs["wavelength"][sel], pairs["z"][sel], pairs["weight"][sel]
    dx = O.output_pitch(n, p, 500e-9, 0.5)
    ip, jp = wl.probe
    floor = 1e-4
    w0 = gpu_lib.build_source(sp, n, p, torch.complex64)
    s, mu = gpu_lib.propagate_polychromatic(w0, p, lam, zs, ws, dx, ip=ip, jp=jp, floor_rel=floor)
    s, mu = host(s), host(mu)
    del w0
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    sr = np.zeros((n, n))
    row = np.zeros((n, n), complex)
    for lk, zk, wk in zip(lam, zs, ws):
        cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], sp.sigma_s_m, sp.sigma_g_m, lk, zk, False)
        cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], sp.sigma_s_m, sp.sigma_g_m, lk, zk, False)
        sr += wk * np.real(np.diag(cx)[:, None] * np.diag(cy)[None, :])
        row += wk * cx[ip][:, None] * cy[jp][None, :]
    mur = row / np.sqrt(sr[ip, jp] * sr)
    mur[sr <= floor * sr.max()] = 0
    assert rel(s, sr) < 1e-5
    assert rel(mu, mur) < 1e-5 / math.sqrt(floor)


def test_polychromatic_small_group_paths_agree(gpu_lib):
    """N = 128 complex64 on a source that is not separable (the GSM source plus a seeded random array at
    5 % of its peak), 12 wavelengths at four distances on a common grid of no pair's pitch: the group of 12
    pairs (its difference sums on the register ring over one tile of 16 pairs) against the same pairs
    followed by 21 pairs of zero weight (a group of 33: two launches of the ring over two tiles each, the
    second at a pair offset of 32). The sums are the same up to FP32 summation order."""
    wl = WI.gsm128()
    n, p = wl.n, wl.pitch_m
    pairs = WI.polychromatic_pairs()
    lam, zs, ws = pairs["wavelength"][:12], pairs["z"][:12], pairs["weight"][:12]
    g = WI.rng(97)
    lam_pad = np.concatenate([lam, g.uniform(500e-9, 700e-9, 21)])
    zs_pad = np.concatenate([zs, g.uniform(0.1, 1.0, 21)])
    ws_pad = np.concatenate([ws, np.zeros(21)])
    dx = 0.87 * O.output_pitch(n, p, 600e-9, 0.5)
    ip, jp = wl.probe
    floor = 1e-3
    w0 = gpu_lib.build_source(wl.source, n, p, torch.complex64)
    w0 += 0.05 * float(w0.abs().max()) * torch.from_numpy(
        WI.random_complex((n, n, n, n), seed=98, dtype=np.complex64)).cuda()
    s1, mu1 = gpu_lib.propagate_polychromatic(w0, p, lam, zs, ws, dx, ip=ip, jp=jp, floor_rel=floor)
    s2, mu2 = gpu_lib.propagate_polychromatic(w0, p, lam_pad, zs_pad, ws_pad, dx, ip=ip, jp=jp, floor_rel=floor)
    s1, mu1, s2, mu2 = host(s1), host(mu1), host(s2), host(mu2)
    del w0
    torch.cuda.empty_cache()
    assert rel(s1, s2) < 1e-5
    assert rel(mu1, mu2) < 1e-5 / math.sqrt(floor)


@pytest.mark.parametrize("count", [24, 64])
def test_polychromatic_on_shared_fft_grid_equals_batch_sum(gpu_lib, count):
    """N = 128 complex64 on a source that is not separable (the GSM source plus a seeded random array at
    5 % of its peak), with pairs of one product lambda z, so that every pair's FFT grid is the common grid:
    the polychromatic S equals the sum over pairs of the batch's S (groups of 24 pairs: the difference sums
    on the register ring over two tiles of 16 pairs; 64: two launches of it). The batch takes the folded
    Fresnel difference sums, so this pins the unfolded bins of the ring on a non-separable source."""
    wl = WI.gsm128()
    n, p = wl.n, wl.pitch_m
    g = WI.rng(99)
    lam = np.sort(g.uniform(500e-9, 700e-9, count))
    lz = 600e-9 * 0.5
    zs = lz / lam
    ws = g.uniform(0.2, 1.0, count)
    dx = O.output_pitch(n, p, 600e-9, 0.5)
    ip, jp = wl.probe
    w0 = gpu_lib.build_source(wl.source, n, p, torch.complex64)
    w0 += 0.05 * float(w0.abs().max()) * torch.from_numpy(
        WI.random_complex((n, n, n, n), seed=100, dtype=np.complex64)).cuda()
    s_poly, _ = gpu_lib.propagate_polychromatic(w0, p, lam, zs, ws, dx, ip=ip, jp=jp)
    s_batch, _ = gpu_lib.propagate_batch(w0, p, lam, zs, ws, ip=ip, jp=jp)
    s_poly = host(s_poly).astype(np.float64)
    s_sum = host(s_batch).astype(np.float64).sum(axis=0)
    del w0
    torch.cuda.empty_cache()
    assert rel(s_poly, s_sum) < 1e-5


def test_polychromatic_rejects(gpu_lib):
    w = torch.zeros((8, 8, 8, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_polychromatic(w, 20e-6, [600e-9], [0.1], [1.0], -1.0)       # out_pitch <= 0
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_polychromatic(w, 20e-6, [600e-9], [0.1], [-1.0], 1e-4)      # negative weight
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_polychromatic(w, 20e-6, [600e-9], [0.1], [1.0], 1e-4, ip=8)  # probe outside
    assert gpu_lib.load().wolf_polychromatic_work_bytes(6, 0) == -1
