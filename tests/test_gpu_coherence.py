"""The degree of coherence (Algorithm 5, eq. defMu, with the floor reading R6) of the HIP path at the
sizes the step runs, against the FP64 oracle.

At N = 64 the spectral density has N^2 = 4096 points (16 workgroups of the max-S reduction), at N = 128
it has 16384 (64 workgroups); in both workloads the maximum of S lies outside the first workgroup, so
the reduction across workgroups sets the floor tau = floor * max S that masks mu.

mu = W / sqrt(S(P1) S(x)) with both S > tau: an error e in W (relative to max |W| = max S) becomes at
most e / sqrt(floor) in mu relative to its own norm, so the tolerance is the W tolerance over
sqrt(floor). The floors are 1e-4 (complex64) and 1e-8 (complex128). The mask must agree exactly,
except on points whose S lies within a small band around tau (FP32 or FP64 rounding of S decides
them): 1e-2 of tau in complex64, 1e-4 in complex128.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle as O
from tests.gpu_util import separable_mu_check
import wolf_inputs as WI

pytestmark = pytest.mark.gpu

LAM = WI.LAMBDA_HENE
TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}
FLOOR = {torch.complex64: 1e-4, torch.complex128: 1e-8}
BAND = {torch.complex64: 1e-2, torch.complex128: 1e-4}
DT = [torch.complex64, torch.complex128]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _mask_and_error(got, ref_mu, s_ref, floor, band, rows=None):
    """Relative L2 error of mu over the points clear of the floor band, and the count of mask
    disagreements there. rows: the P1 indices of a slice (None: full 4D)."""
    tau = floor * s_ref.max()
    ok = s_ref > tau
    clear = np.abs(s_ref / tau - 1) > band
    if rows is None:
        use = clear[:, :, None, None] & clear[None, None, :, :]
        mask = ok[:, :, None, None] & ok[None, None, :, :]
    else:
        ip, jp = rows
        use = clear & bool(clear[ip, jp])
        mask = ok & bool(ok[ip, jp])
    d = (got - ref_mu)[use]
    err = np.linalg.norm(d) / max(np.linalg.norm(ref_mu[use]), 1e-300)
    bad = int(np.sum(use & ~mask & (got != 0)) + np.sum(use & mask & (got == 0) & (np.abs(ref_mu) > 1e-3)))
    return err, bad, mask


@pytest.mark.parametrize("dtype", DT)
def test_mu_tophat_lens64(gpu_lib, dtype):
    """N = 64 top-hat source with a thin lens (f = 0.2 m), Fresnel z = 0.2 m: slices and the full mu
    against the oracle's full 4D W_B. The floor is 1e-3 in both precisions, which leaves about 12 % of
    the points above it; P1 = (20, 41) lies below it (its slice is zero)."""
    wl = WI.tophat_lens64()
    n, p, z = wl.n, wl.pitch_m, wl.z_m
    floor, band = 1e-3, BAND[dtype]
    wb_ref, _ = O.propagate(O.build_source(wl.source, n, p), n, p, LAM, z)
    s_ref = O.spectral_density(wb_ref)
    assert np.argmax(s_ref) >= 256                          # not in the first workgroup of the reduction
    tau = floor * s_ref.max()
    w = gpu_lib.build_source(wl.source, n, p, dtype)
    gpu_lib.propagate_fresnel(w, p, LAM, z, out=w)
    tol = TOL[dtype] / math.sqrt(floor)
    peak = np.unravel_index(np.argmax(s_ref), s_ref.shape)
    probes = [wl.probe, peak, (20, 41), (28, 37)]
    assert any(s_ref[q] > tau for q in probes) and any(s_ref[q] <= tau for q in probes)
    for ip, jp in probes:
        got = host(gpu_lib.degree_of_coherence(w, ip, jp, floor))
        ref = O.degree_of_coherence(wb_ref, ip, jp, floor)
        err, bad, _ = _mask_and_error(got, ref, s_ref, floor, band, rows=(ip, jp))
        assert bad == 0 and err < tol, (ip, jp, err, bad)
        if s_ref[ip, jp] <= tau:
            assert not got.any()
    got = host(gpu_lib.degree_of_coherence(w, -1, -1, floor))
    ref = O.degree_of_coherence_full(wb_ref, floor)
    err, bad, mask = _mask_and_error(got, ref, s_ref, floor, band)
    assert 0.001 < mask.mean() < 0.5
    assert bad == 0 and err < tol, (err, bad)


@pytest.mark.parametrize("dtype", DT)
def test_mu_gsm128(gpu_lib, dtype):
    """N = 128 GSM (the step's workload): slices and the full 2^28-entry mu against the separable oracle,
    compared one first-point row at a time."""
    wl = WI.gsm128()
    n, p, z = wl.n, wl.pitch_m, wl.z_m
    sp = wl.source
    floor, band = FLOOR[dtype], BAND[dtype]
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                   O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, LAM, z)
    s_ref = np.real(np.diag(bx))[:, None] * np.real(np.diag(by))[None, :]
    assert np.argmax(s_ref) >= 256
    w = gpu_lib.build_source(sp, n, p, dtype)
    gpu_lib.propagate_fresnel(w, p, LAM, z, out=w)
    tol = TOL[dtype] / math.sqrt(floor)
    for ip, jp in [wl.probe, (70, 50), (64, 100)]:
        got = host(gpu_lib.degree_of_coherence(w, ip, jp, floor))
        row = bx[ip][:, None] * by[jp][None, :]
        tau = floor * s_ref.max()
        ref = np.where((s_ref > tau) & (s_ref[ip, jp] > tau), row / np.sqrt(s_ref[ip, jp] * np.maximum(s_ref, 1e-300)),
                       0)
        err, bad, _ = _mask_and_error(got, ref, s_ref, floor, band, rows=(ip, jp))
        assert bad == 0 and err < tol, (ip, jp, err, bad)
    mu = gpu_lib.degree_of_coherence(w, -1, -1, floor)
    del w
    err, bad = separable_mu_check(mu, bx, by, floor, band)
    assert bad == 0 and err < tol, (err, bad)
    del mu
    torch.cuda.empty_cache()


def test_mu_scratch_is_not_allocated_under_capture(gpu_lib):
    """The library allocates its per-stream scratch only outside graph capture: the first mu call on a
    stream that is being captured fails with WOLF_EINVAL and records nothing; after one call outside
    capture the same call can be captured, and the replayed graph gives the eager result each time."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    n, p = 16, 20e-6
    sp = WI.gsm_small()[0].source
    w = gpu_lib.build_source(sp, n, p, torch.complex64)
    mu = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    hs = ctypes.c_void_p(s.cuda_stream)
    graph = ctypes.c_void_p()
    with torch.cuda.stream(s):
        assert hip.hipStreamBeginCapture(hs, 2) == 0                      # relaxed mode
        try:
            with pytest.raises(gpu_lib.WolfError) as err:
                gpu_lib.degree_of_coherence(w, 8, 8, out=mu)
            assert err.value.status == gpu_lib.EINVAL
        finally:
            assert hip.hipStreamEndCapture(hs, ctypes.byref(graph)) == 0
            hip.hipGraphDestroy(graph)
        eager = gpu_lib.degree_of_coherence(w, 8, 8).clone()               # allocates the scratch
        s.synchronize()
        assert hip.hipStreamBeginCapture(hs, 2) == 0
        try:
            gpu_lib.degree_of_coherence(w, 8, 8, out=mu)
        finally:
            assert hip.hipStreamEndCapture(hs, ctypes.byref(graph)) == 0
        exe = ctypes.c_void_p()
        assert hip.hipGraphInstantiate(ctypes.byref(exe), graph, None, None, ctypes.c_size_t(0)) == 0
        try:
            for _ in range(3):
                mu.zero_()
                assert hip.hipGraphLaunch(exe, hs) == 0
                s.synchronize()
                assert torch.equal(mu, eager)
                gpu_lib.degree_of_coherence(w, 4, 4)                       # eager work between replays
                s.synchronize()
        finally:
            hip.hipGraphExecDestroy(exe)
            hip.hipGraphDestroy(graph)
