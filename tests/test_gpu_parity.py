"""Parity of the HIP path (through the C-ABI, via the ctypes binding) with the FP64 oracle.

Tolerances:
  complex128: 1e-12 relative L2. Rounding of the O(log N) FFT stages is ~1e-15. The chirp phases
              reach ~1e4 rad and are rounded in FP64 (~1e-12 rad at most).
  complex64:  1e-5 relative L2 over all N^4 entries (the accuracy target of the complex64 path).
              FP32 butterflies give ~6e-8 sqrt(log2 N^2) per entry, and the FP64-built tables are
              rounded to FP32 once.
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np
import pytest
import torch

import oracle as O
from tests.gpu_util import separable_rel
import wolf_inputs as WI

pytestmark = pytest.mark.gpu

LAM = WI.LAMBDA_HENE
TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}
DT = [torch.complex64, torch.complex128]


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def spec(**kw):
    base = dict(model=WI.MODEL_GSM, amplitude=1.0, sigma_s_m=math.inf, sigma_g_m=math.inf,
                geometry=WI.GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=None, mask=None,
                lens_focal_m=0.0, wavelength_m=0.0)
    base.update(kw)
    return SimpleNamespace(**base)


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ---------------------------------------------------------------------------------------------
# a0: FP64 chirp tables
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,pitch,z", [(16, 20e-6, 0.5), (128, 20e-6, 0.5), (256, 10e-6, 0.1), (128, 20e-6, 5.0)])
def test_chirp_table(gpu_lib, n, pitch, z):
    ref = O.chirp_table(n, pitch, LAM, z)
    t128 = host(gpu_lib.chirp_table(n, pitch, LAM, z, torch.complex128))
    assert np.abs(t128 - ref).max() < 1e-11
    t64 = host(gpu_lib.chirp_table(n, pitch, LAM, z, torch.complex64))
    # FP64 value rounded once to FP32: within one FP32 ulp (|q| = 1) of the oracle.
    assert np.abs(t64.real - ref.real).max() <= 6e-8 and np.abs(t64.imag - ref.imag).max() <= 6e-8


# ---------------------------------------------------------------------------------------------
# a1: source builder
# ---------------------------------------------------------------------------------------------
SOURCES = {
    "gsm": dict(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3, amplitude=1.7),
    "gsm_uniform_coherent": dict(),
    "circle_lens": dict(sigma_g_m=0.1e-3, geometry=WI.GEO_CIRCLE, geo_r0_m=0.1e-3, lens_focal_m=0.2, wavelength_m=LAM),
    "square": dict(sigma_s_m=0.2e-3, sigma_g_m=0.08e-3, geometry=WI.GEO_SQUARE, geo_r0_m=0.08e-3),
    "annulus_incoherent": dict(model=WI.MODEL_INCOHERENT, amplitude=2.0, geometry=WI.GEO_ANNULUS, geo_r0_m=0.12e-3,
                               geo_r1_m=0.04e-3),
    "coherent_mask": dict(model=WI.MODEL_COHERENT, geometry=WI.GEO_MASK, mask=WI.random_mask(16, 3)),
    "map": dict(model=WI.MODEL_MAP, sigma_g_m=0.06e-3, intensity_map=WI.intensity_map(16, 20e-6, 4)),
}


@pytest.mark.parametrize("name", list(SOURCES))
@pytest.mark.parametrize("dtype", DT)
def test_build_source(gpu_lib, name, dtype):
    n, p = 16, 20e-6
    sp = spec(**SOURCES[name])
    got = host(gpu_lib.build_source(sp, n, p, dtype))
    ref = O.build_source(sp, n, p)
    assert rel(got, ref) < (1e-14 if dtype == torch.complex128 else 2e-7)
    # Geometry decisions are identical on both sides.
    assert np.array_equal(np.abs(got) > 0, np.abs(ref) > 0)


def test_build_source_circle_boundary(gpu_lib):
    """0.4 mm radius at 20 um pitch is exactly 20 px: boundary pixels are inside on both sides."""
    n, p = 64, 20e-6
    sp = spec(model=WI.MODEL_INCOHERENT, geometry=WI.GEO_CIRCLE, geo_r0_m=0.4e-3)
    got = host(gpu_lib.build_source(sp, n, p, torch.complex64))
    s = np.real(np.einsum("ijij->ij", got))
    ref = O.geometry_mask(n, p, O.GEO_CIRCLE, 0.4e-3)
    assert np.array_equal(s > 0, ref > 0) and s[32 + 20, 32] == 1 and s[32 + 12, 32 + 16] == 1


# ---------------------------------------------------------------------------------------------
# a2-a4: propagation (Fresnel and far field) on random and physical sources, small N
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 4, 8, 16, 32])
@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", DT)
def test_propagate_random(gpu_lib, n, farfield, dtype):
    p, z = 20e-6, 0.05
    w = WI.random_complex((n, n, n, n), seed=10 + n)
    ref, dx = O.propagate(w, n, p, LAM, z, farfield)
    got, gdx = gpu_lib.propagate(dev(w, dtype), p, LAM, z, farfield)
    assert gdx == pytest.approx(dx, rel=1e-15)
    assert rel(host(got), ref) < TOL[dtype]


@pytest.mark.parametrize("kind", [WI.KIND_SECONDARY, WI.KIND_PRIMARY])
def test_propagate_kind(gpu_lib, kind):
    n, p, z = 8, 20e-6, 0.1
    w = WI.random_hermitian_psd(n, seed=3)
    ref, _ = O.propagate(w, n, p, LAM, z, False, kind)
    got, _ = gpu_lib.propagate_fresnel(dev(w, torch.complex128), p, LAM, z, kind)
    assert rel(host(got), ref) < 1e-12


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", DT)
def test_propagate_gsm64(gpu_lib, farfield, dtype):
    """N = 64 from the GPU source builder; oracle on its own source build."""
    n, p, z = 64, 20e-6, 0.3
    sp = spec(sigma_s_m=0.08e-3, sigma_g_m=0.12e-3)
    w = gpu_lib.build_source(sp, n, p, dtype)
    got, _ = gpu_lib.propagate(w, p, LAM, z, farfield)
    ref, _ = O.propagate(O.build_source(sp, n, p), n, p, LAM, z, farfield)
    assert rel(host(got), ref) < TOL[dtype]


def test_propagate_tophat_lens64(gpu_lib):
    """Circular top-hat (20 px), Gaussian mu, thin lens f = 0.2 m, Fresnel z = 0.2 m, N = 64."""
    wl = WI.tophat_lens64()
    n, p = wl.n, wl.pitch_m
    sp = wl.source
    ref, _ = O.propagate(O.build_source(sp, n, p), n, p, wl.wavelength_m, wl.z_m)
    for dtype in DT:
        got, _ = gpu_lib.propagate_fresnel(gpu_lib.build_source(sp, n, p, dtype), p, wl.wavelength_m, wl.z_m)
        assert rel(host(got), ref) < TOL[dtype]


def test_in_place_equals_out_of_place(gpu_lib):
    n, p, z = 16, 20e-6, 0.2
    w = dev(WI.random_complex((n, n, n, n), seed=21), torch.complex64)
    a, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
    b = w.clone()
    gpu_lib.propagate_fresnel(b, p, LAM, z, out=b)
    assert torch.equal(a, b)


def test_deterministic(gpu_lib):
    n, p, z = 32, 20e-6, 0.2
    w = dev(WI.random_complex((n, n, n, n), seed=22), torch.complex64)
    a, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
    b, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------------------------
# a5-a6: observables
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DT)
def test_observables(gpu_lib, dtype):
    n, p, z = 16, 20e-6, 0.5
    sp = spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
    wb_ref, _ = O.propagate(O.build_source(sp, n, p), n, p, LAM, z)
    wb, _ = gpu_lib.propagate_fresnel(gpu_lib.build_source(sp, n, p, dtype), p, LAM, z)
    s = host(gpu_lib.spectral_density(wb))
    assert rel(s, O.spectral_density(wb_ref)) < TOL[dtype]
    mu = host(gpu_lib.degree_of_coherence(wb, 8, 8))
    mu_ref = O.degree_of_coherence(wb_ref, 8, 8)
    assert rel(mu, mu_ref) < 10 * TOL[dtype]
    assert np.abs(mu).max() <= 1 + (1e-6 if dtype == torch.complex64 else 1e-12)
    full = host(gpu_lib.degree_of_coherence(wb))
    assert rel(full, O.degree_of_coherence_full(wb_ref)) < 10 * TOL[dtype]


def test_coherence_floor_masks_dark_points(gpu_lib):
    n, p = 16, 20e-6
    sp = spec(model=WI.MODEL_COHERENT, geometry=WI.GEO_CIRCLE, geo_r0_m=4 * p)
    w = gpu_lib.build_source(sp, n, p, torch.complex128)
    mu = host(gpu_lib.degree_of_coherence(w, 8, 8))
    assert np.array_equal(mu, O.degree_of_coherence(O.build_source(sp, n, p), 8, 8))
    assert not host(gpu_lib.degree_of_coherence(w, 0, 0)).any()


# ---------------------------------------------------------------------------------------------
# a7: adjoint
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", DT)
def test_adjoint_vs_oracle(gpu_lib, farfield, dtype):
    n, p, z = 16, 20e-6, 0.1
    g = WI.random_complex((n, n, n, n), seed=31)
    ref = O.propagate_adjoint(g, n, p, LAM, z, farfield)
    got = gpu_lib.propagate_adjoint(dev(g, dtype), p, LAM, z, farfield)
    assert rel(host(got), ref) < TOL[dtype]


def test_adjoint_dot_product_gpu(gpu_lib):
    n, p, z = 16, 20e-6, 0.1
    w = dev(WI.random_complex((n, n, n, n), seed=41), torch.complex128)
    g = dev(WI.random_complex((n, n, n, n), seed=42), torch.complex128)
    pw, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
    pg = gpu_lib.propagate_adjoint(g, p, LAM, z)
    lhs = torch.vdot(pw.flatten(), g.flatten()).item()
    rhs = torch.vdot(w.flatten(), pg.flatten()).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", DT)
def test_adjoint_full_size_n128(gpu_lib, farfield, dtype):
    """The adjoint at N = 128 (the size the step's adjoint runs at: the half-buffer slab pass with the
    inverse DFT and the first-point passes with the direct DFT), all 2^28 entries, on a separable
    random input G_B = gx (x) gy against the oracle's separable adjoint."""
    n, p, z = 128, 20e-6, 0.5
    r = WI.rng(93)
    gx = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    gy = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    ax, ay = O.propagate_adjoint_separable(gx, gy, n, p, LAM, z, farfield)
    gxt = torch.from_numpy(gx).to(dtype).cuda()
    gyt = torch.from_numpy(gy).to(dtype).cuda()
    g = (gxt[:, None, :, None] * gyt[None, :, None, :]).contiguous()
    got = gpu_lib.propagate_adjoint(g, p, LAM, z, farfield, out=g)       # in place, as the step runs it
    assert _separable_rel(got, ax, ay) < TOL[dtype]
    del g, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n", [32, 64])
def test_autotune_keeps_a_valid_plan(gpu_lib, n, dtype):
    """wolf_autotune times the candidate schedules and keeps the fastest: get_plan returns that plan,
    set_plan accepts it again, and the propagation under it matches the oracle."""
    p, z = 20e-6, 0.1
    try:
        plan, best = gpu_lib.autotune(n, dtype, reps=1)
        assert best > 0 and math.isfinite(best)
        assert gpu_lib.get_plan(n, dtype) == plan
        assert plan["fused_slab"] in (0, 1, 2, 3)
        gpu_lib.set_plan(n, dtype, plan["fused_slab"], plan["slab_chunk"], plan["col_chunk"], plan["coop_cols"],
                         plan["coop_lookahead"])
        assert gpu_lib.get_plan(n, dtype) == plan
        if n == 32:
            w = WI.random_complex((n, n, n, n), seed=52)
            ref, _ = O.propagate(w, n, p, LAM, z)
            got, _ = gpu_lib.propagate_fresnel(dev(w, dtype), p, LAM, z)
            assert rel(host(got), ref) < TOL[dtype]
        else:
            sp = spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
            bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                           O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, LAM, z)
            w = gpu_lib.build_source(sp, n, p, dtype)
            gpu_lib.propagate_fresnel(w, p, LAM, z, out=w)
            assert _separable_rel(w, bx, by) < TOL[dtype]
    finally:
        gpu_lib.set_plan(n, dtype)


@pytest.mark.parametrize("dtype", DT)
def test_nan_input_propagates_without_error(gpu_lib, dtype):
    """A NaN in the input spreads through the transforms (no crash, no error status), S and mu are
    computed, and the next call on clean data is correct (no sticky error)."""
    n, p, z = 16, 20e-6, 0.1
    w = WI.random_complex((n, n, n, n), seed=53)
    bad = w.copy()
    bad[3, 4, 5, 6] = np.nan
    out, _ = gpu_lib.propagate_fresnel(dev(bad, dtype), p, LAM, z)
    o = host(out)
    assert np.isnan(o).all()                     # every output entry depends on every input entry
    host(gpu_lib.spectral_density(out))
    mu = host(gpu_lib.degree_of_coherence(out, 8, 8))
    assert not np.isinf(mu).any()
    ref, _ = O.propagate(w, n, p, LAM, z)
    got, _ = gpu_lib.propagate_fresnel(dev(w, dtype), p, LAM, z)
    assert rel(host(got), ref) < TOL[dtype]


# ---------------------------------------------------------------------------------------------
# Full-size workloads (N = 128 headline; N = 256), every entry against the separable oracle.
# The GSM source is separable, so the oracle's output is bx[m1, m2] by[n1, n2]. The test forms
# those products one slab at a time and compares them with the GPU output.
# ---------------------------------------------------------------------------------------------
_separable_rel = separable_rel


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", DT)
def test_full_size_gsm128(gpu_lib, farfield, dtype):
    wl = WI.gsm128()
    n, p, z = wl.n, wl.pitch_m, wl.z_m
    sp = wl.source
    w = gpu_lib.build_source(sp, n, p, dtype)
    gpu_lib.propagate(w, p, LAM, z, farfield, out=w)
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                   O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, LAM, z, farfield)
    assert _separable_rel(w, bx, by) < TOL[dtype]
    del w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("farfield,dtype", [(False, torch.complex64), (True, torch.complex64),
                                             (False, torch.complex128)])
def test_full_size_gsm256(gpu_lib, farfield, dtype):
    """N = 256 (2^32 elements: 34 GB in complex64, 69 GB in complex128), in place, every entry against
    the separable oracle. At this size the slab does not fit the LDS, so the row and axis passes run."""
    wl = WI.gsm256()[1 if farfield else 0]
    n, p, z = wl.n, wl.pitch_m, wl.z_m
    sp = wl.source
    w = gpu_lib.build_source(sp, n, p, dtype)
    gpu_lib.propagate(w, p, LAM, z, farfield, out=w)
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                   O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, LAM, z, farfield)
    assert _separable_rel(w, bx, by) < TOL[dtype]
    del w
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------------------------
# Every pass schedule gives the same operator (fused slab or row + i2 passes; any chunking).
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DT)
def test_all_schedules_agree(gpu_lib, dtype):
    n, p, z = 32, 20e-6, 0.05
    w = WI.random_complex((n, n, n, n), seed=51)
    ref, _ = O.propagate(w, n, p, LAM, z)
    adj_ref = O.propagate_adjoint(w, n, p, LAM, z)
    nn = n * n
    c = 256 // 4 if 256 // 4 < n else n       # axis tile at N = 32 (N2 = 4)
    plans = [(1, 0, 0, 0, 1), (1, 0, c, 0, 1), (1, 0, nn // 2, 0, 1), (0, 0, 0, 0, 1), (0, nn // 4, c, 0, 1),
             (0, 2, nn // 8, 0, 1), (2, 0, 0, 0, 1), (2, 0, c, 0, 1), (3, 0, 0, 0, 1), (3, 0, c, 0, 1),
             # grouped: slab pass + j1 pass over groups of i1 planes, then the i1 pass
             (3, 4 * n, 0, 0, 1), (1, 8 * n, c, 0, 1), (2, 2 * n, nn // 2, 0, 1), (3, n, nn // 4, 0, 1)]
    try:
        for plan in plans:
            gpu_lib.set_plan(n, dtype, *plan)
            got, _ = gpu_lib.propagate_fresnel(dev(w, dtype), p, LAM, z)
            assert rel(host(got), ref) < TOL[dtype], plan
            adj = gpu_lib.propagate_adjoint(dev(w, dtype), p, LAM, z)
            assert rel(host(adj), adj_ref) < TOL[dtype], plan
            x = dev(w, dtype)  # in place: the grouped plans take their grouped schedule only here
            gpu_lib.propagate_fresnel(x, p, LAM, z, out=x)
            assert torch.equal(x, got), plan
            x = dev(w, dtype)
            gpu_lib.propagate_adjoint(x, p, LAM, z, out=x)
            assert torch.equal(x, adj), plan
            assert gpu_lib.coop_error_flag() == 0, plan
    finally:
        gpu_lib.set_plan(n, dtype)


@pytest.mark.parametrize("n,dtype", [(16, torch.complex64), (64, torch.complex64), (128, torch.complex64),
                                     (16, torch.complex128), (64, torch.complex128)])
def test_persistent_slab_pass_matches_per_slab(gpu_lib, n, dtype):
    """The persistent slab pass (fused_slab = 2, grid-stride over slabs with the next slab in flight)
    runs the same arithmetic as one workgroup per slab, so the outputs agree to rounding (in practice
    bit for bit). At N = 128 each workgroup takes 64 slabs."""
    p, z = 20e-6, 0.5
    if n == 128:
        w = gpu_lib.build_source(WI.gsm128().source, n, p, dtype)
    else:
        w = dev(WI.random_complex((n, n, n, n), seed=60 + n), dtype)
    nn = n * n
    outs = []
    try:
        for mode in (1, 2):
            gpu_lib.set_plan(n, dtype, mode, 0, nn, 0, 1)
            got, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
            outs.append(got)
    finally:
        gpu_lib.set_plan(n, dtype)
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(outs[1] - outs[0]) / torch.linalg.vector_norm(outs[0]))
    assert d <= (1e-6 if dtype == torch.complex64 else 1e-14), d


@pytest.mark.parametrize("n,dtype", [(32, torch.complex64), (64, torch.complex64), (128, torch.complex64),
                                     (32, torch.complex128), (64, torch.complex128)])
def test_half_buffer_slab_pass_matches_per_slab(gpu_lib, n, dtype):
    """The slab pass through a half-size LDS buffer (fused_slab = 3) does the same arithmetic as the
    whole-slab pass: the outputs agree to rounding."""
    p, z = 20e-6, 0.5
    if n == 128:
        w = gpu_lib.build_source(WI.gsm128().source, n, p, dtype)
    else:
        w = dev(WI.random_complex((n, n, n, n), seed=61 + n), dtype)
    nn = n * n
    outs = []
    try:
        for mode in (1, 3):
            gpu_lib.set_plan(n, dtype, mode, 0, nn, 0, 1)
            got, _ = gpu_lib.propagate_fresnel(w, p, LAM, z)
            outs.append(got)
    finally:
        gpu_lib.set_plan(n, dtype)
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(outs[1] - outs[0]) / torch.linalg.vector_norm(outs[0]))
    assert d <= (1e-6 if dtype == torch.complex64 else 1e-14), d


@pytest.mark.parametrize("dtype", DT)
def test_grouped_schedule_full_size(gpu_lib, dtype):
    """N = 128 GSM at full size: the slab pass and the j1 pass over groups of 16 and of 4 i1 planes
    (the complex64 default is 16) give the same bits as the slab pass over all slabs followed by the
    paired j1/i1 column chunks, with a random input (no symmetry to hide a misplaced group)."""
    n, p, z = 128, 20e-6, 0.5
    w0 = dev(WI.random_complex((n, n, n, n), seed=91, dtype=np.complex64 if dtype == torch.complex64
                               else np.complex128), dtype)
    outs = []
    try:
        for plan in ((3, 0, 1024, 0, 1), (3, 16 * n, n * n, 0, 1), (3, 4 * n, 4096, 0, 1)):
            gpu_lib.set_plan(n, dtype, *plan)
            print("plan", dtype, plan, flush=True)
            x = w0.clone()
            gpu_lib.propagate_fresnel(x, p, LAM, z, out=x)
            outs.append(x.cpu())
            del x
            torch.cuda.empty_cache()
    finally:
        gpu_lib.set_plan(n, dtype)
    del w0
    torch.cuda.empty_cache()
    assert torch.equal(outs[0], outs[1])
    assert torch.equal(outs[0], outs[2])


def test_complex128_n128_uses_the_half_buffer_slab_pass(gpu_lib):
    """complex128 at N = 128: the whole slab (256 KB) does not fit the LDS; the default plan takes the
    half-buffer slab pass (3 sweeps instead of 4). Full-size parity is test_full_size_gsm128."""
    assert gpu_lib.get_plan(128, torch.complex128)["fused_slab"] == 3


COOP_COLS = {torch.complex64: (8, 16, 32), torch.complex128: (4, 8, 16)}


@pytest.mark.parametrize("dtype", DT)
def test_cooperative_schedules_agree(gpu_lib, dtype):
    """The cooperative first-point pass (one sweep for j1 and i1, tiles through the L2 of one XCD) at
    N = 32 on a random input, for every tile width and several lookaheads, after the whole-slab and the
    row passes, against the oracle; no bounded wait runs out."""
    n, p, z = 32, 20e-6, 0.05
    w = WI.random_complex((n, n, n, n), seed=51)
    ref, _ = O.propagate(w, n, p, LAM, z)
    c = COOP_COLS[dtype]
    try:
        for plan in [(1, 0, 0, c[0], 1), (1, 0, 0, c[1], 2), (1, 0, 0, c[2], 8), (0, 0, 0, c[1], 1),
                     (3, 0, 0, c[0], 1)]:
            print("coop plan", dtype, plan, flush=True)
            gpu_lib.set_plan(n, dtype, *plan)
            assert gpu_lib.get_plan(n, dtype)["coop_cols"] == plan[3]
            got, _ = gpu_lib.propagate_fresnel(dev(w, dtype), p, LAM, z)
            assert gpu_lib.coop_error_flag() == 0, plan
            assert rel(host(got), ref) < TOL[dtype], plan
    finally:
        gpu_lib.set_plan(n, dtype)


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n", [64, 128])
def test_cooperative_pass_full_size(gpu_lib, dtype, n):
    """The cooperative first-point pass against the two-pass schedule and against the oracle, on GSM
    sources at full size (every tile width that fits the 2 MB tile limit), in place."""
    wl = WI.gsm128()
    p, z = wl.pitch_m, wl.z_m
    sp = wl.source
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                   O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, LAM, z)
    base = gpu_lib.get_plan(n, dtype)
    try:
        b = gpu_lib.build_source(sp, n, p, dtype)
        gpu_lib.propagate_fresnel(b, p, LAM, z, out=b)                 # the default (two-pass) schedule
        for cols in COOP_COLS[dtype]:
            if n * n * cols * (8 if dtype == torch.complex64 else 16) > (2 << 20):
                continue
            print("coop full size", n, dtype, cols, flush=True)
            gpu_lib.set_plan(n, dtype, base["fused_slab"], base["slab_chunk"], 0, cols, 1)
            a = gpu_lib.build_source(sp, n, p, dtype)
            gpu_lib.propagate_fresnel(a, p, LAM, z, out=a)
            assert gpu_lib.coop_error_flag() == 0
            d = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
            assert d <= (1e-6 if dtype == torch.complex64 else 1e-14), (cols, d)
            assert _separable_rel(a, bx, by) < TOL[dtype]
            del a
            torch.cuda.empty_cache()
    finally:
        gpu_lib.set_plan(n, dtype)


@pytest.mark.parametrize("dtype", DT)
def test_cooperative_pass_adjoint_and_source(gpu_lib, dtype):
    """The cooperative pass in the adjoint (inverse DFT signs swapped) and in the one-call source
    propagation (the slab pass forms the source), N = 64, against the oracle and the two-pass form."""
    n, p, z = 64, 20e-6, 0.3
    g = WI.random_complex((n, n, n, n), seed=54)
    ref = O.propagate_adjoint(g, n, p, LAM, z)
    sp = spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
    two, _ = gpu_lib.propagate_source(sp, n, p, LAM, z, dtype=dtype)
    try:
        gpu_lib.set_plan(n, dtype, 3, 0, 0, COOP_COLS[dtype][1], 1)
        got = gpu_lib.propagate_adjoint(dev(g, dtype), p, LAM, z)
        assert gpu_lib.coop_error_flag() == 0
        assert rel(host(got), ref) < TOL[dtype]
        one, _ = gpu_lib.propagate_source(sp, n, p, LAM, z, dtype=dtype)
        assert gpu_lib.coop_error_flag() == 0
        d = float(torch.linalg.vector_norm(one - two) / torch.linalg.vector_norm(two))
        assert d <= (1e-6 if dtype == torch.complex64 else 1e-14), d
    finally:
        gpu_lib.set_plan(n, dtype)


def test_invalid_plan_rejected(gpu_lib):
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.set_plan(128, torch.complex128, 1, 0, 0)      # slab does not fit LDS in complex128
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.set_plan(64, torch.complex64, 1, 0, 3)        # chunk not a divisor
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.set_plan(32, torch.complex64, 0, 1, 0)        # one slab is less than a row-pass workgroup
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.set_plan(64, torch.complex64, 1, 0, 0, 12, 1)      # cooperative tile of 12 columns


def test_overlapping_buffers_rejected(gpu_lib):
    n = 8
    big = torch.zeros((2 * n ** 4,), dtype=torch.complex64, device="cuda")
    w = big[: n ** 4].view(n, n, n, n)
    shifted = big[17: 17 + n ** 4].view(n, n, n, n)
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_fresnel(w, 20e-6, LAM, 0.1, out=shifted)           # partial overlap
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.degree_of_coherence(w, 1, 1, out=big[5: 5 + n * n].view(n, n))   # mu inside w
    # A buffer one element short of N^4, in an allocation of its own (torch's caching allocator would
    # place it inside a larger segment).
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    ptr = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(8 * (n ** 4 - 1))) == 0
    try:
        lib = gpu_lib.load()
        assert lib.wolf_propagate_fresnel(ptr, ptr, n, 20e-6, LAM, 0.1, 0, 0, None, None) == -1
        assert b"too small" in lib.wolf_last_error_message()
    finally:
        hip.hipFree(ptr)


def test_binding_rejects_mismatched_outputs(gpu_lib):
    """Every binding checks a caller's `out` against the call (shape, dtype, device) and the map and
    mask against N before anything is launched: a mis-sized tensor inside a larger caching-allocator
    segment would otherwise be written past its end."""
    n, p = 16, 20e-6
    sp = spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
    w = gpu_lib.build_source(sp, n, p, torch.complex64)
    small = torch.empty((8, 8, 8, 8), dtype=torch.complex64, device="cuda")
    wrong = torch.empty((n, n, n, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        gpu_lib.build_source(sp, n, p, out=small)
    with pytest.raises(ValueError):
        gpu_lib.propagate_source(sp, n, p, LAM, 0.1, out=small)
    with pytest.raises(ValueError):
        gpu_lib.propagate_fresnel(w, p, LAM, 0.1, out=wrong)
    with pytest.raises(ValueError):
        gpu_lib.propagate_adjoint(w, p, LAM, 0.1, out=small)
    with pytest.raises(ValueError):
        gpu_lib.propagate_adjoint(w, p, LAM, 0.1, out=wrong)
    g = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        gpu_lib.propagate_adjoint_diag(g, p, LAM, 0.1, out=small)
    with pytest.raises(ValueError):
        gpu_lib.spectral_density(w, out=torch.empty((n, n), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        gpu_lib.spectral_density(w, out=torch.empty((8, 8), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        gpu_lib.degree_of_coherence(w, 1, 1, out=torch.empty((n, n, n, n), dtype=torch.complex64, device="cuda"))
    with pytest.raises(ValueError):
        gpu_lib.degree_of_coherence(w, -1, -1, out=torch.empty((n, n), dtype=torch.complex64, device="cuda"))
    with pytest.raises(ValueError):
        gpu_lib.build_source(spec(model=WI.MODEL_MAP, sigma_g_m=0.05e-3, intensity_map=np.ones((8, 8))), n, p)
    with pytest.raises(ValueError):
        gpu_lib.build_source(spec(geometry=WI.GEO_MASK, mask=np.ones((n, n + 1))), n, p)
    # The correct tensors still work.
    s = gpu_lib.spectral_density(w, out=torch.empty((n, n), dtype=torch.float32, device="cuda"))
    assert torch.isfinite(s).all()
