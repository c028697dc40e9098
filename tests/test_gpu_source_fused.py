"""The source propagated in one call (wolf_propagate_source): equal, bit for bit, to the source builder
followed by the in-place propagation, whether the half-buffer slab pass forms the source itself
(N = 32 .. 128; GSM or coherent model; no aperture, circle, square or annulus; a lens) or the call
builds the array first (other models and sizes); and within the parity tolerances of the FP64 oracle
(Algorithm 1; Sec. 3.2; Sec. 2.1 eqs. W_fresnel, W_farfield)."""
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
TOL = {torch.complex64: 1e-5, torch.complex128: 1e-12}
DT = [torch.complex64, torch.complex128]


def spec(**kw):
    base = dict(model=WI.MODEL_GSM, amplitude=1.0, sigma_s_m=math.inf, sigma_g_m=math.inf,
                geometry=WI.GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=None, mask=None,
                lens_focal_m=0.0, wavelength_m=0.0)
    base.update(kw)
    return SimpleNamespace(**base)


def rel(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def two_step(gpu_lib, sp, n, p, z, farfield, dtype):
    w = gpu_lib.build_source(sp, n, p, dtype)
    _, dx = gpu_lib.propagate(w, p, LAM, z, farfield, out=w)
    return w, dx


P = 20e-6
# Sources the slab pass forms itself (GEN), one per aperture kind, and sources it does not.
FORMED = {
    "gsm": spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3),
    "gsm_circle_lens": spec(sigma_g_m=0.1e-3, geometry=WI.GEO_CIRCLE, geo_r0_m=9.5 * P, lens_focal_m=0.2,
                            wavelength_m=LAM),
    "coherent_square": spec(model=WI.MODEL_COHERENT, geometry=WI.GEO_SQUARE, geo_r0_m=6 * P),
    "gsm_annulus": spec(sigma_s_m=0.2e-3, sigma_g_m=0.04e-3, geometry=WI.GEO_ANNULUS, geo_r0_m=12 * P,
                        geo_r1_m=5 * P),
}


@pytest.mark.parametrize("farfield", [False, True])
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("name", sorted(FORMED))
def test_formed_source_equals_build_then_propagate(gpu_lib, name, n, dtype, farfield):
    """N = 32, 64 with the half-buffer slab pass set (the default plan there is the whole-slab pass,
    which builds first), over all slabs at once and over groups of 4 i1 planes: both calls run the same
    schedule, and the two schedules give the same bits."""
    sp, z = FORMED[name], 0.3
    res = []
    try:
        for plan in ((3, 0, n * n, 0, 1), (3, 4 * n, 0, 0, 1)):
            gpu_lib.set_plan(n, dtype, *plan)
            a, dxa = gpu_lib.propagate_source(sp, n, P, LAM, z, farfield, dtype=dtype)
            b, dxb = two_step(gpu_lib, sp, n, P, z, farfield, dtype)
            torch.cuda.synchronize()
            assert dxa == dxb
            assert torch.equal(a, b), plan
            res.append(a)
    finally:
        gpu_lib.set_plan(n, dtype)
    assert torch.equal(res[0], res[1])


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("farfield", [False, True])
def test_formed_source_gsm128(gpu_lib, dtype, farfield):
    """The N = 128 GSM workload (2^28 entries): equal to build + propagate, and to the separable
    FP64 oracle within the parity tolerance."""
    wl = WI.gsm128()
    n, p, z, sp = wl.n, wl.pitch_m, wl.z_m, wl.source
    a, _ = gpu_lib.propagate_source(sp, n, p, LAM, z, farfield, dtype=dtype)
    b, _ = two_step(gpu_lib, sp, n, p, z, farfield, dtype)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    del b
    torch.cuda.empty_cache()
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                   O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, LAM, z, farfield)
    assert separable_rel(a, bx, by) < TOL[dtype]
    del a
    torch.cuda.empty_cache()


def test_formed_tophat_lens64_vs_oracle(gpu_lib):
    """The N = 64 top-hat source with a lens (circle aperture, GSM correlation, thin lens), formed by
    the half-buffer slab pass, against the oracle on its own source build."""
    wl = WI.tophat_lens64()
    n, p, sp = wl.n, wl.pitch_m, wl.source
    ref, dxr = O.propagate(O.build_source(sp, n, p), n, p, wl.wavelength_m, wl.z_m)
    for dtype in DT:
        try:
            gpu_lib.set_plan(n, dtype, 3, 0, n * n, 0, 1)
            got, dx = gpu_lib.propagate_source(sp, n, p, wl.wavelength_m, wl.z_m, dtype=dtype)
            torch.cuda.synchronize()
        finally:
            gpu_lib.set_plan(n, dtype)
        assert abs(dx / dxr - 1) < 1e-15
        assert rel(got.cpu().numpy(), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n,name", [(32, "map"), (32, "incoherent"), (32, "mask"), (16, "gsm"), (8, "gsm_circle"),
                                    (32, "gsm")])
def test_built_first_equals_build_then_propagate(gpu_lib, n, name, dtype):
    """Sources and schedules the slab pass does not form (a map, the incoherent model, a mask; N < 32;
    the default whole-slab pass at N = 32)."""
    rng = np.random.default_rng(7)
    sp = {
        "map": spec(model=WI.MODEL_MAP, sigma_g_m=0.06e-3, intensity_map=rng.random((n, n)).astype(np.float32)),
        "incoherent": spec(model=WI.MODEL_INCOHERENT, amplitude=2.0),
        "mask": spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3, geometry=WI.GEO_MASK,
                     mask=(rng.random((n, n)) > 0.3).astype(np.uint8)),
        "gsm": spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3),
        "gsm_circle": spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3, geometry=WI.GEO_CIRCLE, geo_r0_m=3 * P),
    }[name]
    a, _ = gpu_lib.propagate_source(sp, n, P, LAM, 0.2, dtype=dtype)
    b, _ = two_step(gpu_lib, sp, n, P, 0.2, False, dtype)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref, _ = O.propagate(O.build_source(sp, n, P), n, P, LAM, 0.2)
    assert rel(a.cpu().numpy(), ref) < TOL[dtype]


def test_propagate_source_rejects(gpu_lib):
    sp = spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_source(sp, 24, P, LAM, 0.3)  # not a power of two
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_source(sp, 32, P, LAM, -0.3)
    with pytest.raises(gpu_lib.WolfError):
        gpu_lib.propagate_source(spec(model=7), 32, P, LAM, 0.3)


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("name", sorted(FORMED))
def test_formed_by_row_pass_equals_build_then_propagate(gpu_lib, name, n, dtype):
    """The row-pass schedule (fused_slab = 0) over chunks of N slabs, so that launches after the first
    start at a nonzero row: the row pass forms every source decided by the coordinates, with or without
    a lens (N >= 64), and the result equals build + propagate bit for bit."""
    sp, z = FORMED[name], 0.4
    try:
        gpu_lib.set_plan(n, dtype, 0, n, n * n, 0, 1)
        a, _ = gpu_lib.propagate_source(sp, n, P, LAM, z, dtype=dtype)
        b, _ = two_step(gpu_lib, sp, n, P, z, False, dtype)
        torch.cuda.synchronize()
    finally:
        gpu_lib.set_plan(n, dtype)
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()


def test_formed_source_gsm256(gpu_lib):
    """N = 256 complex64 (2^32 entries, 34 GB per array) with the default four-sweep schedule, whose row
    pass forms the source: equal to build + propagate."""
    wl = WI.gsm256()[0]
    n, p, z, sp = wl.n, wl.pitch_m, wl.z_m, wl.source
    a, _ = gpu_lib.propagate_source(sp, n, p, wl.wavelength_m, z)
    b, _ = two_step(gpu_lib, sp, n, p, z, False, torch.complex64)
    torch.cuda.synchronize()
    equal = torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
    assert equal
