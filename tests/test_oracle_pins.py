"""Pins of the FP64 oracle against results that do not come from the oracle itself.

Each test names the mistake in the oracle that it would catch.
"""
from __future__ import annotations

import json
import math
import os
from types import SimpleNamespace

import mpmath
import numpy as np
import pytest

import oracle as O
import wolf_inputs as WI
from tests import closed_forms as CF

HERE = os.path.dirname(os.path.abspath(__file__))
LAM = 632.8e-9


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def spec(**kw):
    base = dict(model=O.MODEL_GSM, amplitude=1.0, sigma_s_m=math.inf, sigma_g_m=math.inf,
                geometry=O.GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=None, mask=None,
                lens_focal_m=0.0, wavelength_m=0.0)
    base.update(kw)
    return SimpleNamespace(**base)


# ---------------------------------------------------------------------------------------------
# The paper's printed numbers (Table 1 and Sec. 5): units, dx, N_a, N_F.
# Catches: a wrong omega/lambda relation or a wrong dx formula (N vs N_z, missing 2 pi).
# ---------------------------------------------------------------------------------------------
def test_paper_printed_numbers():
    g = json.load(open(os.path.join(HERE, "golden", "paper_examples.json")))
    e1 = g["ex1_fresnel_square"]
    lam1 = O.wavelength_from_omega(e1["omega_rad_s"])
    assert round(lam1 / 1e-10, 1) == e1["printed"]["lambda_angstrom"]
    assert round(math.sqrt(2 * math.pi * e1["Nz"])) == e1["printed"]["Na_from_sqrt_2piNz"]
    a = e1["Na"] * e1["dxi_m"]
    assert round(a / 1e-6, 1) == e1["printed"]["a_um"]
    assert round(O.fresnel_number(a, lam1, e1["R_m"]), 2) == e1["printed"]["fresnel_number"]
    # Dark-spot distance R = a^2 / (2 pi lambda) (eq. darkspot): the paper's R to 1%.
    assert abs(a * a / (2 * math.pi * lam1) / e1["R_m"] - 1) < 0.01

    e3 = g["ex3_imaging"]
    lam3 = O.wavelength_from_omega(e3["omega_rad_s"])
    dxb = O.output_pitch(e3["N"], e3["dxi_m"], lam3, e3["R1_m"])
    assert round(dxb / 1e-3, 2) == e3["printed"]["dx_planeB_mm"]
    dxc = O.output_pitch(e3["N"], dxb, lam3, e3["R2_m"])           # plane B -> plane C
    assert round(dxc / 1e-6, 3) == e3["printed"]["dxi_planeC_um"]
    # Lens law (eq. imaging) and magnification -R2/R1.
    assert abs(1 / e3["R1_m"] + 1 / e3["R2_m"] - 1 / e3["f_m"]) < 1e-12
    assert -e3["R2_m"] / e3["R1_m"] == e3["printed"]["lateral_magnification"]

    e4 = g["ex4_gsm_beam"]
    lam4 = O.wavelength_from_omega(e4["omega_rad_s"])
    assert round(lam4 / 1e-9 / 10) * 10 == e4["printed"]["lambda_nm"]
    dx4 = O.output_pitch(e4["N"], e4["dxi_m"], lam4, e4["R_m"])
    assert abs(dx4 / e4["dxi_m"] - 1) < 1e-3 and e4["printed"]["dx_equals_dxi"]


# ---------------------------------------------------------------------------------------------
# Closed-form Gaussian Schell-model propagation (Sec. 5.4; Mandel-Wolf beam).
# Catches: a wrong scale C, a wrong chirp sign (the k (x2^2 - x1^2) / 2R phase), a wrong dx,
# or a wrong source width convention (4 sS^2 vs 2 sS^2).
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_gsm_closed_form_4d(farfield):
    n, p, ss, sg, z = 64, 20e-6, 0.08e-3, 0.12e-3, 0.3
    w = O.build_source(spec(sigma_s_m=ss, sigma_g_m=sg), n, p)
    wb, dx = O.propagate(w, n, p, LAM, z, farfield)
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], ss, sg, LAM, z, farfield)
    cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], ss, sg, LAM, z, farfield)
    ref = cx[:, None, :, None] * cy[None, :, None, :]
    assert rel(wb, ref) < 1e-9


@pytest.mark.parametrize("farfield", [False, True])
def test_gsm_closed_form_separable_n128(farfield):
    n, p, ss, sg, z = 128, 20e-6, 0.1e-3, 0.05e-3, 0.5
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, ss, sg, "x"),
                                   O.gsm_axis_factor(n, p, ss, sg, "y"), n, p, LAM, z, farfield)
    dx = O.output_pitch(n, p, LAM, z)
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], ss, sg, LAM, z, farfield)
    cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], ss, sg, LAM, z, farfield)
    assert rel(np.kron(bx, by), np.kron(cx, cy)) < 1e-11


# ---------------------------------------------------------------------------------------------
# A tilted, off-centre coherent Gaussian beam (rank-1 W = U* (x) U), exact Gaussian integral.
# Catches: the transform direction (conj kernel on the wrong point), the y flip applied on one
# side only, or a transposed operand; each moves the beam the wrong way.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_tilted_beam_closed_form(farfield):
    n, p, w0, z = 64, 20e-6, 80e-6, 0.3
    x0, y0 = 40e-6, -30e-6
    kx, ky = 2 * math.pi / LAM * 1e-3, -2 * math.pi / LAM * 0.7e-3
    xs, ys = O.grid_x(n, p), O.grid_y(n, p)
    u = np.exp(-(xs[:, None] - x0) ** 2 / w0 ** 2 - (ys[None, :] - y0) ** 2 / w0 ** 2
               + 1j * (kx * xs[:, None] + ky * ys[None, :]))
    w = np.conj(u)[:, :, None, None] * u[None, None, :, :]
    wb, dx = O.propagate(w, n, p, LAM, z, farfield)
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    v = CF.gaussian_beam_field(X[:, None], x0, w0, kx, LAM, z, farfield) * \
        CF.gaussian_beam_field(Y[None, :], y0, w0, ky, LAM, z, farfield)
    ref = np.conj(v)[:, :, None, None] * v[None, None, :, :] / (LAM * z) ** 2
    assert rel(wb, ref) < 1e-9
    # The spectral density peaks near the geometric landing point x0 + kappa z / k.
    s = O.spectral_density(wb)
    i, j = np.unravel_index(np.argmax(s), s.shape)
    assert abs(X[i] - (x0 + kx * z * LAM / (2 * math.pi))) < 2 * dx
    assert abs(Y[j] - (y0 + ky * z * LAM / (2 * math.pi))) < 2 * dx


# ---------------------------------------------------------------------------------------------
# Non-separable coherent source: rank-1 reduction to the textbook field Fresnel transform (FFT).
# Catches: mistakes that only show on non-separable sources (the 2D geometry, axis pairing).
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_rank1_circle_matches_field_fft(farfield):
    n, p, z = 32, 20e-6, 0.1
    w = O.build_source(spec(model=O.MODEL_COHERENT, geometry=O.GEO_CIRCLE, geo_r0_m=10 * p), n, p)
    u = O.geometry_mask(n, p, O.GEO_CIRCLE, 10 * p)
    wb, _ = O.propagate(w, n, p, LAM, z, farfield)
    ub = CF.fresnel_field_fft(u.astype(np.complex128), n, p, LAM, z, farfield)
    ref = np.conj(ub)[:, :, None, None] * ub[None, None, :, :] / (LAM * z) ** 2
    assert rel(wb, ref) < 1e-12


# ---------------------------------------------------------------------------------------------
# Invariants on random Hermitian non-negative definite sources.
# Parseval catches any scale error. Hermiticity and PSD catch a conj on the wrong side.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_parseval_hermitian_psd(farfield):
    n, p, z = 8, 20e-6, 0.05
    w = WI.random_hermitian_psd(n, seed=1)
    wb, dx = O.propagate(w, n, p, LAM, z, farfield)
    sa, sb = O.spectral_density(w), O.spectral_density(wb)
    assert abs(sb.sum() * dx ** 2 / (sa.sum() * p ** 2) - 1) < 1e-13
    m = wb.reshape(n * n, n * n)
    assert np.abs(m - m.conj().T).max() < 1e-14 * np.abs(m).max()
    assert np.linalg.eigvalsh(0.5 * (m + m.conj().T)).min() > -1e-12 * np.abs(m).max()
    mu = O.degree_of_coherence_full(wb)
    assert np.abs(mu).max() <= 1 + 1e-12


def test_primary_source_scale():
    """eq. (C) with Lambda = 1/(4 pi) for a primary source: the ratio to the secondary source is
    (lambda / 4 pi)^2."""
    n, p, z = 4, 20e-6, 0.05
    w = WI.random_hermitian_psd(n, seed=2)
    a, _ = O.propagate(w, n, p, LAM, z, False, O.KIND_SECONDARY)
    b, _ = O.propagate(w, n, p, LAM, z, False, O.KIND_PRIMARY)
    assert rel(b, a * (LAM / (4 * math.pi)) ** 2) < 1e-14


# ---------------------------------------------------------------------------------------------
# Incoherent sources (Sec. 5.2): S_B is uniform, Fresnel == far field, and the discrete
# van Cittert-Zernike form holds exactly. The annulus mu follows the Bessel form to pixel accuracy.
# Catches: the chirp applied on the output side only, or a wrong sign in the x1 - x2 dependence.
# ---------------------------------------------------------------------------------------------
def test_coherent_source_is_rank_one_whatever_sigma_g():
    """A coherent source (Sec. 5.1) has |mu| = 1: W = A Y(p1) Y(p2) is rank one, and sigma_g (a GSM
    and MAP parameter) does not enter. Catches: the Gaussian mu applied to the coherent model."""
    n, p = 10, 20e-6
    w = O.build_source(spec(model=O.MODEL_COHERENT, amplitude=1.3, sigma_g_m=0.04e-3, geometry=O.GEO_CIRCLE,
                            geo_r0_m=3.5 * p), n, p)
    ev = np.linalg.eigvalsh(w.reshape(n * n, n * n))
    assert ev[-2] < 1e-12 * ev[-1]
    s = O.spectral_density(w)
    mu = O.degree_of_coherence(w, n // 2, n // 2, 1e-12)
    assert np.allclose(np.abs(mu)[s > 0], 1.0, atol=1e-14)


def test_incoherent_source_identities():
    n, p, z = 16, 20e-6, 0.2
    sp = spec(model=O.MODEL_INCOHERENT, amplitude=2.0, geometry=O.GEO_ANNULUS, geo_r0_m=6 * p,
              geo_r1_m=2 * p)
    w = O.build_source(sp, n, p)
    y = O.geometry_mask(n, p, O.GEO_ANNULUS, 6 * p, 2 * p)
    wf, dx = O.propagate(w, n, p, LAM, z, False)
    wff, _ = O.propagate(w, n, p, LAM, z, True)
    assert rel(wf, wff) < 1e-13
    s = O.spectral_density(wf)
    expect = O.coupling_constant(LAM, z) * p ** 4 * 2.0 * y.sum()
    assert np.abs(s / expect - 1).max() < 1e-13
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    xs, ys = O.grid_x(n, p), O.grid_y(n, p)
    for (m1, n1, m2, n2) in [(3, 4, 9, 1), (8, 8, 0, 15), (15, 2, 5, 11)]:
        bx, by = X[m1] - X[m2], Y[n1] - Y[n2]
        ph = np.exp(2j * math.pi * (bx * xs[:, None] + by * ys[None, :]) / (LAM * z))
        vcz = O.coupling_constant(LAM, z) * p ** 4 * 2.0 * np.sum(y * ph)
        chirp = np.exp(-1j * math.pi * (X[m1] ** 2 + Y[n1] ** 2 - X[m2] ** 2 - Y[n2] ** 2) / (LAM * z))
        assert abs(wf[m1, n1, m2, n2] - chirp * vcz) < 1e-13 * abs(expect)


def test_annulus_mu_bessel_form():
    n, p, z, lam = 64, 1e-3, 5.0, O.wavelength_from_omega(3.7699e15)   # example 2 pitch/omega/R
    sp = spec(model=O.MODEL_INCOHERENT, geometry=O.GEO_ANNULUS, geo_r0_m=11 * p, geo_r1_m=5 * p)
    w = O.build_source(sp, n, p)
    wb, dx = O.propagate(w, n, p, lam, z, True)
    mu = O.degree_of_coherence(wb, n // 2, n // 2)
    X = O.grid_x(n, dx)
    theory = CF.annulus_mu_farfield(np.abs(X), 11 * p, 5 * p, lam, z)
    row = np.abs(mu[:, n // 2])
    first_lobe = np.abs(X) < 0.6 * lam * z / (11 * p)
    assert np.abs(row[first_lobe] - np.abs(theory[first_lobe])).max() < 0.03
    # Phase of mu(0, x2) is the output chirp q(z, x2) (the eq. theory_mu_annular exponential).
    k = n // 2 + 3
    assert abs(np.angle(mu[k, n // 2] / np.sign(theory[k]) * np.exp(-1j * math.pi * X[k] ** 2 / (lam * z)))) < 1e-9


# ---------------------------------------------------------------------------------------------
# Thin lens (Sec. 2.2) and the q algebra (eqs. qprop): Fresnel of a lensed source at z = f equals
# the far field of the unlensed source. Catches: the lens applied with the wrong conjugation.
# ---------------------------------------------------------------------------------------------
def test_lens_at_focal_distance_is_far_field():
    n, p, f = 16, 20e-6, 0.2
    base = dict(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3, geometry=O.GEO_CIRCLE, geo_r0_m=6 * p)
    wl = O.build_source(spec(lens_focal_m=f, wavelength_m=LAM, **base), n, p)
    w0 = O.build_source(spec(**base), n, p)
    a, _ = O.propagate(wl, n, p, LAM, f, False)
    b, _ = O.propagate(w0, n, p, LAM, f, True)
    assert rel(a, b) < 1e-12


# ---------------------------------------------------------------------------------------------
# Imaging through a thin lens (Sec. 2.2, eqs. WA_imaging, imaging, WC_imaging). On the sampled
# grids the chain is exact: with the lens law 1/R1 + 1/R2 = 1/f the three middle chirps cancel
# (q(R1) q*(f) q(R2) = 1), and two forward DFTs reverse the index. So, per axis, the plane-C
# sample k sees the source sample N - k (mod N), and
#   W_C[k1; k2] = (R1/R2)^2 phi*(k1) phi(k2) W_A[N - k1; N - k2],
#   phi(k) = exp(i pi (|x'_k|^2 / R2 + |xi_(N-k)|^2 / R1) / lambda),   x' on the pitch (R2/R1) d.
# Catches: the lens with the wrong conjugation or focal length, a dropped lens, the stages in the
# wrong order, the wrong plane-B pitch.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,r1,r2", [(8, 0.2, 0.2), (16, 0.2, 0.2), (16, 0.15, 0.45), (8, 0.5, 0.25)])
def test_imaging_conjugate_planes_reverse_the_source(n, r1, r2):
    p = 20e-6
    f = r1 * r2 / (r1 + r2)
    wa = WI.random_hermitian_psd(n, seed=21 + n)
    wc, pc = O.image_through_lens(wa, n, p, LAM, r1, f, r2)
    assert abs(pc / (p * r2 / r1) - 1) < 1e-14
    rev = (n - np.arange(n)) % n
    c = np.arange(n) - n / 2
    xi2 = (p * c[rev]) ** 2                       # xi of the reversed source index, per axis
    xc2 = (pc * c) ** 2                           # x' of the image index, per axis
    ph = np.exp(1j * math.pi * ((xc2[:, None] + xc2[None, :]) / r2 + (xi2[:, None] + xi2[None, :]) / r1) / LAM)
    ref = (r1 / r2) ** 2 * np.conj(ph)[:, :, None, None] * wa[np.ix_(rev, rev, rev, rev)] * ph[None, None, :, :]
    assert rel(wc, ref) < 1e-11
    # the image S is the mirrored source S scaled by 1 / magnification^2
    assert rel(O.spectral_density(wc), (r1 / r2) ** 2 * O.spectral_density(wa)[np.ix_(rev, rev)]) < 1e-11


@pytest.mark.parametrize("geo", [O.GEO_CIRCLE, O.GEO_SQUARE])
def test_imaging_coherent_source_with_pupil_matches_field_optics(geo):
    """A coherent source W = U* U stays rank one; through the lens with a finite pupil its image is
    U_C* U_C, with U_C from two single-field Fresnel transforms (numpy FFT) and the pupil-limited
    lens T = P q*(f) in between. Catches: the pupil on the wrong point, P applied twice or not at all."""
    n, p, lam, r1, r2 = 16, 20e-6, LAM, 0.2, 0.3
    f = r1 * r2 / (r1 + r2) * 1.1                      # slightly defocused: no exact cancellation
    rng = WI.rng(17)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    wa = np.conj(u)[:, :, None, None] * u[None, None, :, :]
    pb = lam * r1 / (n * p)
    a = 0.3 * n * pb                                   # pupil radius (half side for the square)
    ub = CF.fresnel_field_fft(u, n, p, lam, r1)
    c = np.arange(n) - n / 2
    d2i, d2j = c[:, None] ** 2 + 0 * c[None, :], 0 * c[:, None] + c[None, :] ** 2
    thr = (a / pb) ** 2 * (1 + 1e-9)
    pupil = (d2i + d2j <= thr) if geo == O.GEO_CIRCLE else ((d2i <= thr) & (d2j <= thr))
    assert 0 < pupil.sum() < n * n
    xb2 = (pb * c[:, None]) ** 2 + (pb * c[None, :]) ** 2
    uc = CF.fresnel_field_fft(pupil * np.exp(-1j * math.pi * xb2 / (lam * f)) * ub, n, pb, lam, r2)
    cc = 1.0 / (lam * r1) ** 2 / (lam * r2) ** 2
    ref = cc * np.conj(uc)[:, :, None, None] * uc[None, None, :, :]
    wc, _ = O.image_through_lens(wa, n, p, lam, r1, f, r2, geo, a)
    assert rel(wc, ref) < 1e-12


# ---------------------------------------------------------------------------------------------
# Exact free-space kernel (eq. h_free) against the Fresnel operator (eqs. approx_L, W_fresnel).
# With equal source and output pitch d = sqrt(lambda z / N), the grids span rho ~ sqrt(N lambda z),
# so every term that the Fresnel expansion drops shrinks like 1/z: the phase -k rho^4 / (8 z^3) and
# the amplitude terms of Lambda(r)/r. Expanding h to the next order,
#   h ~ (1/(lambda z)) (1 - 3 rho^2 / (4 z^2)) exp(i k (rho^2/(2z) - rho^4/(8 z^3)))   (secondary)
#   h ~ (1/(4 pi z)) (1 - rho^2 / (2 z^2)) ...                                          (primary)
# must leave an error that shrinks like 1/z^2.
# Catches: a wrong conjugation or grid in the direct sum (an O(1) difference), a wrong scale or
# obliquity factor (a difference that does not shrink at these rates), a lost or wrong phase term.
# ---------------------------------------------------------------------------------------------
def _next_order_kernel_sum(w, n, p, lam, z, kind):
    dx = lam * z / (n * p)
    c = np.arange(n) - n / 2
    xo, yo, xs, ys = dx * c, -dx * c, p * c, -p * c
    Xo, Yo, Xs, Ys = np.repeat(xo, n), np.tile(yo, n), np.repeat(xs, n), np.tile(ys, n)
    rho2 = (Xo[:, None] - Xs[None, :]) ** 2 + (Yo[:, None] - Ys[None, :]) ** 2
    k = 2 * math.pi / lam
    if kind == O.KIND_SECONDARY:
        amp = (1 - 0.75 * rho2 / z ** 2) / (lam * z)
    else:
        amp = (1 - 0.5 * rho2 / z ** 2) / (4 * math.pi * z)
    h = amp * np.exp(1j * k * (rho2 / (2 * z) - rho2 ** 2 / (8 * z ** 3)))
    m = w.reshape(n * n, n * n)
    return (p ** 4 * (np.conj(h) @ m @ h.T)).reshape(n, n, n, n)


@pytest.mark.parametrize("kind", [O.KIND_SECONDARY, O.KIND_PRIMARY])
def test_direct_kernel_converges_to_fresnel(kind):
    n = 8
    w = WI.random_hermitian_psd(n, seed=33)
    e1, e2 = [], []
    for z in (2e-3, 4e-3, 8e-3, 16e-3):
        p = math.sqrt(LAM * z / n)
        wd, dxd = O.propagate_direct(w, n, p, LAM, z, kind)
        wf, dxf = O.propagate(w, n, p, LAM, z, False, kind)
        assert abs(dxd / p - 1) < 1e-12 and dxd == dxf
        e1.append(rel(wd, wf))
        e2.append(rel(wd, _next_order_kernel_sum(w, n, p, LAM, z, kind)))
    assert e1[0] < 1e-2
    for a, b in zip(e1, e1[1:]):
        assert 0.45 < b / a < 0.55, e1          # Fresnel error ~ 1/z
    for a, b in zip(e2, e2[1:]):
        assert 0.22 < b / a < 0.28, e2          # next-order error ~ 1/z^2


def test_direct_kernel_is_hermitian_and_psd():
    """h* W h keeps a Hermitian non-negative definite W so (eq. W_general holds for any kernel)."""
    n, p, z = 4, 20e-6, 3e-3
    w = WI.random_hermitian_psd(n, seed=34)
    wd, _ = O.propagate_direct(w, n, p, LAM, z)
    m = wd.reshape(n * n, n * n)
    assert np.abs(m - m.conj().T).max() < 1e-12 * np.abs(m).max()
    assert np.linalg.eigvalsh(m).min() > -1e-12 * np.abs(m).max()


# ---------------------------------------------------------------------------------------------
# Zero padding (Sec. 3.3): the paper pads the N x N array to N_z x N_z, transforms, and crops back,
# with N_z in the relation of eq. (spatial_resolution). Done literally here: embed the N^4 source in
# an N_z^4 zero array, propagate that at size N_z, crop the central N^4. The oracle's definition with
# n_fft = N_z must give the same array. N need not be a power of two.
# Catches: N instead of N_z in dx, an off-by-one crop (centre), padding on the wrong axes.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,nz", [(4, 8), (6, 10), (6, 16), (10, 10)])
@pytest.mark.parametrize("farfield", [False, True])
def test_zero_padding_equals_embed_propagate_crop(n, nz, farfield):
    p, z = 20e-6, 0.05
    w = WI.random_hermitian_psd(n, seed=40 + n)
    s0 = (nz - n) // 2
    big = np.zeros((nz,) * 4, dtype=np.complex128)
    sl = slice(s0, s0 + n)
    big[sl, sl, sl, sl] = w
    wb_big, dx_big = O.propagate(big, nz, p, LAM, z, farfield)
    got, dx = O.propagate(w, n, p, LAM, z, farfield, n_fft=nz)
    assert dx == dx_big == LAM * z / (nz * p)
    assert rel(got, wb_big[sl, sl, sl, sl]) < 1e-12


@pytest.mark.parametrize("n,nz", [(96, 96), (120, 240), (100, 256)])
def test_gsm_closed_form_non_power_of_two(n, nz):
    """GSM (separable) at N = 96, 100, 120, with and without padding, against the re-derived closed
    form: nothing in the definition needs N or N_z to be a power of two."""
    p, z, ss, sg = 20e-6, 0.5, 0.1e-3, 0.05e-3
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, ss, sg, "x"), O.gsm_axis_factor(n, p, ss, sg, "y"),
                                   n, p, LAM, z, n_fft=nz)
    dx = O.output_pitch(n, p, LAM, z, nz)
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], ss, sg, LAM, z, False)
    cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], ss, sg, LAM, z, False)
    assert rel(np.kron(bx, by), np.kron(cx, cy)) < 1e-8


def test_q_algebra():
    n, p, z = 64, 20e-6, 0.3
    beta = 1.7
    # q(R, xi / beta) = q(beta^2 R, xi)
    assert np.abs(O.chirp_table(n, p / beta, LAM, z) - O.chirp_table(n, p, LAM, beta ** 2 * z)).max() < 1e-12
    # q(R1) q*(R2) = q(R1 R2 / (R2 - R1)), and q q* = 1
    r1, r2 = 0.3, 0.7
    lhs = O.chirp_table(n, p, LAM, r1) * np.conj(O.chirp_table(n, p, LAM, r2))
    assert np.abs(lhs - O.chirp_table(n, p, LAM, r1 * r2 / (r2 - r1))).max() < 1e-11
    t = O.chirp_table(n, p, LAM, z)
    assert np.abs(np.abs(t) - 1).max() < 1e-15


def test_chirp_table_high_precision():
    """Each FP64 entry agrees with a 40-digit evaluation of exp(i pi xi^2 / (lambda R))."""
    n, p, z = 256, 10e-6, 0.1
    t = O.chirp_table(n, p, LAM, z)
    mpmath.mp.dps = 40
    for i in [0, 1, 7, 100, 128, 129, 200, 255]:
        ph = mpmath.pi * (mpmath.mpf(p) * (i - n // 2)) ** 2 / (mpmath.mpf(LAM) * mpmath.mpf(z))
        ref = complex(mpmath.cos(ph), mpmath.sin(ph))
        assert abs(t[i] - ref) < 5e-12


# ---------------------------------------------------------------------------------------------
# Other routes to the same operator: a literal loop over the eight indices (N = 4), the full
# N^2 x N^2 kernel, and Algorithm 2 step by step with numpy FFTs (checks the centring reading).
# ---------------------------------------------------------------------------------------------
def test_brute_force_loop_n4():
    n, p, z = 4, 20e-6, 0.01
    w = WI.random_complex((n, n, n, n), seed=3)
    dx = O.output_pitch(n, p, LAM, z)
    xs, ys, X, Y = O.grid_x(n, p), O.grid_y(n, p), O.grid_x(n, dx), O.grid_y(n, dx)
    s = p ** 4 / (LAM * z) ** 2

    def h(xo, yo, xi, eta):
        return complex(np.exp(1j * math.pi * ((xo - xi) ** 2 + (yo - eta) ** 2) / (LAM * z)))

    out = np.zeros_like(w)
    for m1 in range(n):
        for n1 in range(n):
            for m2 in range(n):
                for n2 in range(n):
                    acc = 0j
                    for i1 in range(n):
                        for j1 in range(n):
                            a = np.conj(h(X[m1], Y[n1], xs[i1], ys[j1]))
                            for i2 in range(n):
                                for j2 in range(n):
                                    acc += a * w[i1, j1, i2, j2] * h(X[m2], Y[n2], xs[i2], ys[j2])
                    out[m1, n1, m2, n2] = s * acc
    ref, _ = O.propagate(w, n, p, LAM, z)
    assert rel(ref, out) < 1e-13


@pytest.mark.parametrize("farfield", [False, True])
def test_matrix_and_alg2_routes(farfield):
    n, p, z = 8, 20e-6, 0.05
    w = WI.random_complex((n, n, n, n), seed=4)
    a, _ = O.propagate(w, n, p, LAM, z, farfield)
    assert rel(O.propagate_matrix(w, n, p, LAM, z, farfield), a) < 1e-13
    b, _ = O.propagate_alg2(w, n, p, LAM, z, farfield)
    assert rel(b, a) < 1e-13


def test_separable_route():
    n, p, z = 16, 20e-6, 0.2
    wx, wy = O.gsm_axis_factor(n, p, 0.1e-3, 0.05e-3, "x"), O.gsm_axis_factor(n, p, 0.1e-3, 0.05e-3, "y")
    w = wx[:, None, :, None] * wy[None, :, None, :]
    assert rel(w, O.build_source(spec(sigma_s_m=0.1e-3, sigma_g_m=0.05e-3), n, p)) < 1e-15
    bx, by = O.propagate_separable(wx, wy, n, p, LAM, z)
    a, _ = O.propagate(w, n, p, LAM, z)
    assert rel(bx[:, None, :, None] * by[None, :, None, :], a) < 1e-13


# ---------------------------------------------------------------------------------------------
# Adjoint: dot-product test and, for diagonal G_B, the Toeplitz closed form.
# Catches: a transposed or unconjugated kernel in the adjoint.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_adjoint_dot_product(farfield):
    n, p, z = 8, 20e-6, 0.05
    w = WI.random_complex((n, n, n, n), seed=5)
    g = WI.random_complex((n, n, n, n), seed=6)
    pw, _ = O.propagate(w, n, p, LAM, z, farfield)
    pg = O.propagate_adjoint(g, n, p, LAM, z, farfield)
    lhs = np.vdot(pw, g)
    rhs = np.vdot(w, pg)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_adjoint_diagonal_toeplitz():
    """G_B = diag(g): G_A(xi1, xi2) = s q(xi1) q*(xi2) sum_x g(x) exp(-2 pi i x.(xi1 - xi2) / (lambda z))."""
    n, p, z = 8, 20e-6, 0.05
    gs = WI.rng(7).standard_normal((n, n))
    gb = np.zeros((n, n, n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            gb[i, j, i, j] = gs[i, j]
    ga = O.propagate_adjoint(gb, n, p, LAM, z)
    dx = O.output_pitch(n, p, LAM, z)
    X, Y, xs, ys = O.grid_x(n, dx), O.grid_y(n, dx), O.grid_x(n, p), O.grid_y(n, p)
    s = p ** 4 / (LAM * z) ** 2
    for (i1, j1, i2, j2) in [(0, 0, 0, 0), (1, 2, 3, 4), (7, 0, 2, 6), (5, 5, 1, 3)]:
        dxi, deta = xs[i1] - xs[i2], ys[j1] - ys[j2]
        acc = np.sum(gs * np.exp(-2j * math.pi * (X[:, None] * dxi + Y[None, :] * deta) / (LAM * z)))
        qq = np.exp(1j * math.pi * (xs[i1] ** 2 + ys[j1] ** 2 - xs[i2] ** 2 - ys[j2] ** 2) / (LAM * z))
        assert abs(ga[i1, j1, i2, j2] - s * qq * acc) < 1e-12 * s * np.abs(gs).sum()


# ---------------------------------------------------------------------------------------------
# Fit gradient vs central finite differences of the oracle's own loss.
# Catches: a missing factor 2 or a missing term in dL/dI, dL/dsg.
# ---------------------------------------------------------------------------------------------
def test_fit_gradient_finite_differences():
    n, p, z = 8, 20e-6, 0.05
    imap = WI.intensity_map(n, p, seed=4, env_sigma_m=0.05e-3).astype(np.float64)
    tsrc = O.build_source(spec(sigma_s_m=0.05e-3, sigma_g_m=0.03e-3), n, p)
    target = O.spectral_density(O.propagate(tsrc, n, p, LAM, z)[0])
    sg = 0.04e-3
    loss, d_i, d_sg = O.fit_gradient(imap, sg, target, n, p, LAM, z)
    assert abs(loss - O.fit_loss(imap, sg, target, n, p, LAM, z)) < 1e-12 * loss
    for (i, j) in [(3, 4), (0, 7), (4, 4)]:
        h = 1e-6 * imap[i, j]
        ip, im = imap.copy(), imap.copy()
        ip[i, j] += h
        im[i, j] -= h
        fd = (O.fit_loss(ip, sg, target, n, p, LAM, z) - O.fit_loss(im, sg, target, n, p, LAM, z)) / (2 * h)
        assert abs(fd - d_i[i, j]) < 1e-6 * np.abs(d_i).max()
    h = 1e-6 * sg
    fd = (O.fit_loss(imap, sg + h, target, n, p, LAM, z) - O.fit_loss(imap, sg - h, target, n, p, LAM, z)) / (2 * h)
    assert abs(fd - d_sg) < 1e-6 * abs(d_sg)


# ---------------------------------------------------------------------------------------------
# Source builder (Sec. 3.2; Algorithms 6-7; eqs. circle, W_def).
# ---------------------------------------------------------------------------------------------
def test_source_builder_definitions():
    n, p = 16, 20e-6
    # Circle: pixel-unit boundary included (20 px radius at 20 um pitch gives 0.4 mm exactly).
    y = O.geometry_mask(64, 20e-6, O.GEO_CIRCLE, 0.4e-3)
    assert y[32 + 20, 32] == 1 and y[32 + 12, 32 + 16] == 1 and y[32 + 15, 32 + 14] == 0
    assert y.sum() == sum(1 for a in range(-32, 32) for b in range(-32, 32) if a * a + b * b <= 400)
    # GSM diagonal gives S = A exp(-xi^2 / (2 sS^2)) and |mu| = exp(-|d|^2 / (2 sg^2)).
    w = O.build_source(spec(amplitude=3.0, sigma_s_m=0.1e-3, sigma_g_m=0.05e-3), n, p)
    s = O.spectral_density(w)
    xs, ys = O.grid_x(n, p), O.grid_y(n, p)
    r2 = xs[:, None] ** 2 + ys[None, :] ** 2
    assert np.abs(s - 3.0 * np.exp(-r2 / (2 * (0.1e-3) ** 2))).max() < 1e-14
    mu = O.degree_of_coherence(w, 8, 8)
    d2 = (xs[:, None] - xs[8]) ** 2 + (ys[None, :] - ys[8]) ** 2
    assert np.abs(mu - np.exp(-d2 / (2 * (0.05e-3) ** 2))).max() < 1e-14
    # MAP model: S = A I exactly (eq. W_def with mu(xi, xi) = 1).
    imap = WI.intensity_map(n, p, seed=4)
    wm = O.build_source(spec(model=O.MODEL_MAP, amplitude=2.0, sigma_g_m=0.05e-3, intensity_map=imap), n, p)
    assert np.abs(O.spectral_density(wm) - 2.0 * imap).max() < 1e-6 * imap.max()
    # Lens: |W| unchanged, phase q(f, xi1) q*(f, xi2).
    wl = O.build_source(spec(sigma_s_m=0.1e-3, lens_focal_m=0.2, wavelength_m=LAM), n, p)
    w0 = O.build_source(spec(sigma_s_m=0.1e-3), n, p)
    assert np.abs(np.abs(wl) - np.abs(w0)).max() < 1e-15
    ph = wl[3, 4, 9, 1] / w0[3, 4, 9, 1]
    expect = np.exp(1j * math.pi * (r2[3, 4] - r2[9, 1]) / (LAM * 0.2))
    assert abs(ph - expect) < 1e-13


def test_degree_of_coherence_floor():
    n = 8
    w = O.build_source(spec(model=O.MODEL_COHERENT, geometry=O.GEO_CIRCLE, geo_r0_m=2 * 20e-6), n, 20e-6)
    mu = O.degree_of_coherence(w, 4, 4)
    y = O.geometry_mask(n, 20e-6, O.GEO_CIRCLE, 2 * 20e-6)
    assert np.array_equal(np.abs(mu) > 0, y > 0)
    assert np.allclose(mu[y > 0], 1.0)
    assert not O.degree_of_coherence(w, 0, 0).any()       # P1 outside the source: mu = 0


# ---------------------------------------------------------------------------------------------
# Any output grid, and the polychromatic sum on a common grid (R17). The closed form holds at any
# observation point. Catches: the output pitch entering the chirp or the DFT frequency wrongly.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_gsm_closed_form_any_output_grid(farfield):
    n, p, ss, sg, z = 64, 20e-6, 0.08e-3, 0.12e-3, 0.3     # the window holds the source to e^-16
    w = O.build_source(spec(sigma_s_m=ss, sigma_g_m=sg), n, p)
    dx = 0.73 * O.output_pitch(n, p, LAM, z)          # not the FFT grid
    wb, d = O.propagate(w, n, p, LAM, z, farfield, out_pitch=dx)
    assert d == dx
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], ss, sg, LAM, z, farfield)
    cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], ss, sg, LAM, z, farfield)
    assert rel(wb, cx[:, None, :, None] * cy[None, :, None, :]) < 1e-9


def test_polychromatic_sum_of_closed_forms():
    """Three wavelengths at one distance on a common grid: S and the mu row of the weighted sum of the
    closed-form CSDs. The source fits the window to e^-16 and the grid is the FFT grid of the shortest
    wavelength, so that no kernel is sampled beyond its Nyquist rate."""
    n, p, ss, sg, z = 32, 20e-6, 0.04e-3, 0.06e-3, 0.2
    lams, zs, ws = [500e-9, 600e-9, 700e-9], [z, z, z], [0.5, 1.0, 0.8]
    dx = O.output_pitch(n, p, 500e-9, z)
    w = O.build_source(spec(sigma_s_m=ss, sigma_g_m=sg), n, p)
    ip, jp = 14, 17
    s, mu = O.polychromatic(w, n, p, lams, zs, ws, dx, ip=ip, jp=jp, floor_rel=1e-6)
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    tot = 0
    for lam, wk in zip(lams, ws):
        cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], ss, sg, lam, z, False)
        cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], ss, sg, lam, z, False)
        tot = tot + wk * cx[:, None, :, None] * cy[None, :, None, :]
    sr = np.real(np.einsum("ijij->ij", tot))
    assert rel(s, sr) < 1e-9
    row = tot[ip, jp]
    mur = row / np.sqrt(sr[ip, jp] * sr)
    mur[sr <= 1e-6 * sr.max()] = 0
    assert rel(mu, mur) < 1e-8


# ---------------------------------------------------------------------------------------------
# The full 4D degree of coherence (Algorithm 5 at every P1, eq. defMu, floor reading R6) against
# closed forms, where the floor masks a large part of the grid on both points.
# Catches: a mask applied to one point only, a missing mask, S taken from the wrong point, or a
# missing square root.
# ---------------------------------------------------------------------------------------------
def _mu_full_one_sided(w, floor_rel=1e-12):
    """A planted mistake (for the pin tests below only): the floor applied to the second point only."""
    s = np.real(np.einsum("ijij->ij", w))
    ok = s > floor_rel * s.max()
    root = np.sqrt(np.where(s > 0, s, 1.0))
    mu = w / (root[:, :, None, None] * root[None, None, :, :])
    return np.where(ok[None, None, :, :], mu, 0.0)


def _mu_full_unmasked(w, floor_rel=1e-12):
    """A planted mistake: no floor at all (S below tau divides W anyway)."""
    s = np.real(np.einsum("ijij->ij", w))
    root = np.sqrt(np.where(s > 0, s, 1.0))
    return w / (root[:, :, None, None] * root[None, None, :, :])


def _gsm_source_mu_error(mu_fn):
    """GSM source plane: S = A exp(-xi^2 / (2 sS^2)) and mu = exp(-|xi1 - xi2|^2 / (2 sg^2)) (reading R3).
    sS = 20 um at a 20 um pitch puts most of the 16 x 16 grid below the floor 1e-12 max S."""
    n, p, a, ss, sg, floor = 16, 20e-6, 2.5, 20e-6, 50e-6, 1e-12
    w = O.build_source(spec(amplitude=a, sigma_s_m=ss, sigma_g_m=sg), n, p)
    xs, ys = O.grid_x(n, p), O.grid_y(n, p)
    r2 = xs[:, None] ** 2 + ys[None, :] ** 2
    s_cf = a * np.exp(-r2 / (2 * ss ** 2))
    tau = floor * a                                  # max S = A, at the grid centre
    assert np.abs(s_cf / tau - 1).min() > 1e-3       # no point sits on the floor
    ok = s_cf > tau
    assert 0.2 < ok.mean() < 0.8                     # the mask matters on both sides
    d2 = (xs[:, None, None, None] - xs[None, None, :, None]) ** 2 + \
         (ys[None, :, None, None] - ys[None, None, None, :]) ** 2
    ref = np.where(ok[:, :, None, None] & ok[None, None, :, :], np.exp(-d2 / (2 * sg ** 2)), 0.0)
    return np.abs(mu_fn(w, floor) - ref).max()


def _coherent_circle_mu_error(mu_fn):
    """Coherent top-hat (mu = 1 on the source, Sec. 5.1): mu = Y(p1) Y(p2) exactly, whatever the floor."""
    n, p = 16, 20e-6
    w = O.build_source(spec(model=O.MODEL_COHERENT, amplitude=0.7, geometry=O.GEO_CIRCLE, geo_r0_m=5 * p), n, p)
    y = O.geometry_mask(n, p, O.GEO_CIRCLE, 5 * p)
    ref = y[:, :, None, None] * y[None, None, :, :]
    with np.errstate(invalid="ignore", divide="ignore"):
        got = mu_fn(w, 1e-12)
    return np.nan_to_num(np.abs(got - ref), nan=np.inf).max()


def _propagated_gsm_mu_error(mu_fn):
    """Propagated GSM (Mandel-Wolf beam): mu(x1, x2) = exp(-|x2 - x1|^2 / (2 sg^2 D^2))
    exp(i k (|x2|^2 - |x1|^2) / (2 Rz)), masked where S = A D^-2 exp(-|x|^2 / (2 sS^2 D^2)) is below
    1e-3 of its maximum on either point. Window and source as in the 4D closed-form pin (truncation
    below 1e-9); with the floor at 1e-3 the oracle's error in W is at most ~1e-9 / 1e-3 in mu."""
    n, p, ss, sg, z, floor = 64, 20e-6, 0.08e-3, 0.12e-3, 0.3, 1e-3
    w = O.build_source(spec(sigma_s_m=ss, sigma_g_m=sg), n, p)
    wb, dx = O.propagate(w, n, p, LAM, z)
    X, Y = O.grid_x(n, dx), O.grid_y(n, dx)
    cx = CF.gsm_axis_closed_form(X[:, None], X[None, :], ss, sg, LAM, z, False)
    cy = CF.gsm_axis_closed_form(Y[:, None], Y[None, :], ss, sg, LAM, z, False)
    sx, sy = np.real(np.diag(cx)), np.real(np.diag(cy))
    s_cf = sx[:, None] * sy[None, :]
    tau = floor * s_cf.max()
    assert np.abs(s_cf / tau - 1).min() > 1e-4
    ok = s_cf > tau
    assert 0.005 < ok.mean() < 0.5
    mux = cx / np.sqrt(sx[:, None] * sx[None, :])
    muy = cy / np.sqrt(sy[:, None] * sy[None, :])
    ref = np.where(ok[:, :, None, None] & ok[None, None, :, :], mux[:, None, :, None] * muy[None, :, None, :], 0.0)
    return np.abs(mu_fn(wb, floor) - ref).max()


@pytest.mark.parametrize("case,tol", [(_gsm_source_mu_error, 1e-14), (_coherent_circle_mu_error, 1e-14),
                                      (_propagated_gsm_mu_error, 1e-5)])
def test_mu_full_closed_forms(case, tol):
    assert case(O.degree_of_coherence_full) < tol


@pytest.mark.parametrize("planted", [_mu_full_one_sided, _mu_full_unmasked])
def test_mu_full_pins_reject_planted_masks(planted):
    """The planted one-sided and missing masks fail the GSM pins (so the pins do constrain the mask)."""
    assert _gsm_source_mu_error(planted) > 1e-3
    assert _propagated_gsm_mu_error(planted) > 1e-3


def test_mu_slice_matches_full_closed_form():
    """The slice mu(P1, .) (Algorithm 5) is row P1 of the full mu; both masked on both points."""
    n, p, ss, sg, z, floor = 64, 20e-6, 0.08e-3, 0.12e-3, 0.3, 1e-3
    w = O.build_source(spec(sigma_s_m=ss, sigma_g_m=sg), n, p)
    wb, _ = O.propagate(w, n, p, LAM, z)
    full = O.degree_of_coherence_full(wb, floor)
    for ip, jp in [(32, 32), (30, 35), (0, 0), (5, 60)]:
        sl = O.degree_of_coherence(wb, ip, jp, floor)
        assert np.array_equal(sl != 0, full[ip, jp] != 0)
        assert np.abs(sl - full[ip, jp]).max() < 1e-14


# ---------------------------------------------------------------------------------------------
# The separable adjoint (used for the full-size adjoint parity at N = 128): the dot-product test
# against the separable forward operator at N = 128, and equality with the 4D adjoint at N = 8.
# Catches: a transposed or unconjugated axis factor, the scale on the wrong factor.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("farfield", [False, True])
def test_adjoint_separable_dot_product_n128(farfield):
    n, p, z = 128, 20e-6, 0.5
    r = WI.rng(91)
    w = [r.standard_normal((n, n)) + 1j * r.standard_normal((n, n)) for _ in range(2)]
    g = [r.standard_normal((n, n)) + 1j * r.standard_normal((n, n)) for _ in range(2)]
    bx, by = O.propagate_separable(w[0], w[1], n, p, LAM, z, farfield)
    ax, ay = O.propagate_adjoint_separable(g[0], g[1], n, p, LAM, z, farfield)
    # <a (x) b, c (x) d> = <a, c> <b, d> for the 4D tensors of the separable factors.
    lhs = np.vdot(bx, g[0]) * np.vdot(by, g[1])
    rhs = np.vdot(w[0], ax) * np.vdot(w[1], ay)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("farfield", [False, True])
def test_adjoint_separable_equals_4d(farfield):
    n, p, z = 8, 20e-6, 0.05
    r = WI.rng(92)
    gx = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    gy = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    ax, ay = O.propagate_adjoint_separable(gx, gy, n, p, LAM, z, farfield)
    g4 = gx[:, None, :, None] * gy[None, :, None, :]
    ref = O.propagate_adjoint(g4, n, p, LAM, z, farfield)
    assert rel(ax[:, None, :, None] * ay[None, :, None, :], ref) < 1e-13
