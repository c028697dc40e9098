"""Plain FP64 reference implementation of the CSD propagation path (test infrastructure only).

Every array is complex128 or float64. Nothing here is tuned; each function writes out the
passage it cites, so that a reader can check it against the paper by eye.

Conventions, from the paper:
  * CSD array ``W[i1, j1, i2, j2]``, a 4D N x N x N x N array (Sec. 3.1, the CSDA).
  * Grid: xi = d (i - N/2), eta = d (N/2 - j). This is eqs. (point)/(n12) with n = (i, -j) and
    n0 = (N/2, -N/2).
  * W = <U*(r1) U(r2)>. The propagated CSD is eq. (W_general), W_B = iiiint h*(x1, xi1) W_A h(x2, xi2).

Readings taken where the paper is ambiguous:
  R1 Transform signs. Eqs. (W_fresnel) and (W_farfield) print a minus sign on both Fourier
     kernels. Eq. (W_general) with h from eq. (h_free) puts h* on xi1, so the xi1 kernel is
     exp(+2 pi i x1.xi1 / (lambda R)) and the xi2 kernel is exp(-2 pi i x2.xi2 / (lambda R)).
     Algorithm 2 agrees: a direct FFT over the second point and an inverse FFT over the first.
  R2 Scale. C = Lambda1* Lambda2 / R^2 (eq. (C)), with the discrete area element d^4 of the
     four source coordinates. A secondary source at normal incidence has
     Lambda = (k / 4 pi i)(cos + cos) = 1 / (i lambda), so C = 1 / (lambda R)^2.
     A primary source has Lambda = 1 / (4 pi), so C = 1 / (4 pi R)^2.
  R3 Gaussian Schell model, eq. (GSM_source) and Sec. 5.4. The exponents need minus signs:
     W = A exp(-(xi1^2 + xi2^2) / (4 sS^2)) exp(-|xi1 - xi2|^2 / (2 sg^2)), which gives
     S = A exp(-xi^2 / (2 sS^2)). sS = inf means uniform S; sg = inf means full coherence.
  R4 Geometry, eq. (circle): Y = 1 iff |xi| <= a. The decision is taken in pixel units as
     d2 <= (a/d)^2 (1 + 1e-9), where d2 = (i - N/2)^2 + (j - N/2)^2 is an exact integer. The
     slack absorbs the decimal-to-binary rounding of a and d.
     Annulus = outer circle minus inner circle, both as in eq. (circle).
     Square: |xi| <= a and |eta| <= a, with a the half side.
  R5 Thin lens (Sec. 2.2): T = P q*(f, x), W+ = T*(x1) W- T(x2) = q(f, x1) W- q*(f, x2).
  R6 mu where S vanishes (Algorithm 5). mu = W(P1, x) / sqrt(S(P1) S(x)) where both
     S(P1) > tau and S(x) > tau, with tau = floor_rel * max S; mu = 0 elsewhere.
  R7 Incoherent source: Kronecker delta W[p1; p2] = A Y(p1) delta(p1, p2), with no 1/d^2
     factor.
  R8 Exact free-space kernel (eq. h_free, for the validity check of the approximation eq. approx_L
     and the Fresnel expansion): h = Lambda(r) exp(i k r) / r with r = sqrt(z^2 + |x - xi|^2).
     Secondary source at normal incidence: cos(theta_i) = 1 and cos(theta_o) = z / r, so
     Lambda = (k / (4 pi i)) (1 + z / r); primary: Lambda = 1 / (4 pi). The factor 1/i and the
     common phase exp(i k z) cancel between h* and h, so they are left out.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np

C_LIGHT = 299_792_458.0  # speed of light (m/s), used in omega = 2 pi c / lambda (eq. q_factor)

MODEL_GSM, MODEL_MAP, MODEL_COHERENT, MODEL_INCOHERENT = 0, 1, 2, 3
GEO_NONE, GEO_CIRCLE, GEO_SQUARE, GEO_ANNULUS, GEO_MASK = 0, 1, 2, 3, 4
KIND_SECONDARY, KIND_PRIMARY = 0, 1
GEO_SLACK = 1e-9


# ----------------------------------------------------------------------------------------------
# Units and sampling
# ----------------------------------------------------------------------------------------------
def wavelength_from_omega(omega: float) -> float:
    """Free-space relation omega = 2 pi c / lambda (text after eq. q_factor)."""
    return 2.0 * math.pi * C_LIGHT / omega


def omega_from_wavelength(lam: float) -> float:
    return 2.0 * math.pi * C_LIGHT / lam


def grid_x(n: int, pitch: float) -> np.ndarray:
    """x coordinate of index i: pitch (i - N/2) (eqs. point, n12)."""
    return pitch * (np.arange(n, dtype=np.float64) - n / 2)


def grid_y(n: int, pitch: float) -> np.ndarray:
    """y coordinate of index j: pitch (N/2 - j). The y axis is flipped (eq. n12)."""
    return pitch * (n / 2 - np.arange(n, dtype=np.float64))


def output_pitch(n: int, pitch: float, lam: float, z: float, n_fft: Optional[int] = None) -> float:
    """Sec. 3.3, eq. (spatial_resolution): dx = 2 pi c R / (omega N dxi) = lambda R / (N dxi).

    With zero padding to n_fft points, N in this relation is n_fft (Sec. 3.3, the remark on zero
    padding): the output grid is finer, and the result is cropped back to N points."""
    return lam * z / ((n if n_fft is None else n_fft) * pitch)


def fresnel_number(a: float, lam: float, z: float) -> float:
    """N_F = a^2 / (lambda R) (Sec. 5.1)."""
    return a * a / (lam * z)


# ----------------------------------------------------------------------------------------------
# Propagator q and the coupling constant
# ----------------------------------------------------------------------------------------------
def q(R: float, r2, lam: float):
    """eq. (q_factor): q(R, xi) = exp(i pi xi^2 / (lambda R)), with r2 = xi . xi."""
    return np.exp(1j * math.pi * np.asarray(r2, dtype=np.float64) / (lam * R))


def chirp_table(n: int, pitch: float, lam: float, z: float) -> np.ndarray:
    """q(z, .) along one axis, at the axis coordinates pitch (i - N/2), i = 0..N-1.

    The 2D propagator is the product of the two axis factors: q(R, (xi, eta)) = q(R, xi) q(R, eta).
    The y flip does not change it, because eta^2 = (pitch (N/2 - j))^2.
    """
    return q(z, grid_x(n, pitch) ** 2, lam)


def coupling_constant(lam: float, z: float, kind: int = KIND_SECONDARY) -> float:
    """eq. (C): C = Lambda1* Lambda2 / R^2 (reading R2)."""
    if kind == KIND_SECONDARY:
        return 1.0 / (lam * z) ** 2
    if kind == KIND_PRIMARY:
        return 1.0 / (4.0 * math.pi * z) ** 2
    raise ValueError("kind")


def kernel_1d(n: int, pitch: float, lam: float, z: float, farfield: bool, axis: str,
              n_fft: Optional[int] = None, out_pitch: Optional[float] = None) -> np.ndarray:
    """One axis factor K[m, i] of the propagation kernel h(x, xi), on the output and source grids.

    Fresnel (eqs. h_free, approx_L, W_fresnel): h(x, xi) = exp(i pi |x - xi|^2 / (lambda R)).
    Far field (eq. W_farfield, q(R, xi) set to 1): h(x, xi) = exp(i pi |x|^2 / (lambda R)) exp(-2 pi i x.xi / (lambda R)).
    Both factorise into an x factor times a y factor. The constant amplitude Lambda / R is in C.
    n_fft: the output pitch of zero padding to n_fft points (see output_pitch); the N output samples
    are the central ones of the padded grid, at the same centred coordinates.
    out_pitch: any other output pitch (the same centred coordinates, out_pitch (i - N/2)); eq. (W_general)
    holds at any observation point, the grid of eq. (spatial_resolution) is only the FFT's.
    """
    dx = out_pitch if out_pitch is not None else output_pitch(n, pitch, lam, z, n_fft)
    if axis == "x":
        xo, xs = grid_x(n, dx), grid_x(n, pitch)
    else:
        xo, xs = grid_y(n, dx), grid_y(n, pitch)
    if farfield:
        return np.exp(1j * math.pi * xo[:, None] ** 2 / (lam * z)) * \
            np.exp(-2j * math.pi * xo[:, None] * xs[None, :] / (lam * z))
    return np.exp(1j * math.pi * (xo[:, None] - xs[None, :]) ** 2 / (lam * z))


# ----------------------------------------------------------------------------------------------
# Source plane (Sec. 3.2, Algorithms 6-7, eqs. GSM_source, circle, W_def)
# ----------------------------------------------------------------------------------------------
def geometry_mask(n: int, pitch: float, geometry: int, r0: float = 0.0, r1: float = 0.0,
                  mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Y(p) in {0, 1} on the N x N grid (eq. GSM_source, eq. circle; reading R4)."""
    c = np.arange(n, dtype=np.float64) - n / 2
    di2 = c[:, None] ** 2 + 0.0 * c[None, :]
    dj2 = 0.0 * c[:, None] + c[None, :] ** 2
    if geometry == GEO_NONE:
        return np.ones((n, n))
    if geometry == GEO_MASK:
        return (np.asarray(mask) != 0).astype(np.float64)
    rho0 = r0 / pitch
    t0 = rho0 * rho0 * (1.0 + GEO_SLACK)
    if geometry == GEO_CIRCLE:
        return ((di2 + dj2) <= t0).astype(np.float64)
    if geometry == GEO_SQUARE:
        return ((di2 <= t0) & (dj2 <= t0)).astype(np.float64)
    if geometry == GEO_ANNULUS:
        rho1 = r1 / pitch
        t1 = rho1 * rho1 * (1.0 + GEO_SLACK)
        d2 = di2 + dj2
        return ((d2 <= t0) & (d2 > t1)).astype(np.float64)
    raise ValueError("geometry")


def build_source(spec, n: int, pitch: float) -> np.ndarray:
    """Source CSD array W0 (Algorithm 1 steps 1-3, Sec. 3.2).

    W0[p1; p2] = Y(p1) Y(p2) W_rho(xi1, xi2) (eq. GSM_source), where
      GSM        W_rho = A exp(-(xi1^2 + xi2^2) / (4 sS^2)) exp(-|xi1 - xi2|^2 / (2 sg^2))   (R3)
      MAP        W_rho = A sqrt(I(p1)) sqrt(I(p2)) exp(-|xi1 - xi2|^2 / (2 sg^2))          (eq. W_def)
      COHERENT   W_rho = A                                                                 (Sec. 5.1)
      INCOHERENT W_rho = A delta(p1, p2)                                                   (R7)
    An optional thin lens then multiplies by q(f, xi1) q*(f, xi2) (R5).
    """
    x, y = grid_x(n, pitch), grid_y(n, pitch)
    X = x[:, None] + 0.0 * y[None, :]
    Y = 0.0 * x[:, None] + y[None, :]
    r2 = X ** 2 + Y ** 2
    geo = geometry_mask(n, pitch, spec.geometry, spec.geo_r0_m, spec.geo_r1_m, spec.mask)
    A = spec.amplitude
    if spec.model == MODEL_INCOHERENT:
        w = np.zeros((n, n, n, n), dtype=np.complex128)
        d = A * geo
        for i in range(n):
            for j in range(n):
                w[i, j, i, j] = d[i, j]
    else:
        if spec.model == MODEL_GSM:
            inv4s2 = 0.0 if math.isinf(spec.sigma_s_m) else 1.0 / (4.0 * spec.sigma_s_m ** 2)
            amp = np.exp(-r2 * inv4s2)                      # sqrt(S(xi)) / sqrt(A)
        elif spec.model == MODEL_MAP:
            amp = np.sqrt(np.asarray(spec.intensity_map, dtype=np.float64))
        elif spec.model == MODEL_COHERENT:
            amp = np.ones((n, n))
        else:
            raise ValueError("model")
        amp = amp * geo
        # The Gaussian degree of coherence belongs to the GSM and MAP models only; a coherent source
        # has mu = 1 whatever sigma_g says (Sec. 5.1).
        uses_g = spec.model in (MODEL_GSM, MODEL_MAP) and not math.isinf(spec.sigma_g_m)
        inv2g2 = 1.0 / (2.0 * spec.sigma_g_m ** 2) if uses_g else 0.0
        dX = X[:, :, None, None] - X[None, None, :, :]
        dY = Y[:, :, None, None] - Y[None, None, :, :]
        mu = np.exp(-(dX ** 2 + dY ** 2) * inv2g2)
        w = (A * amp[:, :, None, None] * amp[None, None, :, :] * mu).astype(np.complex128)
    if spec.lens_focal_m != 0.0:
        ql = q(spec.lens_focal_m, r2, spec.wavelength_m)
        w = w * ql[:, :, None, None] * np.conj(ql)[None, None, :, :]
    return w


def gsm_axis_factor(n: int, pitch: float, sigma_s: float, sigma_g: float, axis: str = "x",
                    amplitude: float = 1.0) -> np.ndarray:
    """One axis factor w[i1, i2] of a GSM source (R3); W0[i1, j1, i2, j2] = wx[i1, i2] wy[j1, j2].

    The GSM exponent is a sum of an x term and a y term, so W0 is separable.
    The amplitude A is carried by the x factor.
    """
    c = grid_x(n, pitch) if axis == "x" else grid_y(n, pitch)
    inv4s2 = 0.0 if math.isinf(sigma_s) else 1.0 / (4.0 * sigma_s ** 2)
    inv2g2 = 0.0 if math.isinf(sigma_g) else 1.0 / (2.0 * sigma_g ** 2)
    f = np.exp(-(c[:, None] ** 2 + c[None, :] ** 2) * inv4s2 - (c[:, None] - c[None, :]) ** 2 * inv2g2)
    return (amplitude if axis == "x" else 1.0) * f.astype(np.complex128)


# ----------------------------------------------------------------------------------------------
# Propagation (Sec. 2.1 eqs. W_general, W_fresnel, W_farfield; Sec. 3.4 Algorithms 2-3)
# ----------------------------------------------------------------------------------------------
def _sum_axis(w: np.ndarray, k: np.ndarray, axis: int) -> np.ndarray:
    """out[..., m, ...] = sum_i k[m, i] w[..., i, ...]: one iterated sum over one source coordinate."""
    out = np.tensordot(k, w, axes=([1], [axis]))      # the new axis comes first
    return np.moveaxis(out, 0, axis)


def propagate(w: np.ndarray, n: int, pitch: float, lam: float, z: float, farfield: bool = False,
              kind: int = KIND_SECONDARY, n_fft: Optional[int] = None,
              out_pitch: Optional[float] = None) -> Tuple[np.ndarray, float]:
    """W_B(x1, x2) = C d^4 sum_{xi1, xi2} h*(x1, xi1) W_A(xi1, xi2) h(x2, xi2) (eq. W_general, R1, R2).

    The four source coordinates (xi1, eta1, xi2, eta2) are summed one at a time, each against
    its own axis factor of h. h factorises into an x factor and a y factor (see kernel_1d).
    Any even n is allowed; n_fft (>= n) selects the output grid of zero padding (output_pitch).
    out_pitch: evaluate on the grid of that pitch instead (see kernel_1d).
    Returns (W_B, dx), where dx is the output pitch of eq. (spatial_resolution), or out_pitch.
    """
    kx = kernel_1d(n, pitch, lam, z, farfield, "x", n_fft, out_pitch)
    ky = kernel_1d(n, pitch, lam, z, farfield, "y", n_fft, out_pitch)
    s = coupling_constant(lam, z, kind) * pitch ** 4
    out = _sum_axis(w, kx, 2)              # sum over xi2 with h(x2, xi2)
    out = _sum_axis(out, ky, 3)            # sum over eta2
    out = _sum_axis(out, np.conj(kx), 0)   # sum over xi1 with h*(x1, xi1)
    out = _sum_axis(out, np.conj(ky), 1)   # sum over eta1
    return s * out, (out_pitch if out_pitch is not None else output_pitch(n, pitch, lam, z, n_fft))


def propagate_matrix(w: np.ndarray, n: int, pitch: float, lam: float, z: float,
                     farfield: bool = False, kind: int = KIND_SECONDARY) -> np.ndarray:
    """Same operator with the full 2D kernel as one N^2 x N^2 matrix H[(m, n), (i, j)] = h(x_mn, xi_ij).

    W_B = C d^4 conj(H) W_A H^T. Small N only (cost N^6).
    """
    dx = output_pitch(n, pitch, lam, z)
    xs, ys = grid_x(n, pitch), grid_y(n, pitch)
    xo, yo = grid_x(n, dx), grid_y(n, dx)
    XS = np.repeat(xs, n)
    YS = np.tile(ys, n)
    XO = np.repeat(xo, n)
    YO = np.tile(yo, n)
    if farfield:
        H = np.exp(1j * math.pi * (XO ** 2 + YO ** 2)[:, None] / (lam * z)) * \
            np.exp(-2j * math.pi * (XO[:, None] * XS[None, :] + YO[:, None] * YS[None, :]) / (lam * z))
    else:
        H = np.exp(1j * math.pi * ((XO[:, None] - XS[None, :]) ** 2 + (YO[:, None] - YS[None, :]) ** 2)
                   / (lam * z))
    s = coupling_constant(lam, z, kind) * pitch ** 4
    m = w.reshape(n * n, n * n)
    return (s * (np.conj(H) @ m @ H.T)).reshape(n, n, n, n)


def qfunction(w: np.ndarray, n: int, d: float, lam: float, R: float) -> np.ndarray:
    """Algorithm 3: W' = W exp[i omega / (2 c R) (xi2^2 - xi1^2)] = q*(R, xi1) q(R, xi2) W."""
    x, y = grid_x(n, d), grid_y(n, d)
    r2 = x[:, None] ** 2 + y[None, :] ** 2
    qq = q(R, r2, lam)
    return w * np.conj(qq)[:, :, None, None] * qq[None, None, :, :]


def propagate_alg2(w: np.ndarray, n: int, pitch: float, lam: float, z: float,
                   farfield: bool = False, kind: int = KIND_SECONDARY) -> Tuple[np.ndarray, float]:
    """Algorithm 2 (freespaceprop), step by step, with numpy FFTs.

    Steps: q-function (Fresnel only); a 2D direct FFT over the last two axes of every slab;
    transpose (2, 3, 0, 1); a 2D inverse FFT over the last two axes; transpose back;
    dx (eq. spatial_resolution); q-function at the output pitch.
    Two points are not written in the paper (reading R2 and the centring). The FFTs act on the
    centred index i - N/2 (fftshift o fft o ifftshift). The scale C d^4 is applied with the
    1/N^2 of numpy's ifft2 undone.
    """
    w1 = qfunction(w, n, pitch, lam, z) if not farfield else w.copy()
    w2 = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(w1, axes=(2, 3)), axes=(2, 3)), axes=(2, 3))
    w3 = np.transpose(w2, (2, 3, 0, 1))
    w4 = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(w3, axes=(2, 3)), axes=(2, 3)), axes=(2, 3))
    w5 = np.transpose(w4, (2, 3, 0, 1))
    dx = output_pitch(n, pitch, lam, z)
    w6 = qfunction(w5, n, dx, lam, z)
    s = coupling_constant(lam, z, kind) * pitch ** 4 * n * n
    return s * w6, dx


def propagate_separable(wx: np.ndarray, wy: np.ndarray, n: int, pitch: float, lam: float, z: float,
                        farfield: bool = False, kind: int = KIND_SECONDARY,
                        n_fft: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """For W_A[i1, j1, i2, j2] = wx[i1, i2] wy[j1, j2], the operator of `propagate` gives
    W_B = bx[m1, m2] by[n1, n2], with bx = C d^4 conj(Kx) wx Kx^T and by = conj(Ky) wy Ky^T.
    This is the same sum with the x and y coordinates summed separately.
    """
    kx = kernel_1d(n, pitch, lam, z, farfield, "x", n_fft)
    ky = kernel_1d(n, pitch, lam, z, farfield, "y", n_fft)
    s = coupling_constant(lam, z, kind) * pitch ** 4
    return s * (np.conj(kx) @ wx @ kx.T), np.conj(ky) @ wy @ ky.T


def propagate_adjoint(g: np.ndarray, n: int, pitch: float, lam: float, z: float,
                      farfield: bool = False, kind: int = KIND_SECONDARY) -> np.ndarray:
    """Adjoint P^H of the operator of `propagate` for the real inner product Re sum conj(a) b.

    For P(W) = C d^4 conj(H) W H^T, P^H(G) = C d^4 H^T G conj(H). Element-wise:
    G_A(xi1, xi2) = C d^4 sum_{x1, x2} h(x1, xi1) G_B(x1, x2) h*(x2, xi2).
    """
    kx = kernel_1d(n, pitch, lam, z, farfield, "x")
    ky = kernel_1d(n, pitch, lam, z, farfield, "y")
    s = coupling_constant(lam, z, kind) * pitch ** 4
    out = _sum_axis(g, kx.T, 0)            # sum over x1 with h(x1, xi1)
    out = _sum_axis(out, ky.T, 1)
    out = _sum_axis(out, np.conj(kx).T, 2)  # sum over x2 with h*(x2, xi2)
    out = _sum_axis(out, np.conj(ky).T, 3)
    return s * out


def propagate_adjoint_separable(gx: np.ndarray, gy: np.ndarray, n: int, pitch: float, lam: float, z: float,
                                farfield: bool = False, kind: int = KIND_SECONDARY) -> Tuple[np.ndarray, np.ndarray]:
    """The adjoint of `propagate_adjoint` for a separable G_B[m1, n1, m2, n2] = gx[m1, m2] gy[n1, n2]:
    P^H(G_B) = ax[i1, i2] ay[j1, j2], with ax = C d^4 Kx^T gx conj(Kx) and ay = Ky^T gy conj(Ky).
    This is the same sum with the x and y output coordinates summed separately (as propagate_separable).
    """
    kx = kernel_1d(n, pitch, lam, z, farfield, "x")
    ky = kernel_1d(n, pitch, lam, z, farfield, "y")
    s = coupling_constant(lam, z, kind) * pitch ** 4
    return s * (kx.T @ gx @ np.conj(kx)), ky.T @ gy @ np.conj(ky)


# ----------------------------------------------------------------------------------------------
# Exact free-space kernel (eq. h_free; the check of eq. approx_L and of the Fresnel expansion; R8)
# ----------------------------------------------------------------------------------------------
def rs_kernel_matrix(n: int, pitch: float, lam: float, z: float, kind: int = KIND_SECONDARY) -> np.ndarray:
    """H[(m, n), (i, j)] = |Lambda(r)| exp(i k (r - z)) / r between the output point x_mn (grid of
    eq. spatial_resolution) and the source point xi_ij, with r = sqrt(z^2 + |x - xi|^2) (R8).

    r - z is computed as rho^2 / (r + z), which has no cancellation.
    """
    dx = output_pitch(n, pitch, lam, z)
    xo, yo = grid_x(n, dx), grid_y(n, dx)
    xs, ys = grid_x(n, pitch), grid_y(n, pitch)
    Xo = np.repeat(xo, n)
    Yo = np.tile(yo, n)
    Xs = np.repeat(xs, n)
    Ys = np.tile(ys, n)
    rho2 = (Xo[:, None] - Xs[None, :]) ** 2 + (Yo[:, None] - Ys[None, :]) ** 2
    r = np.sqrt(z * z + rho2)
    if kind == KIND_SECONDARY:
        amp = (1.0 + z / r) / (2.0 * lam)
    elif kind == KIND_PRIMARY:
        amp = np.full_like(r, 1.0 / (4.0 * math.pi))
    else:
        raise ValueError("kind")
    return amp / r * np.exp(2j * math.pi * (rho2 / (r + z)) / lam)


def propagate_direct(w: np.ndarray, n: int, pitch: float, lam: float, z: float,
                     kind: int = KIND_SECONDARY) -> Tuple[np.ndarray, float]:
    """eq. (W_general) with the exact kernel of eq. (h_free), summed directly on the grids (no
    approximation eq. approx_L, no Fresnel expansion): W_B = d^4 conj(H) W_A H^T with H from
    rs_kernel_matrix. The output grid is that of the Fresnel operator, for element-wise comparison.
    Returns (W_B, dx)."""
    h = rs_kernel_matrix(n, pitch, lam, z, kind)
    wm = w.reshape(n * n, n * n)
    out = pitch ** 4 * (np.conj(h) @ wm @ h.T)
    return out.reshape(n, n, n, n), output_pitch(n, pitch, lam, z)


# ----------------------------------------------------------------------------------------------
# Thin lens and imaging (Sec. 2.2: lens transmission, eqs. WA_imaging, imaging, WC_imaging; R5)
# ----------------------------------------------------------------------------------------------
def lens_transmission(n: int, pitch: float, lam: float, focal: float, pupil_geometry: int = GEO_NONE,
                      pupil_radius: float = 0.0) -> np.ndarray:
    """T(x) = P(x) q*(f, x) on the N x N grid of `pitch` (Sec. 2.2).

    P is the pupil: 1 inside a circle (or a square of half side `pupil_radius`), decided in pixel
    units as R4, and 0 outside; GEO_NONE means no aperture (P = 1). The pupil carries no aberration
    phase. focal = inf (or 0) means no lens phase, only the aperture.
    """
    x, y = grid_x(n, pitch), grid_y(n, pitch)
    r2 = x[:, None] ** 2 + y[None, :] ** 2
    if math.isinf(focal) or focal == 0.0:
        t = np.ones((n, n), dtype=np.complex128)
    else:
        t = np.conj(q(focal, r2, lam))
    if pupil_geometry != GEO_NONE:
        if pupil_geometry not in (GEO_CIRCLE, GEO_SQUARE):
            raise ValueError("pupil geometry")
        t = t * geometry_mask(n, pitch, pupil_geometry, pupil_radius)
    return t


def apply_lens(w: np.ndarray, n: int, pitch: float, lam: float, focal: float, pupil_geometry: int = GEO_NONE,
               pupil_radius: float = 0.0) -> np.ndarray:
    """W+(x1, x2) = T*(x1) W-(x1, x2) T(x2): the CSD just after a thin lens (Sec. 2.2, R5)."""
    t = lens_transmission(n, pitch, lam, focal, pupil_geometry, pupil_radius)
    return np.conj(t)[:, :, None, None] * w * t[None, None, :, :]


def propagate_lens(w: np.ndarray, n: int, pitch: float, lam: float, focal: float, z: float,
                   pupil_geometry: int = GEO_NONE, pupil_radius: float = 0.0,
                   kind: int = KIND_SECONDARY) -> Tuple[np.ndarray, float]:
    """A thin lens at the plane of `w` (grid `pitch`), then Fresnel propagation by z: the second
    stage of eq. (WC_imaging) before the lens law is used. Returns (W, output pitch)."""
    return propagate(apply_lens(w, n, pitch, lam, focal, pupil_geometry, pupil_radius), n, pitch, lam, z,
                     False, kind)


def image_through_lens(w: np.ndarray, n: int, pitch: float, lam: float, r1: float, focal: float, r2: float,
                       pupil_geometry: int = GEO_NONE, pupil_radius: float = 0.0,
                       kind: int = KIND_SECONDARY) -> Tuple[np.ndarray, float]:
    """Source plane A -> lens plane B (Fresnel, R1) -> lens T = P q*(f) -> image plane C (Fresnel, R2),
    eq. (WC_imaging) without the approximations that follow it. Returns (W_C, pitch at C)."""
    wb, pb = propagate(w, n, pitch, lam, r1, False, kind)
    return propagate_lens(wb, n, pb, lam, focal, r2, pupil_geometry, pupil_radius, kind)


# ----------------------------------------------------------------------------------------------
# Observables (Sec. 3.5, Algorithms 4-5, eqs. defS, defMu)
# ----------------------------------------------------------------------------------------------
def spectral_density(w: np.ndarray) -> np.ndarray:
    """Algorithm 4 / eq. (defS): S[i, j] = W[i, j; i, j]. Returns the real part."""
    n = w.shape[0]
    s = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            s[i, j] = w[i, j, i, j].real
    return s


def degree_of_coherence(w: np.ndarray, ip: int, jp: int, floor_rel: float = 1e-12) -> np.ndarray:
    """Algorithm 5 / eq. (defMu), read as R6:
    mu[i, j] = W[ip, jp; i, j] / sqrt(S[ip, jp] S[i, j]) where both S exceed tau; 0 elsewhere."""
    s = spectral_density(w)
    tau = floor_rel * s.max()
    n = w.shape[0]
    mu = np.zeros((n, n), dtype=np.complex128)
    s0 = s[ip, jp]
    if not s0 > tau:
        return mu
    for i in range(n):
        for j in range(n):
            if s[i, j] > tau:
                mu[i, j] = w[ip, jp, i, j] / math.sqrt(s0 * s[i, j])
    return mu


def polychromatic(w: np.ndarray, n: int, pitch: float, lams, zs, weights, out_pitch: float,
                  farfield: bool = False, kind: int = KIND_SECONDARY, ip: int = 0, jp: int = 0,
                  floor_rel: float = 1e-12) -> Tuple[np.ndarray, np.ndarray]:
    """Polychromatic light from one source, read as R17: the CSD at each frequency propagates on its
    own (eq. W_general at wavelength lams[k] and distance zs[k]); on a common output grid of pitch
    out_pitch the weighted CSDs add, W(x1, x2) = sum_k weights[k] W_k(x1, x2), and S and mu follow from
    the sum (Algorithms 4-5). Returns (S, mu(P1, .))."""
    total = None
    for lam, z, wk in zip(lams, zs, weights):
        wb, _ = propagate(w, n, pitch, lam, z, farfield, kind, out_pitch=out_pitch)
        total = wk * wb if total is None else total + wk * wb
    return spectral_density(total), degree_of_coherence(total, ip, jp, floor_rel)


def degree_of_coherence_full(w: np.ndarray, floor_rel: float = 1e-12) -> np.ndarray:
    """eq. (defMu) for every pair: mu[p1; p2] = W[p1; p2] / sqrt(S[p1] S[p2]), masked as R6."""
    s = spectral_density(w)
    tau = floor_rel * s.max()
    ok = s > tau
    root = np.where(ok, np.sqrt(np.where(ok, s, 1.0)), 1.0)
    mu = w / (root[:, :, None, None] * root[None, None, :, :])
    return np.where(ok[:, :, None, None] & ok[None, None, :, :], mu, 0.0)


# ----------------------------------------------------------------------------------------------
# Differentiable fit of a custom intensity map and sigma_g (observable S at plane B)
# ----------------------------------------------------------------------------------------------
def fit_loss(imap: np.ndarray, sigma_g: float, target_s: np.ndarray, n: int, pitch: float,
             lam: float, z: float, farfield: bool = False) -> float:
    """L = sum_x (S_B(x) - S_t(x))^2, with S_B from the MAP model (eq. W_def, Gaussian mu)."""
    from types import SimpleNamespace
    spec = SimpleNamespace(model=MODEL_MAP, amplitude=1.0, sigma_s_m=math.inf, sigma_g_m=sigma_g,
                           geometry=GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=imap,
                           mask=None, lens_focal_m=0.0, wavelength_m=0.0)
    w = build_source(spec, n, pitch)
    wb, _ = propagate(w, n, pitch, lam, z, farfield)
    return float(np.sum((spectral_density(wb) - target_s) ** 2))


def fit_gradient(imap: np.ndarray, sigma_g: float, target_s: np.ndarray, n: int, pitch: float,
                 lam: float, z: float, farfield: bool = False):
    """Gradient of `fit_loss` via the adjoint: G_B = diag(2 (S_B - S_t)), G_A = P^H(G_B), then
    dL/dtheta = sum Re(conj(G_A) dW_A/dtheta) for each real parameter theta.

    With a = sqrt(I) and mu_g = exp(-|xi1 - xi2|^2 / (2 sg^2)):
      dL/dI(p) = (1 / (2 a(p))) [sum_p2 Re(conj(G_A[p; p2]) a(p2) mu_g(p, p2))
                                 + sum_p1 Re(conj(G_A[p1; p]) a(p1) mu_g(p1, p))]
      dL/dsg  = sum Re(conj(G_A) W_A) |xi1 - xi2|^2 / sg^3
    Returns (loss, dL/dI (N x N), dL/dsg).
    """
    from types import SimpleNamespace
    spec = SimpleNamespace(model=MODEL_MAP, amplitude=1.0, sigma_s_m=math.inf, sigma_g_m=sigma_g,
                           geometry=GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=imap,
                           mask=None, lens_focal_m=0.0, wavelength_m=0.0)
    wa = build_source(spec, n, pitch)
    wb, _ = propagate(wa, n, pitch, lam, z, farfield)
    sb = spectral_density(wb)
    gs = 2.0 * (sb - target_s)
    gb = np.zeros_like(wb)
    for i in range(n):
        for j in range(n):
            gb[i, j, i, j] = gs[i, j]
    ga = propagate_adjoint(gb, n, pitch, lam, z, farfield)
    a = np.sqrt(np.asarray(imap, dtype=np.float64))
    x, y = grid_x(n, pitch), grid_y(n, pitch)
    X = x[:, None] + 0.0 * y[None, :]
    Y = 0.0 * x[:, None] + y[None, :]
    d2 = (X[:, :, None, None] - X[None, None]) ** 2 + (Y[:, :, None, None] - Y[None, None]) ** 2
    mu = np.exp(-d2 / (2.0 * sigma_g ** 2))
    re = np.real(np.conj(ga) * mu)                 # Re(conj(G_A) mu_g), mu_g real
    rows = np.einsum("abcd,cd->ab", re, a)          # sum_p2 Re(conj(G[p; p2]) mu) a(p2)
    cols = np.einsum("abcd,ab->cd", re, a)          # sum_p1 Re(conj(G[p1; p]) mu) a(p1)
    d_i = (rows + cols) / (2.0 * a)
    d_sg = float(np.sum(np.real(np.conj(ga) * wa) * d2) / sigma_g ** 3)
    loss = float(np.sum((sb - target_s) ** 2))
    return loss, d_i, d_sg
