"""Closed forms and textbook routines that pin the oracle (test infrastructure).

None of these is the oracle's own arithmetic. Each is a separate result from optics or from
the mathematics, and the discrete operator must reproduce it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import j1


def gsm_axis_closed_form(x1, x2, sigma_s, sigma_g, lam, z, farfield):
    """One axis factor of the propagated Gaussian Schell-model CSD (Sec. 5.4 beam; re-derived).

    The source axis factor is exp(-(x1^2 + x2^2) / (4 sS^2) - (x2 - x1)^2 / (2 sg^2)). Propagated
    with the per-axis Fresnel kernel and scale 1/(lambda z), it gives
        (1/D) exp(-(x1^2 + x2^2) / (4 sS^2 D^2) - (x2 - x1)^2 / (2 sg^2 D^2) + i k (x2^2 - x1^2) / (2 Rz))
    with 1/delta^2 = 1/(4 sS^2) + 1/sg^2. Fresnel: D^2 = 1 + (z / (k sS delta))^2 and
    Rz = z (1 + (k sS delta / z)^2). Far field (source chirp set to 1): D = z / (k sS delta), Rz = z.
    This is the Mandel-Wolf beam expansion. The 2D result is the product of the x and y factors.
    """
    k = 2 * math.pi / lam
    delta = 1.0 / math.sqrt(1.0 / (4 * sigma_s ** 2) + 1.0 / sigma_g ** 2)
    if farfield:
        D, Rz = z / (k * sigma_s * delta), z
    else:
        D = math.sqrt(1 + (z / (k * sigma_s * delta)) ** 2)
        Rz = z * (1 + (k * sigma_s * delta / z) ** 2)
    return (1.0 / D) * np.exp(-(x1 ** 2 + x2 ** 2) / (4 * sigma_s ** 2 * D ** 2)
                              - (x2 - x1) ** 2 / (2 * sigma_g ** 2 * D ** 2)
                              + 1j * k * (x2 ** 2 - x1 ** 2) / (2 * Rz))


def gaussian_beam_field(x, x0, w0, kappa, lam, z, farfield):
    """V(x) = integral of h(x, xi) exp(-(xi - x0)^2 / w0^2 + i kappa xi) d xi, per axis, exactly.

    h is the Fresnel kernel exp(i pi (x - xi)^2 / (lambda z)), or for the far field
    exp(i pi x^2 / (lambda z)) exp(-2 pi i x xi / (lambda z)). The integral is the Gaussian integral
    integral of exp(-a xi^2 + b xi + c) = sqrt(pi / a) exp(b^2 / (4a) + c), with Re a > 0.
    """
    a = 1.0 / w0 ** 2 - (0.0 if farfield else 1j * math.pi / (lam * z))
    b = 2 * x0 / w0 ** 2 + 1j * kappa - 2j * math.pi * x / (lam * z)
    c = -x0 ** 2 / w0 ** 2 + 1j * math.pi * x ** 2 / (lam * z)
    return np.sqrt(math.pi / a) * np.exp(b ** 2 / (4 * a) + c)


def fresnel_field_fft(u, n, pitch, lam, z, farfield=False):
    """Textbook single-field Fresnel transform on the grid, with numpy's FFT.

    U_B(x) = d^2 sum_xi h(x, xi) U(xi). The Fresnel kernel is h = q(x) q(xi) exp(-2 pi i x.xi / (lambda z)).
    Since x xi / (lambda z) = (m - N/2)(i - N/2) / N on the grids, the sum is a centred 2D DFT.
    """
    c = np.arange(n) - n / 2
    xs = pitch * c
    dx = lam * z / (n * pitch)
    xo = dx * c
    src = u.copy()
    if not farfield:
        src = src * np.exp(1j * math.pi * (xs[:, None] ** 2 + xs[None, :] ** 2) / (lam * z))
    f = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(src)))
    return pitch ** 2 * np.exp(1j * math.pi * (xo[:, None] ** 2 + xo[None, :] ** 2) / (lam * z)) * f


def annulus_mu_farfield(b, a_o, a_i, lam, z):
    """|mu| of a uniform incoherent annulus in the far field (van Cittert-Zernike, Sec. 5.2).

    The printed eq. (theory_mu_annular) is missing the area weights. This is the reading with them:
    [a_o^2 2J1(v_o)/v_o - a_i^2 2J1(v_i)/v_i] / (a_o^2 - a_i^2), with v = k a b / z.
    """
    k = 2 * math.pi / lam

    def jinc(v):
        v = np.asarray(v, dtype=np.float64)
        out = np.ones_like(v)
        nz = np.abs(v) > 1e-12
        out[nz] = 2 * j1(v[nz]) / v[nz]
        return out

    return (a_o ** 2 * jinc(k * a_o * b / z) - a_i ** 2 * jinc(k * a_i * b / z)) / (a_o ** 2 - a_i ** 2)
