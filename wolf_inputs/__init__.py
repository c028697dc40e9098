"""Seeded synthetic inputs and workload recipes, shared by the tests, the bench and the oracle.

This module holds none of the propagation method's arithmetic. It only draws seeded random
numbers (numpy PCG64 via ``default_rng``) and states the workload parameters: grid size, pitch,
wavelength, distances and source parameters. Each side (the HIP path and the CPU oracle) turns
those parameters into arrays on its own.

Workloads follow the paper's own workload shapes: Gaussian Schell-model sources (Sec. 5.4 and the
GSM appendix, used by the paper's performance section), apertures with partial coherence, and
incoherent sources (Sec. 5.2). The paper uses no public dataset; every input here is synthetic.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

#: Source models (the paper's source-model plug-ins of Sec. 3.2 and Sec. 4).
MODEL_GSM = 0          # Gaussian Schell-model: sqrt(S) Gaussian, mu Gaussian
MODEL_MAP = 1          # custom intensity map I(p), Gaussian mu
MODEL_COHERENT = 2     # mu == 1, uniform amplitude
MODEL_INCOHERENT = 3   # Kronecker delta in (p1, p2)

#: Geometries (the paper's geometry plug-ins, Sec. 3.2 and the circle appendix).
GEO_NONE = 0
GEO_CIRCLE = 1
GEO_SQUARE = 2
GEO_ANNULUS = 3
GEO_MASK = 4

KIND_SECONDARY = 0
KIND_PRIMARY = 1


@dataclasses.dataclass
class SourceSpec:
    """Plain description of a source plane; both sides build W0 from it independently."""
    model: int = MODEL_GSM
    amplitude: float = 1.0
    sigma_s_m: float = math.inf      # r.m.s. width of S; inf means uniform S
    sigma_g_m: float = math.inf      # r.m.s. width of mu; inf means fully coherent
    geometry: int = GEO_NONE
    geo_r0_m: float = 0.0            # circle/annulus outer radius, square half side
    geo_r1_m: float = 0.0            # annulus inner radius
    intensity_map: Optional[np.ndarray] = None   # (N, N) float32, model MAP only
    mask: Optional[np.ndarray] = None            # (N, N) uint8, geometry MASK only
    lens_focal_m: float = 0.0        # 0: no lens
    wavelength_m: float = 0.0        # needed iff lens_focal_m != 0


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    pitch_m: float
    wavelength_m: float
    z_m: float
    source: SourceSpec
    farfield: bool = False
    kind: int = KIND_SECONDARY
    probe: tuple = (0, 0)            # (ip, jp) point P1 for the mu slice


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    g = rng(seed)
    a = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    return a.astype(dtype)


def random_hermitian_psd(n: int, seed: int, rank: Optional[int] = None) -> np.ndarray:
    """A random Hermitian non-negative definite CSD array of shape (n, n, n, n).

    W[p1; p2] = sum_r conj(u_r[p1]) u_r[p2] / rank, with u_r complex Gaussian vectors, which is
    Hermitian and non-negative definite by construction.
    """
    m = n * n
    r = m if rank is None else rank
    g = rng(seed)
    u = (g.standard_normal((r, m)) + 1j * g.standard_normal((r, m))) / math.sqrt(2 * r)
    w = np.conj(u).T @ u
    return w.reshape(n, n, n, n)


def smooth_random_field(n: int, seed: int, sigma_px: float = 3.0) -> np.ndarray:
    """Standardised Gaussian-blurred (periodic) N(0,1) field on an n x n grid."""
    from scipy.ndimage import gaussian_filter

    g = rng(seed)
    f = gaussian_filter(g.standard_normal((n, n)), sigma=sigma_px, mode="wrap")
    f = (f - f.mean()) / f.std()
    return f


def intensity_map(n: int, pitch_m: float, seed: int = 4, env_sigma_m: float = 0.3e-3,
                  sigma_px: float = 3.0) -> np.ndarray:
    """Seeded smooth positive intensity map I(p) = env(p) * exp(0.5 g(p)), float32 (n, n).

    env is a centred Gaussian of r.m.s. width env_sigma_m on the grid xi = pitch (i - n/2),
    eta = pitch (n/2 - j); g is a smooth random field.
    """
    i = np.arange(n, dtype=np.float64)
    x = pitch_m * (i - n / 2)
    y = pitch_m * (n / 2 - i)
    r2 = x[:, None] ** 2 + y[None, :] ** 2
    env = np.exp(-r2 / (2 * env_sigma_m ** 2))
    return (env * np.exp(0.5 * smooth_random_field(n, seed, sigma_px))).astype(np.float32)


def random_mask(n: int, seed: int, p: float = 0.6) -> np.ndarray:
    return (rng(seed).random((n, n)) < p).astype(np.uint8)


# --------------------------------------------------------------------------------------------
# Workload recipes.  Lengths in metres.
# --------------------------------------------------------------------------------------------
LAMBDA_HENE = 632.8e-9


def gsm_small() -> List[Workload]:
    """N=16 Gaussian Schell-model source, Fresnel z=0.5 m and far field."""
    src = SourceSpec(model=MODEL_GSM, sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
    return [Workload("gsm16_fresnel", 16, 20e-6, LAMBDA_HENE, 0.5, src, False, probe=(8, 8)),
            Workload("gsm16_farfield", 16, 20e-6, LAMBDA_HENE, 0.5, src, True, probe=(8, 8))]


def tophat_lens64() -> Workload:
    """N=64 circular top-hat (radius 0.4 mm = 20 px), Gaussian mu, thin lens f=0.2 m, z=0.2 m."""
    src = SourceSpec(model=MODEL_GSM, sigma_s_m=math.inf, sigma_g_m=0.1e-3, geometry=GEO_CIRCLE,
                     geo_r0_m=0.4e-3, lens_focal_m=0.2, wavelength_m=LAMBDA_HENE)
    return Workload("tophat_lens64", 64, 20e-6, LAMBDA_HENE, 0.2, src, False, probe=(32, 32))


def gsm128() -> Workload:
    """N=128 GSM source (sigma_S=0.1 mm, sigma_g=0.05 mm, pitch 20 um), lambda 632.8 nm, z=0.5 m."""
    src = SourceSpec(model=MODEL_GSM, sigma_s_m=0.1e-3, sigma_g_m=0.05e-3)
    return Workload("gsm128_fresnel", 128, 20e-6, LAMBDA_HENE, 0.5, src, False, probe=(64, 64))


def polychromatic_pairs() -> Dict[str, np.ndarray]:
    """16 wavelengths uniform over 500-700 nm (inclusive), Gaussian spectral weights
    (centre 600 nm, r.m.s. 50 nm), 4 distances; 64 (lambda, z) pairs, lambda-major."""
    lam = 500e-9 + 200e-9 * np.arange(16) / 15.0
    w = np.exp(-(lam - 600e-9) ** 2 / (2 * (50e-9) ** 2))
    zs = np.array([0.1, 0.5, 1.0, 5.0])
    L, Z = np.meshgrid(lam, zs, indexing="ij")
    W, _ = np.meshgrid(w, zs, indexing="ij")
    return {"wavelength": L.ravel(), "z": Z.ravel(), "weight": W.ravel()}


def fit_map64() -> Workload:
    """N=64 custom intensity map (seed 4) with Gaussian mu (sigma_g 0.1 mm), z=0.3 m."""
    n, pitch = 64, 20e-6
    src = SourceSpec(model=MODEL_MAP, sigma_g_m=0.1e-3, intensity_map=intensity_map(n, pitch, 4))
    return Workload("fit_map64", n, pitch, LAMBDA_HENE, 0.3, src, False, probe=(32, 32))


def fit_target64() -> Workload:
    """Target of the fit: GSM sigma_S=0.15 mm, sigma_g=0.06 mm on the same grid and distance."""
    src = SourceSpec(model=MODEL_GSM, sigma_s_m=0.15e-3, sigma_g_m=0.06e-3)
    return Workload("fit_target64", 64, 20e-6, LAMBDA_HENE, 0.3, src, False, probe=(32, 32))


def gsm256() -> List[Workload]:
    """N=256 GSM source (sigma_S=0.5 mm, sigma_g=0.1 mm, pitch 10 um), z=1 m Fresnel and far field."""
    src = SourceSpec(model=MODEL_GSM, sigma_s_m=0.5e-3, sigma_g_m=0.1e-3)
    return [Workload("gsm256_fresnel", 256, 10e-6, LAMBDA_HENE, 1.0, src, False, probe=(128, 128)),
            Workload("gsm256_farfield", 256, 10e-6, LAMBDA_HENE, 1.0, src, True, probe=(128, 128))]
