"""Differentiable spectral density of a propagated custom-map source (torch.autograd.Function).

Forward:  I, sigma_g -> W_A (custom map with a Gaussian degree of coherence; eq. W_def)
          -> W_B (Fresnel or far-field propagation; eqs. W_fresnel, W_farfield) -> S_B = Re diag W_B.
Backward: dL/dS_B -> adjoint propagation of diag(dL/dS_B) -> dL/dI and dL/dsigma_g.
Every step runs in libwolf kernels; this module only orders the calls.
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import torch

from . import (GEO_NONE, MODEL_MAP, build_source, fit_gradient, propagate, propagate_adjoint_diag,
               spectral_density)


def _map_source(imap: torch.Tensor, sigma_g: float):
    return SimpleNamespace(model=MODEL_MAP, amplitude=1.0, sigma_s_m=math.inf, sigma_g_m=float(sigma_g),
                           geometry=GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=imap, mask=None,
                           lens_focal_m=0.0, wavelength_m=0.0)


class PropagatedSpectralDensity(torch.autograd.Function):
    """S_B(I, sigma_g) on the output grid (pitch lambda z / (N pitch)).

    imap: CUDA float32 (N, N), all entries > 0.  sigma_g: float64 0-dim tensor (metres).
    """

    @staticmethod
    def forward(ctx, imap, sigma_g, pitch: float, wavelength: float, z: float, farfield: bool = False,
                dtype: torch.dtype = torch.complex64):
        n = imap.shape[0]
        sg = float(sigma_g)
        imap_c = imap.detach().contiguous()
        w = build_source(_map_source(imap_c, sg), n, pitch, dtype, device=imap.device)
        propagate(w, pitch, wavelength, z, farfield, out=w)
        s = spectral_density(w)
        ctx.save_for_backward(imap_c)
        ctx.cfg = (pitch, wavelength, z, farfield, dtype, sg, sigma_g.device, sigma_g.dtype)
        return s

    @staticmethod
    def backward(ctx, grad_s):
        (imap,) = ctx.saved_tensors
        pitch, wavelength, z, farfield, dtype, sg, sg_dev, sg_dtype = ctx.cfg
        real = torch.float32 if dtype == torch.complex64 else torch.float64
        g = propagate_adjoint_diag(grad_s.detach().to(real).contiguous(), pitch, wavelength, z, farfield,
                                   dtype=dtype)
        d_imap, d_sigma = fit_gradient(g, imap, pitch, sg)
        return d_imap, d_sigma.reshape(()).to(device=sg_dev, dtype=sg_dtype), None, None, None, None, None


def propagated_spectral_density(imap, sigma_g, pitch, wavelength, z, farfield=False, dtype=torch.complex64):
    return PropagatedSpectralDensity.apply(imap, sigma_g, pitch, wavelength, z, farfield, dtype)


def fit_step(imap, sigma_g, target_s, pitch, wavelength, z, farfield=False, dtype=torch.complex64):
    """One forward + backward of L = sum (S_B - S_t)^2. Returns the loss (a 0-dim tensor); the
    gradients land in imap.grad and sigma_g.grad."""
    s = propagated_spectral_density(imap, sigma_g, pitch, wavelength, z, farfield, dtype)
    loss = torch.sum((s.to(target_s.dtype) - target_s) ** 2)
    loss.backward()
    return loss
