"""wolf: MI355X-native propagation of the cross-spectral density of a planar source.

This is the Python binding of libwolf (include/wolf.h). It only marshals arguments: torch
tensors supply device memory and the current HIP stream, and every step runs in the library's
HIP kernels. There is no CPU fallback. If libwolf.so is not built, `load()` raises.

The method is that of Magalhaes & Rebordao, "PyWolf" (arXiv 2203.02734): a source CSD array
W[i1, j1, i2, j2] (Sec. 3.1) propagated in the Fresnel or far-field approximation (Sec. 2.1,
Sec. 3.4), then the spectral density and the degree of coherence (Sec. 3.5).
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Tuple

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libwolf.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE = 0, -1, -2, -3, -4
C64, C128 = 0, 1
SECONDARY, PRIMARY = 0, 1
MODEL_GSM, MODEL_MAP, MODEL_COHERENT, MODEL_INCOHERENT = 0, 1, 2, 3
GEO_NONE, GEO_CIRCLE, GEO_SQUARE, GEO_ANNULUS, GEO_MASK = 0, 1, 2, 3, 4

EXPORTED = ["wolf_build_source", "wolf_propagate_fresnel", "wolf_propagate_farfield", "wolf_propagate_adjoint",
            "wolf_spectral_density", "wolf_degree_of_coherence", "wolf_propagate_batch", "wolf_chirp_table",
            "wolf_output_pitch", "wolf_status_string", "wolf_last_error_message", "wolf_version",
            "wolf_set_plan", "wolf_get_plan", "wolf_autotune", "wolf_diag_embed", "wolf_fit_gradient",
            "wolf_fit_work_bytes", "wolf_coop_error_flag", "wolf_propagate_adjoint_diag", "wolf_batch_work_bytes",
            "wolf_propagate_lens", "wolf_propagate_direct", "wolf_direct_work_bytes",
            "wolf_propagate_padded", "wolf_propagate_polychromatic", "wolf_polychromatic_work_bytes",
            "wolf_propagate_source", "wolf_memory_ceiling", "wolf_degree_of_coherence_noalloc"]


class WolfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed with status {status}: {detail}")
        self.status = status


class _Source(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("geometry", ctypes.c_int32), ("amplitude", ctypes.c_double),
                ("sigma_s_m", ctypes.c_double), ("sigma_g_m", ctypes.c_double), ("geo_r0_m", ctypes.c_double),
                ("geo_r1_m", ctypes.c_double), ("intensity_map", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("lens_focal_m", ctypes.c_double), ("wavelength_m", ctypes.c_double)]


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libwolf.so (once). Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libwolf.so not found at {path}; build it with paper_2203_02734_amd.build.build()")
    lib = ctypes.CDLL(path)
    i32, f64, vp = ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "wolf_build_source": [ctypes.POINTER(_Source), i32, f64, i32, vp, vp],
        "wolf_propagate_source": [ctypes.POINTER(_Source), i32, f64, f64, f64, i32, i32, i32, vp, pd, vp],
        "wolf_propagate_fresnel": [vp, vp, i32, f64, f64, f64, i32, i32, pd, vp],
        "wolf_propagate_farfield": [vp, vp, i32, f64, f64, f64, i32, i32, pd, vp],
        "wolf_propagate_lens": [vp, vp, i32, f64, f64, f64, i32, f64, f64, i32, i32, pd, vp],
        "wolf_propagate_direct": [vp, vp, i32, f64, f64, f64, i32, i32, vp, pd, vp],
        "wolf_propagate_padded": [vp, vp, i32, i32, f64, f64, f64, i32, i32, i32, vp, pd, vp],
        "wolf_propagate_adjoint": [vp, vp, i32, f64, f64, f64, i32, i32, i32, vp],
        "wolf_propagate_adjoint_diag": [vp, vp, i32, f64, f64, f64, i32, i32, i32, vp],
        "wolf_spectral_density": [vp, i32, i32, vp, vp],
        "wolf_degree_of_coherence": [vp, i32, i32, i32, i32, f64, vp, vp],
        "wolf_degree_of_coherence_noalloc": [vp, i32, i32, i32, i32, f64, vp, vp],
        "wolf_propagate_batch": [vp, i32, f64, i32, pd, pd, pd, i32, i32, i32, i32, i32, f64, vp, vp, vp, vp],
        "wolf_propagate_polychromatic": [vp, i32, f64, i32, pd, pd, pd, f64, i32, i32, i32, i32, i32, f64, vp, vp, vp,
                                         vp],
        "wolf_chirp_table": [i32, f64, f64, f64, i32, vp, vp],
        "wolf_set_plan": [i32, i32, i32, ctypes.c_int64, ctypes.c_int64, i32, i32],
        "wolf_get_plan": [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "wolf_coop_error_flag": [vp, ctypes.POINTER(i32)],
        "wolf_autotune": [i32, i32, vp, i32, pd, vp],
        "wolf_diag_embed": [vp, i32, i32, vp, vp],
        "wolf_fit_gradient": [vp, vp, i32, f64, f64, i32, vp, vp, vp, vp],
        "wolf_memory_ceiling": [vp, ctypes.c_int64, i32, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    lib.wolf_output_pitch.argtypes = [i32, f64, f64, f64]
    lib.wolf_output_pitch.restype = f64
    lib.wolf_status_string.argtypes = [i32]
    lib.wolf_status_string.restype = ctypes.c_char_p
    lib.wolf_last_error_message.argtypes = []
    lib.wolf_last_error_message.restype = ctypes.c_char_p
    lib.wolf_version.restype = i32
    lib.wolf_fit_work_bytes.argtypes = [i32, i32]
    lib.wolf_fit_work_bytes.restype = ctypes.c_int64
    lib.wolf_batch_work_bytes.argtypes = [i32, i32]
    lib.wolf_batch_work_bytes.restype = ctypes.c_int64
    lib.wolf_direct_work_bytes.argtypes = [i32, i32]
    lib.wolf_direct_work_bytes.restype = ctypes.c_int64
    lib.wolf_polychromatic_work_bytes.argtypes = [i32, i32]
    lib.wolf_polychromatic_work_bytes.restype = ctypes.c_int64
    _lib = lib
    return lib


def _check(status: int, where: str) -> None:
    if status != OK:
        lib = load()
        raise WolfError(status, where, lib.wolf_last_error_message().decode() or lib.wolf_status_string(status).decode())


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _code(dtype: torch.dtype) -> int:
    if dtype == torch.complex64:
        return C64
    if dtype == torch.complex128:
        return C128
    raise TypeError(f"unsupported dtype {dtype}; use torch.complex64 or torch.complex128")


def _real(dtype: torch.dtype) -> torch.dtype:
    return torch.float32 if dtype == torch.complex64 else torch.float64


def _csd(w: torch.Tensor, name: str = "w") -> int:
    if not (isinstance(w, torch.Tensor) and w.is_cuda):
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if w.dim() != 4 or len(set(w.shape)) != 1:
        raise ValueError(f"{name} must have shape (N, N, N, N)")
    if not w.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    _code(w.dtype)
    return w.shape[0]


def _out(out: torch.Tensor, shape, dtype: torch.dtype, device, name: str = "out") -> torch.Tensor:
    """Checks a caller's output tensor against the call: a contiguous tensor of exactly `shape` and
    `dtype` on `device`. The library only checks that a buffer lies inside one device allocation, and
    torch's caching allocator places many tensors in one allocation, so a wrong shape or dtype here
    would let the kernels write into neighbouring tensors."""
    if not (isinstance(out, torch.Tensor) and out.is_cuda):
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if tuple(out.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(out.shape)}")
    if out.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {out.dtype}")
    if not out.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and out.device != torch.device(device):
        raise ValueError(f"{name} is on {out.device}, expected {device}")
    return out


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else None)


def output_pitch(n: int, pitch: float, wavelength: float, z: float) -> float:
    """eq. (spatial_resolution): dx = lambda z / (N pitch)."""
    return load().wolf_output_pitch(n, pitch, wavelength, z)


def build_source(spec, n: int, pitch: float, dtype: torch.dtype = torch.complex64,
                 out: Optional[torch.Tensor] = None, device=None) -> torch.Tensor:
    """Source CSD array W0 (Sec. 3.2). `spec` has the fields of wolf_source (see include/wolf.h):
    model, amplitude, sigma_s_m, sigma_g_m, geometry, geo_r0_m, geo_r1_m, intensity_map, mask,
    lens_focal_m, wavelength_m. A host intensity map or mask is copied to the device."""
    lib = load()
    dev = torch.device(device) if device is not None else (out.device if out is not None else torch.device("cuda"))
    if out is None:
        out = torch.empty((n, n, n, n), dtype=dtype, device=dev)
    else:
        _code(out.dtype)
        _out(out, (n, n, n, n), out.dtype, dev)
    s, _keep = _source_struct(spec, out.device, n)
    _check(lib.wolf_build_source(ctypes.byref(s), n, pitch, _code(out.dtype), _ptr(out), _stream()),
           "wolf_build_source")
    # The uploaded map/mask may be freed now: the caching allocator orders their reuse after this
    # kernel on the same stream.
    return out


def _source_struct(spec, device, n: int):
    """wolf_source for `spec`, with a host intensity map or mask copied to `device` (the tensors are
    returned so that they outlive the call). A map or mask must be (n, n)."""
    imap = getattr(spec, "intensity_map", None)
    mask = getattr(spec, "mask", None)
    imap_t = None if imap is None else torch.as_tensor(np.asarray(imap) if not isinstance(imap, torch.Tensor) else imap,
                                                       dtype=torch.float32).to(device).contiguous()
    mask_t = None if mask is None else torch.as_tensor(np.asarray(mask) if not isinstance(mask, torch.Tensor) else mask,
                                                       dtype=torch.uint8).to(device).contiguous()
    for t, name in ((imap_t, "intensity_map"), (mask_t, "mask")):
        if t is not None and tuple(t.shape) != (n, n):
            raise ValueError(f"{name} must have shape ({n}, {n}), got {tuple(t.shape)}")
    s = _Source(int(spec.model), int(spec.geometry), float(spec.amplitude), float(spec.sigma_s_m),
                float(spec.sigma_g_m), float(spec.geo_r0_m), float(spec.geo_r1_m),
                imap_t.data_ptr() if imap_t is not None else None, mask_t.data_ptr() if mask_t is not None else None,
                float(spec.lens_focal_m), float(spec.wavelength_m))
    return s, (imap_t, mask_t)


def propagate_source(spec, n: int, pitch: float, wavelength: float, z: float, farfield: bool = False,
                     kind: int = SECONDARY, dtype: torch.dtype = torch.complex64,
                     out: Optional[torch.Tensor] = None, device=None) -> Tuple[torch.Tensor, float]:
    """The source of `spec` (as build_source) propagated over z in the Fresnel or far-field form, in
    one call: equal to build_source followed by the in-place propagation, without W0 in memory where
    the slab pass forms it. Returns (W_B, dx)."""
    lib = load()
    dev = torch.device(device) if device is not None else (out.device if out is not None else torch.device("cuda"))
    if out is None:
        out = torch.empty((n, n, n, n), dtype=dtype, device=dev)
    else:
        _code(out.dtype)
        _out(out, (n, n, n, n), out.dtype, dev)
    s, _keep = _source_struct(spec, out.device, n)
    dx = ctypes.c_double(0.0)
    _check(lib.wolf_propagate_source(ctypes.byref(s), n, pitch, wavelength, z, int(bool(farfield)), kind,
                                     _code(out.dtype), _ptr(out), ctypes.byref(dx), _stream()),
           "wolf_propagate_source")
    return out, dx.value


def _propagate(fn_name: str, w: torch.Tensor, pitch: float, wavelength: float, z: float, kind: int,
               out: Optional[torch.Tensor]) -> Tuple[torch.Tensor, float]:
    lib = load()
    n = _csd(w)
    if out is None:
        out = torch.empty_like(w)
    else:
        _out(out, w.shape, w.dtype, w.device)
    dx = ctypes.c_double(0.0)
    _check(getattr(lib, fn_name)(_ptr(w), _ptr(out), n, pitch, wavelength, z, kind, _code(w.dtype),
                                 ctypes.byref(dx), _stream()), fn_name)
    return out, dx.value


def propagate_fresnel(w: torch.Tensor, pitch: float, wavelength: float, z: float, kind: int = SECONDARY,
                      out: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, float]:
    """Fresnel propagation over z (Sec. 2.1 eq. W_fresnel; Algorithm 2). Returns (W_B, dx)."""
    return _propagate("wolf_propagate_fresnel", w, pitch, wavelength, z, kind, out)


def propagate_farfield(w: torch.Tensor, pitch: float, wavelength: float, z: float, kind: int = SECONDARY,
                       out: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, float]:
    """Far-field propagation (Sec. 2.1 eq. W_farfield). Returns (W_B, dx)."""
    return _propagate("wolf_propagate_farfield", w, pitch, wavelength, z, kind, out)


def propagate(w, pitch, wavelength, z, farfield=False, kind=SECONDARY, out=None):
    return (propagate_farfield if farfield else propagate_fresnel)(w, pitch, wavelength, z, kind, out)


def propagate_lens(w: torch.Tensor, pitch: float, wavelength: float, focal: float, z: float,
                   pupil_geometry: int = GEO_NONE, pupil_radius: float = 0.0, kind: int = SECONDARY,
                   out: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, float]:
    """Thin lens T = P q*(f) at the plane of w (pitch `pitch`), then Fresnel propagation by z
    (Sec. 2.2). focal = 0: pupil only. Returns (W, dx)."""
    lib = load()
    n = _csd(w, "w")
    if out is None:
        out = torch.empty_like(w)
    else:
        _out(out, w.shape, w.dtype, w.device)
    dx = ctypes.c_double(0.0)
    _check(lib.wolf_propagate_lens(_ptr(w), _ptr(out), n, pitch, wavelength, focal, pupil_geometry, pupil_radius,
                                   z, kind, _code(w.dtype), ctypes.byref(dx), _stream()), "wolf_propagate_lens")
    return out, dx.value


def image_through_lens(w: torch.Tensor, pitch: float, wavelength: float, r1: float, focal: float, r2: float,
                       pupil_geometry: int = GEO_NONE, pupil_radius: float = 0.0, kind: int = SECONDARY,
                       out: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, float]:
    """Source plane -> lens plane (Fresnel, r1) -> thin lens with pupil -> image plane (Fresnel, r2):
    eqs. WA_imaging and WC_imaging. Two operator launches; the second runs in place on `out`.
    The pupil radius is in metres on the lens plane. Returns (W_C, pitch at the image plane)."""
    wb, pb = propagate_fresnel(w, pitch, wavelength, r1, kind, out)
    return propagate_lens(wb, pb, wavelength, focal, r2, pupil_geometry, pupil_radius, kind, out=wb)


def propagate_direct(w: torch.Tensor, pitch: float, wavelength: float, z: float, kind: int = SECONDARY,
                     out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, float]:
    """Direct sum with the exact free-space kernel (eq. h_free), on the output grid of
    propagate_fresnel: the reference for the error of the Fresnel approximation. Returns (W_B, dx)."""
    lib = load()
    n = _csd(w, "w")
    if out is None:
        out = torch.empty_like(w)
    else:
        _out(out, w.shape, w.dtype, w.device)
    nbytes = int(lib.wolf_direct_work_bytes(n, _code(w.dtype)))
    if nbytes < 0:
        raise WolfError(EUNSUPPORTED, "wolf_direct_work_bytes", f"N={n} unsupported")
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=w.device)
    dx = ctypes.c_double(0.0)
    _check(lib.wolf_propagate_direct(_ptr(w), _ptr(out), n, pitch, wavelength, z, kind, _code(w.dtype), _ptr(work),
                                     ctypes.byref(dx), _stream()), "wolf_propagate_direct")
    return out, dx.value


def fresnel_validity(w: torch.Tensor, pitch: float, wavelength: float, z: float, kind: int = SECONDARY) -> dict:
    """Error of the Fresnel propagation of w against the exact-kernel direct sum (eqs. h_free,
    approx_L): relative L2 distance of W_B and of S_B, and the largest difference of S_B relative
    to max S_B. Both propagations run in the library; the norms are taken on the device."""
    wd, _ = propagate_direct(w, pitch, wavelength, z, kind)
    wf, _ = propagate_fresnel(w, pitch, wavelength, z, kind)
    sd, sf = spectral_density(wd), spectral_density(wf)
    d = {"rel_l2_w": float(torch.linalg.vector_norm(wf - wd) / torch.linalg.vector_norm(wd)),
         "rel_l2_s": float(torch.linalg.vector_norm(sf - sd) / torch.linalg.vector_norm(sd)),
         "max_s_rel": float((sf - sd).abs().max() / sd.abs().max())}
    return d


def propagate_padded(w: torch.Tensor, pitch: float, wavelength: float, z: float, n_fft: Optional[int] = None,
                     farfield: bool = False, kind: int = SECONDARY, out: Optional[torch.Tensor] = None,
                     work: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, float]:
    """Propagation for any even N, with zero padding of the transform to n_fft points and the result
    cropped back to N (Sec. 3.3; n_fft = N by default). Returns (W_B, dx), dx = lambda z / (n_fft pitch)."""
    lib = load()
    n = _csd(w, "w")
    if out is None:
        out = torch.empty_like(w)
    else:
        _out(out, w.shape, w.dtype, w.device)
    if work is None:
        work = torch.empty_like(w)
    dx = ctypes.c_double(0.0)
    _check(lib.wolf_propagate_padded(_ptr(w), _ptr(out), n, n if n_fft is None else int(n_fft), pitch, wavelength, z,
                                     int(bool(farfield)), kind, _code(w.dtype), _ptr(work), ctypes.byref(dx),
                                     _stream()), "wolf_propagate_padded")
    return out, dx.value


def propagate_adjoint(g: torch.Tensor, pitch: float, wavelength: float, z: float, farfield: bool = False,
                      kind: int = SECONDARY, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Adjoint of the propagation (gradient of W_B mapped to the gradient of W_A)."""
    lib = load()
    n = _csd(g, "g")
    if out is None:
        out = torch.empty_like(g)
    else:
        _out(out, g.shape, g.dtype, g.device)
    _check(lib.wolf_propagate_adjoint(_ptr(g), _ptr(out), n, pitch, wavelength, z, int(bool(farfield)), kind,
                                      _code(g.dtype), _stream()), "wolf_propagate_adjoint")
    return out


def propagate_adjoint_diag(g: torch.Tensor, pitch: float, wavelength: float, z: float, farfield: bool = False,
                           kind: int = SECONDARY, dtype: torch.dtype = torch.complex64,
                           out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Adjoint propagation of diag(g) for a real (N, N) g (the gradient of a loss of S_B)."""
    lib = load()
    n = g.shape[0]
    if g.shape != (n, n) or g.dtype != _real(dtype) or not g.is_cuda or not g.is_contiguous():
        raise ValueError("g must be a contiguous CUDA (N, N) tensor of the matching real dtype")
    if out is None:
        out = torch.empty((n, n, n, n), dtype=dtype, device=g.device)
    else:
        _out(out, (n, n, n, n), dtype, g.device)
    _check(lib.wolf_propagate_adjoint_diag(_ptr(g), _ptr(out), n, pitch, wavelength, z, int(bool(farfield)), kind,
                                           _code(dtype), _stream()), "wolf_propagate_adjoint_diag")
    return out


def spectral_density(w: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """S[i, j] = Re W[i, j; i, j] (Algorithm 4)."""
    lib = load()
    n = _csd(w)
    if out is None:
        out = torch.empty((n, n), dtype=_real(w.dtype), device=w.device)
    else:
        _out(out, (n, n), _real(w.dtype), w.device)
    _check(lib.wolf_spectral_density(_ptr(w), n, _code(w.dtype), _ptr(out), _stream()), "wolf_spectral_density")
    return out


def degree_of_coherence(w: torch.Tensor, ip: int = -1, jp: int = -1, floor_rel: float = 1e-12,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """mu(P1, .) for P1 = (ip, jp) (Algorithm 5), or the full N^4 mu when ip = jp = -1."""
    lib = load()
    n = _csd(w)
    shape = (n, n, n, n) if (ip == -1 and jp == -1) else (n, n)
    if out is None:
        out = torch.empty(shape, dtype=w.dtype, device=w.device)
    else:
        _out(out, shape, w.dtype, w.device)
    _check(lib.wolf_degree_of_coherence(_ptr(w), n, _code(w.dtype), ip, jp, floor_rel, _ptr(out), _stream()),
           "wolf_degree_of_coherence")
    return out


def chirp_table(n: int, pitch: float, wavelength: float, z: float, dtype: torch.dtype = torch.complex128,
                device=None) -> torch.Tensor:
    """FP64-built q(z, pitch (i - N/2)) along one axis (eq. q_factor)."""
    lib = load()
    out = torch.empty((n,), dtype=dtype, device=device or torch.device("cuda"))
    _check(lib.wolf_chirp_table(n, pitch, wavelength, z, _code(dtype), _ptr(out), _stream()), "wolf_chirp_table")
    return out


def propagate_batch(w_src: torch.Tensor, pitch: float, wavelengths, zs, weights, farfield: bool = False,
                    kind: int = SECONDARY, ip: int = 0, jp: int = 0, floor_rel: float = 1e-12,
                    work: Optional[torch.Tensor] = None):
    """All (lambda, z) pairs of one source: returns (S[k], mu[k]) stacked over pairs."""
    lib = load()
    n = _csd(w_src, "w_src")
    lam = np.ascontiguousarray(wavelengths, dtype=np.float64)
    zz = np.ascontiguousarray(zs, dtype=np.float64)
    ww = np.ascontiguousarray(weights, dtype=np.float64)
    if not (lam.shape == zz.shape == ww.shape and lam.ndim == 1):
        raise ValueError("wavelengths, zs and weights must be 1D arrays of the same length")
    k = lam.shape[0]
    if work is None:
        work = torch.empty(batch_work_bytes(n, w_src.dtype), dtype=torch.uint8, device=w_src.device)
    s = torch.empty((k, n, n), dtype=_real(w_src.dtype), device=w_src.device)
    mu = torch.empty((k, n, n), dtype=w_src.dtype, device=w_src.device)
    pd = ctypes.POINTER(ctypes.c_double)
    _check(lib.wolf_propagate_batch(_ptr(w_src), n, pitch, k, lam.ctypes.data_as(pd), zz.ctypes.data_as(pd),
                                    ww.ctypes.data_as(pd), int(bool(farfield)), kind, _code(w_src.dtype), ip, jp,
                                    floor_rel, _ptr(work), _ptr(s), _ptr(mu), _stream()), "wolf_propagate_batch")
    return s, mu


def propagate_polychromatic(w_src: torch.Tensor, pitch: float, wavelengths, zs, weights, out_pitch: float,
                            farfield: bool = False, kind: int = SECONDARY, ip: int = 0, jp: int = 0,
                            floor_rel: float = 1e-12, work: Optional[torch.Tensor] = None):
    """Polychromatic light on a common output grid of pitch out_pitch: S and mu(P1, .) of
    sum_k weights[k] W_k, W_k the source propagated at (wavelengths[k], zs[k]). Returns (S, mu), N x N each."""
    lib = load()
    n = _csd(w_src, "w_src")
    lam = np.ascontiguousarray(wavelengths, dtype=np.float64)
    zz = np.ascontiguousarray(zs, dtype=np.float64)
    ww = np.ascontiguousarray(weights, dtype=np.float64)
    if not (lam.shape == zz.shape == ww.shape and lam.ndim == 1):
        raise ValueError("wavelengths, zs and weights must be 1D arrays of the same length")
    if work is None:
        work = torch.empty(polychromatic_work_bytes(n, w_src.dtype), dtype=torch.uint8, device=w_src.device)
    s = torch.empty((n, n), dtype=_real(w_src.dtype), device=w_src.device)
    mu = torch.empty((n, n), dtype=w_src.dtype, device=w_src.device)
    pd = ctypes.POINTER(ctypes.c_double)
    _check(lib.wolf_propagate_polychromatic(_ptr(w_src), n, pitch, lam.shape[0], lam.ctypes.data_as(pd),
                                            zz.ctypes.data_as(pd), ww.ctypes.data_as(pd), float(out_pitch),
                                            int(bool(farfield)), kind, _code(w_src.dtype), ip, jp, floor_rel,
                                            _ptr(work), _ptr(s), _ptr(mu), _stream()), "wolf_propagate_polychromatic")
    return s, mu


def polychromatic_work_bytes(n: int, dtype: torch.dtype) -> int:
    """Bytes of the `work` buffer that propagate_polychromatic needs for (n, dtype)."""
    b = int(load().wolf_polychromatic_work_bytes(n, _code(dtype)))
    if b < 0:
        raise WolfError(EUNSUPPORTED, "wolf_polychromatic_work_bytes", f"N={n} unsupported")
    return b


def batch_work_bytes(n: int, dtype: torch.dtype) -> int:
    """Bytes of the `work` buffer that propagate_batch needs for (n, dtype)."""
    b = int(load().wolf_batch_work_bytes(n, _code(dtype)))
    if b < 0:
        raise WolfError(EUNSUPPORTED, "wolf_batch_work_bytes", f"N={n} unsupported")
    return b


def set_plan(n: int, dtype: torch.dtype, fused_slab: int = -1, slab_chunk: int = -1, col_chunk: int = -1,
             coop_cols: int = 0, coop_lookahead: int = 1) -> None:
    """Fix the pass schedule for (n, dtype); fused_slab = slab_chunk = col_chunk = -1 restores the
    default (see include/wolf.h)."""
    _check(load().wolf_set_plan(n, _code(dtype), fused_slab, slab_chunk, col_chunk, coop_cols, coop_lookahead),
           "wolf_set_plan")


def get_plan(n: int, dtype: torch.dtype):
    f, s, c, w, la = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().wolf_get_plan(n, _code(dtype), ctypes.byref(f), ctypes.byref(s), ctypes.byref(c), ctypes.byref(w),
                                ctypes.byref(la)), "wolf_get_plan")
    return {"fused_slab": f.value, "slab_chunk": s.value, "col_chunk": c.value, "coop_cols": w.value,
            "coop_lookahead": la.value}


def coop_error_flag() -> int:
    """1 if a cooperative pass on the current stream timed out waiting for a tile (synchronises)."""
    f = ctypes.c_int32()
    _check(load().wolf_coop_error_flag(_stream(), ctypes.byref(f)), "wolf_coop_error_flag")
    return f.value


def autotune(n: int, dtype: torch.dtype = torch.complex64, reps: int = 3, work: Optional[torch.Tensor] = None):
    """Time the candidate schedules for (n, dtype) on a scratch array and keep the fastest.
    Returns (plan, best ms)."""
    if work is None:
        work = torch.empty((n, n, n, n), dtype=dtype, device="cuda")
    best = ctypes.c_double(0.0)
    _check(load().wolf_autotune(n, _code(dtype), _ptr(work), reps, ctypes.byref(best), _stream()), "wolf_autotune")
    return get_plan(n, dtype), best.value


def memory_ceiling(buf: torch.Tensor, mode: int = 0) -> None:
    """One streaming pass over the bytes of `buf` (0: read and write in place, 1: write zeros, 2: read;
    3, 4, 5: the same with nontemporal loads and stores): a measurement aid for the memory ceilings
    (see include/wolf.h)."""
    if not (buf.is_cuda and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous CUDA tensor")
    _check(load().wolf_memory_ceiling(_ptr(buf), buf.numel() * buf.element_size(), mode, _stream()),
           "wolf_memory_ceiling")


def diag_embed(g: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    """out[p1; p2] = g[p1] delta(p1, p2): the gradient with respect to W of a loss of S = Re diag(W)."""
    n = g.shape[0]
    if g.shape != (n, n) or g.dtype != _real(dtype) or not g.is_cuda or not g.is_contiguous():
        raise ValueError("g must be a contiguous CUDA (N, N) tensor of the matching real dtype")
    out = torch.empty((n, n, n, n), dtype=dtype, device=g.device)
    _check(load().wolf_diag_embed(_ptr(g), n, _code(dtype), _ptr(out), _stream()), "wolf_diag_embed")
    return out


def fit_gradient(ga: torch.Tensor, imap: torch.Tensor, pitch: float, sigma_g: float):
    """(dL/dI, dL/dsigma_g) of the custom-map source from G_A = dL/dW_A (see include/wolf.h)."""
    lib = load()
    n = _csd(ga, "ga")
    if imap.shape != (n, n) or imap.dtype != torch.float32 or not imap.is_cuda or not imap.is_contiguous():
        raise ValueError("imap must be a contiguous CUDA float32 (N, N) tensor")
    nbytes = lib.wolf_fit_work_bytes(n, _code(ga.dtype))
    if nbytes < 0:
        raise WolfError(EUNSUPPORTED, "wolf_fit_gradient", f"N={n} unsupported")
    work = torch.empty((nbytes,), dtype=torch.uint8, device=ga.device)
    d_imap = torch.empty((n, n), dtype=torch.float32, device=ga.device)
    d_sigma = torch.empty((1,), dtype=torch.float64, device=ga.device)
    _check(lib.wolf_fit_gradient(_ptr(ga), _ptr(imap), n, pitch, sigma_g, _code(ga.dtype), _ptr(work), _ptr(d_imap),
                                 _ptr(d_sigma), _stream()), "wolf_fit_gradient")
    return d_imap, d_sigma
