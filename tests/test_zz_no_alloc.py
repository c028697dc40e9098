"""The allocation-free degree of coherence (wolf_degree_of_coherence_noalloc, for callers that cannot
allocate) against the allocating entry point (wolf_degree_of_coherence), through the C ABI: the same
kernels on the same input give the same result bit for bit. Two calls in a row, the second with a
smaller input, so that the static scratch holds the first call's contents when the second starts;
slices and the full 4D mu; both precisions. Also its argument checks."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import wolf_inputs as WI

pytestmark = pytest.mark.gpu

LAM = WI.LAMBDA_HENE


def _call(lib, name, w, ip, jp, floor, out):
    code = 0 if w.dtype == torch.complex64 else 1
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(lib, name)(ctypes.c_void_p(w.data_ptr()), w.shape[0], code, ip, jp, floor,
                              ctypes.c_void_p(out.data_ptr()), st)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_noalloc_mu_equals_allocating_entry(gpu_lib, dtype):
    lib = gpu_lib.load()
    p, z, floor = 20e-6, 0.3, 1e-6
    sp = WI.gsm_small()[0].source
    for n, (ip, jp) in ((32, (16, 16)), (16, (5, 9))):          # the second call is smaller
        print("noalloc mu", dtype, n, flush=True)
        w = gpu_lib.build_source(sp, n, p, dtype)
        gpu_lib.propagate_fresnel(w, p, LAM, z, out=w)
        for i, j in ((ip, jp), (-1, -1)):
            shape = (n, n, n, n) if i < 0 else (n, n)
            a = torch.empty(shape, dtype=dtype, device="cuda").fill_(complex(float("nan"), 0.0))
            b = torch.empty(shape, dtype=dtype, device="cuda").fill_(complex(float("nan"), 0.0))
            assert _call(lib, "wolf_degree_of_coherence_noalloc", w, i, j, floor, a) == 0, \
                lib.wolf_last_error_message()
            assert _call(lib, "wolf_degree_of_coherence", w, i, j, floor, b) == 0
            torch.cuda.synchronize()
            assert torch.equal(a, b), (n, i, j)
        # The slice against the oracle, as the allocating entry point is checked.
        wb = w.cpu().numpy().astype(np.complex128)
        ref = O.degree_of_coherence(wb, ip, jp, floor)
        got = torch.empty((n, n), dtype=dtype, device="cuda")
        assert _call(lib, "wolf_degree_of_coherence_noalloc", w, ip, jp, floor, got) == 0
        torch.cuda.synchronize()
        err = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err < (1e-5 if dtype == torch.complex64 else 1e-12), err


def test_noalloc_mu_rejects_invalid_arguments(gpu_lib):
    lib = gpu_lib.load()
    n = 8
    w = torch.zeros((n,) * 4, dtype=torch.complex64, device="cuda")
    mu = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    assert _call(lib, "wolf_degree_of_coherence_noalloc", w, n, 0, 1e-6, mu) == -1       # P1 out of range
    assert _call(lib, "wolf_degree_of_coherence_noalloc", w, 0, 0, -1.0, mu) == -1       # negative floor
    # A full mu into a buffer of one slice: the ABI sees the allocation, so the buffer gets one of its own
    # (inside torch's caching allocator it would share a larger segment).
    hip = ctypes.CDLL("libamdhip64.so")
    ptr = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(8 * n * n)) == 0
    try:
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        assert lib.wolf_degree_of_coherence_noalloc(ctypes.c_void_p(w.data_ptr()), n, 0, -1, -1, 1e-6, ptr, st) == -1
        assert b"too small" in lib.wolf_last_error_message()
    finally:
        hip.hipFree(ptr)
