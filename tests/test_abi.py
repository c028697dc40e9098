"""CPU checks of the C-ABI boundary: the library loads, exports every symbol the header declares,
and validates arguments before touching the device. No compute call needs a GPU here."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wolf.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2203_02734_amd as wolf
    if not os.path.exists(wolf.LIB_PATH):
        from paper_2203_02734_amd import build
        build.build()
    return wolf.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"WOLF_API\s+[\w\s\*]+?\b(wolf_\w+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_symbols()
    for required in ["wolf_build_source", "wolf_propagate_fresnel", "wolf_propagate_farfield",
                     "wolf_spectral_density", "wolf_degree_of_coherence", "wolf_propagate_adjoint"]:
        assert required in names


def test_exports_every_declared_symbol(lib):
    import paper_2203_02734_amd as wolf
    out = subprocess.run(["nm", "-D", "--defined-only", wolf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (wolf_\w+)", out))
    for name in declared_symbols():
        assert name in exported, name
        assert hasattr(lib, name)
    # Nothing but the C-ABI is exported.
    assert all(n.startswith("wolf_") for n in re.findall(r" T (\w+)", out))


def test_binding_covers_header(lib):
    import paper_2203_02734_amd as wolf
    assert set(declared_symbols()) == set(wolf.EXPORTED)


def test_status_strings_and_version(lib):
    assert lib.wolf_version() >= 1
    for code in [0, -1, -2, -3, -4]:
        assert lib.wolf_status_string(code).startswith(b"WOLF_")


def test_output_pitch_matches_paper_relation(lib):
    # eq. (spatial_resolution), example 4 (Table 1): dx = lambda R / (N dxi) ~ dxi.
    import oracle as O
    lam = O.wavelength_from_omega(2.992e15)
    assert lib.wolf_output_pitch(200, 1e-4, lam, 3.1746) == pytest.approx(O.output_pitch(200, 1e-4, lam, 3.1746),
                                                                          rel=1e-15)


@pytest.mark.parametrize("n", [0, 1, 3, 12, 200, 512, -4])
def test_unsupported_sizes_fft_path(lib, n):
    """The FFT-based operator takes powers of two in [2, 256]."""
    assert lib.wolf_propagate_fresnel(None, None, n, 1e-5, 5e-7, 0.1, 0, 0, None, None) == -2
    assert lib.wolf_propagate_farfield(None, None, n, 1e-5, 5e-7, 0.1, 0, 0, None, None) == -2
    assert lib.wolf_propagate_adjoint(None, None, n, 1e-5, 5e-7, 0.1, 0, 0, 0, None) == -2


@pytest.mark.parametrize("n", [0, 1, 3, 5, 258, 512, -4])
def test_unsupported_sizes_any_even(lib, n):
    """The builder, the observables and the padded operator take any even N in [2, 256]."""
    assert lib.wolf_spectral_density(None, n, 0, None, None) == -2
    assert lib.wolf_degree_of_coherence(None, n, 0, 0, 0, 1e-12, None, None) == -2
    assert lib.wolf_chirp_table(n, 1e-5, 5e-7, 0.1, 0, None, None) == -2
    assert lib.wolf_propagate_padded(None, None, n, 512, 1e-5, 5e-7, 0.1, 0, 0, 0, None, None, None) == -2


@pytest.mark.parametrize("args", [
    (16, 0.0, 5e-7, 0.1), (16, -1e-5, 5e-7, 0.1), (16, 1e-5, 0.0, 0.1), (16, 1e-5, 5e-7, 0.0),
    (16, float("nan"), 5e-7, 0.1), (16, 1e-5, float("inf"), 0.1), (16, 1e-5, 5e-7, -3.0)])
def test_invalid_physics_arguments(lib, args):
    n, p, lam, z = args
    assert lib.wolf_propagate_fresnel(None, None, n, p, lam, z, 0, 0, None, None) == -1
    assert lib.wolf_chirp_table(n, p, lam, z, 0, None, None) == -1


def test_invalid_enums_and_nulls(lib):
    assert lib.wolf_propagate_fresnel(None, None, 16, 1e-5, 5e-7, 0.1, 0, 7, None, None) == -1   # dtype
    assert lib.wolf_propagate_fresnel(None, None, 16, 1e-5, 5e-7, 0.1, 5, 0, None, None) == -1   # kind
    assert lib.wolf_propagate_fresnel(None, None, 16, 1e-5, 5e-7, 0.1, 0, 0, None, None) == -1   # null
    assert b"null" in lib.wolf_last_error_message()
    assert lib.wolf_propagate_adjoint(None, None, 16, 1e-5, 5e-7, 0.1, 2, 0, 0, None) == -1      # farfield flag
    assert lib.wolf_degree_of_coherence(None, 16, 0, 16, 0, 1e-12, None, None) == -1             # ip range
    assert lib.wolf_degree_of_coherence(None, 16, 0, -1, 3, 1e-12, None, None) == -1
    assert lib.wolf_degree_of_coherence(None, 16, 0, 0, 0, -1.0, None, None) == -1               # floor
    assert lib.wolf_build_source(None, 16, 1e-5, 0, None, None) == -1


def test_build_source_validation(lib):
    import paper_2203_02734_amd as wolf
    S = wolf._Source
    bad = [S(9, 0, 1.0, 1e-4, 1e-4, 0, 0, None, None, 0, 0),       # model
           S(0, 9, 1.0, 1e-4, 1e-4, 0, 0, None, None, 0, 0),       # geometry
           S(0, 0, -1.0, 1e-4, 1e-4, 0, 0, None, None, 0, 0),      # amplitude
           S(0, 0, 1.0, 0.0, 1e-4, 0, 0, None, None, 0, 0),        # sigma_s
           S(0, 0, 1.0, 1e-4, -1.0, 0, 0, None, None, 0, 0),       # sigma_g
           S(0, 1, 1.0, 1e-4, 1e-4, 0.0, 0, None, None, 0, 0),     # circle radius
           S(0, 3, 1.0, 1e-4, 1e-4, 1e-4, 2e-4, None, None, 0, 0), # annulus r1 >= r0
           S(0, 0, 1.0, 1e-4, 1e-4, 0, 0, None, None, 0.2, 0.0),   # lens without wavelength
           S(1, 0, 1.0, 1e-4, 1e-4, 0, 0, None, None, 0, 0),       # map without a device map
           S(0, 4, 1.0, 1e-4, 1e-4, 0, 0, None, None, 0, 0)]       # mask without a device mask
    for s in bad:
        assert lib.wolf_build_source(ctypes.byref(s), 16, 1e-5, 0, None, None) == -1


def test_propagate_source_validation(lib):
    """wolf_propagate_source checks its size, physics, flags and source before any device work."""
    import paper_2203_02734_amd as wolf
    S = wolf._Source
    good = S(0, 0, 1.0, 1e-4, 1e-4, 0, 0, None, None, 0, 0)
    for n in (0, 1, 3, 12, 200, 512, -4):
        assert lib.wolf_propagate_source(ctypes.byref(good), n, 1e-5, 5e-7, 0.1, 0, 0, 0, None, None, None) == -2
    for p, lam, z in ((0.0, 5e-7, 0.1), (1e-5, -5e-7, 0.1), (1e-5, 5e-7, float("nan")), (1e-5, 5e-7, 0.0)):
        assert lib.wolf_propagate_source(ctypes.byref(good), 16, p, lam, z, 0, 0, 0, None, None, None) == -1
    assert lib.wolf_propagate_source(ctypes.byref(good), 16, 1e-5, 5e-7, 0.1, 2, 0, 0, None, None, None) == -1  # flag
    assert lib.wolf_propagate_source(ctypes.byref(good), 16, 1e-5, 5e-7, 0.1, 0, 5, 0, None, None, None) == -1  # kind
    assert lib.wolf_propagate_source(ctypes.byref(good), 16, 1e-5, 5e-7, 0.1, 0, 0, 7, None, None, None) == -1  # dtype
    assert lib.wolf_propagate_source(None, 16, 1e-5, 5e-7, 0.1, 0, 0, 0, None, None, None) == -1
    assert b"null" in lib.wolf_last_error_message()
    bad = S(0, 3, 1.0, 1e-4, 1e-4, 1e-4, 2e-4, None, None, 0, 0)  # annulus r1 >= r0
    assert lib.wolf_propagate_source(ctypes.byref(bad), 16, 1e-5, 5e-7, 0.1, 0, 0, 0, None, None, None) == -1
    assert lib.wolf_propagate_source(ctypes.byref(good), 16, 1e-5, 5e-7, 0.1, 0, 0, 0, None, None, None) == -1  # w_out


def test_host_pointer_is_rejected(lib):
    buf = (ctypes.c_float * (2 * 16 ** 4))()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.wolf_propagate_fresnel(p, p, 16, 1e-5, 5e-7, 0.1, 0, 0, None, None) == -1


def test_product_path_does_not_use_the_oracle():
    """The product package neither imports nor names the oracle."""
    pkg = os.path.join(ROOT, "paper_2203_02734_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
