"""The C ABI: the library loads on the CPU, exports every declared symbol, and its host-only
arithmetic and argument checks behave as documented (no device work here)."""
import ctypes
import json
import os
import subprocess

import pytest

from paper_2305_02678_amd import nam

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


@pytest.fixture(scope="module")
def L():
    return nam.lib(build_if_missing=True)


def test_every_declared_function_is_exported(L):
    names = nam.header_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", nam.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(L, n)


def test_version_and_error_string(L):
    assert L.nam_version() >= 100
    assert isinstance(L.nam_last_error(), bytes)


def test_pyramid_bytes_reproduces_the_papers_tile_size(L):
    g = json.load(open(GOLDEN))["latent_tile_bytes"]
    assert nam.pyramid_bytes(g["width"], g["height"], g["channels"], g["levels"], nam.F16) == g["value"]
    # the full chain adds a third: sum 4^-l -> 4/3 (minus the rounding of the last levels)
    full = nam.pyramid_bytes(4096, 4096, 8, 13, nam.F16)
    assert full == sum((4096 >> l) ** 2 for l in range(13)) * 8 * 2
    assert nam.pyramid_bytes(2048, 2048, 16, 12, nam.F32) == sum((2048 >> l) ** 2 for l in range(12)) * 64


def test_texels_per_update_ratio(L):
    g = json.load(open(GOLDEN))["gradient_updates_ratio"]
    a = nam.pyramid_bytes(g["fine"], g["fine"], 8, 1, nam.F32)
    b = nam.pyramid_bytes(g["coarse"], g["coarse"], 8, 1, nam.F32)
    assert a // b == g["value"]


@pytest.mark.parametrize("w,h,c,levels,status", [
    (48, 64, 8, 1, nam.NAM_E_SHAPE),        # not a power of two
    (64, 64, 8, 8, nam.NAM_E_SHAPE),        # more levels than the chain has
    (64, 64, 8, 0, nam.NAM_E_SHAPE),
    (64, 64, 12, 1, nam.NAM_E_UNSUPPORTED),  # channels
    (65536, 64, 8, 1, nam.NAM_E_UNSUPPORTED),
])
def test_pyramid_checks(L, w, h, c, levels, status):
    with pytest.raises(nam.NamError) as e:
        nam.pyramid_bytes(w, h, c, levels, nam.F16)
    assert e.value.status == status


def test_null_handles_are_rejected_without_a_device(L):
    assert L.nam_destroy(None) == nam.NAM_E_INVALID_ARG
    assert L.nam_material_free(None) == nam.NAM_E_INVALID_ARG
    assert L.nam_decode(None, None, 0, None, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_fetch(None, None, 0, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert b"NULL" in L.nam_last_error()
    assert L.nam_pyramid_bytes(None, 0, None) == nam.NAM_E_INVALID_ARG
    h = ctypes.c_void_p()
    assert L.nam_create(0, None) == nam.NAM_E_INVALID_ARG


def test_null_arguments_of_the_material_file_sampler_and_frame_calls(L):
    """Every entry point added for learned frames, material files and importance sampling checks
    its handles before touching a device."""
    assert L.nam_material_load_framed(None, None, None, None, None, 2, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_material_save(None, b"x.nam") == nam.NAM_E_INVALID_ARG
    assert L.nam_material_load_file(None, b"x.nam", None) == nam.NAM_E_INVALID_ARG
    assert L.nam_material_set_sampler(None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_sampler_params(None, None, 0, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_sampler_pdf(None, None, 0, None, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_sampler_sample(None, None, 0, None, None, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_proxy_pdf(None, 0, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_proxy_sample(None, 0, None, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
    assert L.nam_decode_stochastic(None, None, 0, None, None, None, None, None, None, None) == nam.NAM_E_INVALID_ARG
