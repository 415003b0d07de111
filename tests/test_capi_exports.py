"""CPU checks of the C ABI: every function declared in include/sfft.h is
exported by the built library, and host-side parameter logic (no GPU call)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "sfft.h")
LIB = os.path.join(ROOT, "paper_2109_09334_amd", "libsfft.so")


def declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfft_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def exported():
    if not os.path.exists(LIB):
        import paper_2109_09334_amd.build as b
        b.build()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


def test_header_declares_the_boundary():
    names = declared()
    for must in ("sfft_build_system", "sfft_solve", "sfft_subtract", "sfft_submit", "sfft_poll",
                 "sfft_create", "sfft_destroy", "sfft_strerror"):
        assert must in names


def test_every_declared_symbol_is_exported(exported):
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_host_logic():
    import torch  # noqa: F401  (shares the HIP runtime with the library)
    import paper_2109_09334_amd as sf
    L = sf.lib()
    P = sf.Params
    assert P(4096, 4096, 7, 7, 2, 2).num_unknowns == 1356
    assert P(1024, 1024, 5, 5, 2, 2).num_unknowns == 732
    assert P(256, 256, 5, 5, 0, 0).num_unknowns == 122
    assert P(512, 512, 5, 5, 1, 1).num_unknowns == 366
    assert P(64, 64, 3, 3, 2, 2, const_phot=1).num_unknowns == 6 * 49 - 5 + 6
    ok = sf.Context.check
    assert ok(P(4096, 4096, 7, 7, 2, 2)) == sf.OK
    assert ok(P(6144, 6144, 7, 7, 2, 2)) == sf.OK
    assert ok(P(2048, 4096, 5, 5, 1, 1)) == sf.OK
    # lengths other than 2^a 3^b run as Bluestein lines of a power of two <= 8192
    assert ok(P(100, 128, 3, 3, 1, 1)) == sf.OK                # 100 = 4 * 25
    assert ok(P(2046, 4094, 7, 7, 2, 2)) == sf.OK              # DECam CCD: 2 3 11 31, 2 23 89
    assert ok(P(4096, 4098, 7, 7, 2, 2)) == sf.E_UNSUPPORTED   # its Bluestein length 16384
    assert ok(P(101, 128, 3, 3, 1, 1)) == sf.E_UNSUPPORTED     # odd
    assert ok(P(8192, 8192, 3, 3, 1, 1)) == sf.OK
    assert ok(P(64, 64, -1, 3, 1, 1)) == sf.E_INVAL
    assert ok(P(64, 64, 3, 3, 1, 1, precision=7)) == sf.E_INVAL
    assert ok(P(16, 16, 8, 8, 0, 0)) == sf.E_INVAL             # 2w+1 > n
    assert ok(P(64, 64, 3, 3, 5, 1)) == sf.E_UNSUPPORTED       # DK > 4
    # the mixed form: FP32 images, DK <= 3, sides of 48 pixels or more
    M = dict(precision=sf.MIXED)
    assert ok(P(64, 64, 3, 3, 3, 1, **M)) == sf.OK
    assert ok(P(64, 64, 3, 3, 4, 1, **M)) == sf.E_UNSUPPORTED
    assert ok(P(64, 64, 3, 3, 1, 1, dtype=sf.F64, **M)) == sf.E_UNSUPPORTED
    assert ok(P(2046, 48, 9, 2, 1, 1, **M)) == sf.OK
    assert ok(P(2046, 34, 9, 2, 1, 1, **M)) == sf.E_UNSUPPORTED
    assert ok(P(32, 8192, 3, 2, 1, 1, **M)) == sf.E_UNSUPPORTED
    assert ok(P(32, 8192, 3, 2, 1, 1, precision=sf.FP64)) == sf.OK
    assert sf.Context.workspace_bytes(P(4096, 4096, 7, 7, 2, 2)) > 0
    assert L.sfft_strerror(sf.E_NOT_SPD).decode().startswith("normal matrix")
