"""Host-side checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching the GPU."""
import ctypes as ct
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nat():
    import paper_2201_11924_amd.native as n
    return n


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(simsense_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_exports_every_declared_symbol(nat):
    names = declared_symbols()
    assert {"simsense_create", "simsense_compute", "simsense_destroy"} <= names
    for n in names:
        assert hasattr(nat.lib(), n), n


def base_params():
    return dict(width=320, height=240, max_disp=64, census_w=7, census_h=9, census_mode=0, p1=7, p2=86,
                uniqueness_pct=10, lr_max_diff=1, num_paths=8, median=3, subpixel=1, focal_px=400.0,
                baseline_m=0.055)


BAD = [dict(width=0), dict(height=-3), dict(width=9000), dict(max_disp=0), dict(max_disp=257),
       dict(census_w=6), dict(census_h=4), dict(census_mode=2), dict(census_w=11, census_h=13, census_mode=1),
       dict(p1=-1), dict(p1=10, p2=9), dict(p2=240), dict(uniqueness_pct=100), dict(num_paths=3),
       dict(num_paths=16), dict(median=5), dict(subpixel=2), dict(focal_px=float("nan"))]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_params_rejected_on_host(nat, bad):
    p = nat.Params.from_dict(dict(base_params(), **bad))
    assert nat.lib().simsense_scratch_bytes(ct.byref(p)) == -1
    h = ct.c_void_p()
    assert nat.lib().simsense_create(ct.byref(p), ct.byref(h)) == -1
    assert h.value is None


def test_abi_size_and_null_checks(nat):
    p = nat.Params.from_dict(base_params())
    assert nat.lib().simsense_scratch_bytes(ct.byref(p)) > 0
    p.struct_size = 12
    assert nat.lib().simsense_scratch_bytes(ct.byref(p)) == -6
    assert nat.lib().simsense_create(None, None) == -2
    assert nat.lib().simsense_compute(None, None, None, 0, None, None, None, None) == -2
    assert nat.lib().simsense_destroy(None) == 0
    assert nat.lib().simsense_ir_noise(None, None, None, None, 0, None) == 0
    assert nat.lib().simsense_ir_noise(None, None, None, None, -1, None) == -1
    assert nat.lib().simsense_ir_noise(None, None, None, None, 5, None) == -2
    good = nat.Params.from_dict(base_params())
    assert nat.lib().simsense_census(ct.byref(good), None, 320, None, None) == -2
    assert nat.lib().simsense_strerror(-4) == b"HIP runtime or kernel launch error"


def test_scratch_bytes_scale(nat):
    # 8 path buffers of W*H*Dpad bytes dominate the handle's scratch
    p = dict(base_params(), width=1280, height=720, max_disp=128)
    b = nat.scratch_bytes(p)
    assert 8 * 1280 * 720 * 128 <= b < 8 * 1280 * 720 * 128 + 40 * 1280 * 720


def test_noalloc_host_checks(nat):
    # argument errors and the scratch limit are reported before any device work
    lib = nat.lib()
    big = nat.Params.from_dict(dict(base_params(), width=1280, height=720, max_disp=128))
    fake = ct.c_void_p(256)
    assert lib.simsense_compute_noalloc(ct.byref(big), fake, fake, 1280, fake, None, None, None) == nat.ERR_TOO_LARGE
    assert lib.simsense_compute_noalloc(ct.byref(big), None, None, 1280, None, None, None, None) == -2
    bad = nat.Params.from_dict(dict(base_params(), num_paths=3))
    assert lib.simsense_compute_noalloc(ct.byref(bad), fake, fake, 320, fake, None, None, None) == -1
    small = nat.Params.from_dict(base_params())
    assert lib.simsense_compute_noalloc(ct.byref(small), fake, fake, 100, fake, None, None, None) == -1
    assert nat.scratch_bytes(base_params()) <= nat.NOALLOC_SCRATCH_BYTES
