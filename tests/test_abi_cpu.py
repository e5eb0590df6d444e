"""The C-ABI library loads, exports every symbol its header declares, and its
host-side argument checks reject bad calls before touching a GPU."""
import ctypes
import math
import os
import re

import pytest

from paper_2603_27830_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgp4mi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgp4_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _native.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert {s[0] for s in _native.SIGNATURES} == set(names)


def test_version_strerror_and_sizes():
    L = _native.lib()
    assert L.sgp4_version() == 2
    for code in range(-7, 1):
        assert _native.strerror(code)
    assert L.sgp4_consts_bytes(-1) == 0
    assert L.sgp4_consts_bytes(1000) > L.sgp4_consts_bytes(10) > 0


def test_argument_errors_need_no_gpu():
    L = _native.lib()
    E = {v: k for k, v in _native.ERRORS.items()}
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    # negative sizes
    assert L.sgp4_propagate(fake, -1, fake, 10, 0, fake, fake, fake, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_propagate(fake, 10, fake, -1, 0, fake, fake, fake, None) == E["SGP4_E_SIZE"]
    # n * T overflow
    assert L.sgp4_propagate(fake, 2**31 - 1, fake, 2**40, 0, fake, fake, fake, None) == E["SGP4_E_SIZE"]
    # precision
    assert L.sgp4_propagate(fake, 10, fake, 10, 3, fake, fake, fake, None) == E["SGP4_E_PRECISION"]
    assert L.sgp4_vjp(10, fake, fake, fake, 10, 1, fake, None, fake, None) == E["SGP4_E_PRECISION"]
    assert L.sgp4_jacobian(10, fake, fake, fake, 10, 1, fake, None) == E["SGP4_E_PRECISION"]
    assert L.sgp4_jacobian(-1, fake, fake, fake, 10, 0, fake, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_jacobian(10, None, fake, fake, 10, 0, fake, None) == E["SGP4_E_ARG"]
    assert L.sgp4_jacobian(2**31 - 1, fake, fake, fake, 2**30, 0, fake, None) == E["SGP4_E_SIZE"]
    # the per-satellite list forms of the VJP and the Jacobian
    vr, jr = L.sgp4_vjp_ragged, L.sgp4_jacobian_ragged
    assert vr(10, fake, fake, fake, fake, 100, 1, fake, None, fake, None) == E["SGP4_E_PRECISION"]
    assert vr(-1, fake, fake, fake, fake, 100, 0, fake, None, fake, None) == E["SGP4_E_SIZE"]
    assert vr(10, fake, fake, fake, fake, -1, 0, fake, None, fake, None) == E["SGP4_E_SIZE"]
    assert vr(10, fake, fake, None, fake, 100, 0, fake, None, fake, None) == E["SGP4_E_ARG"]
    assert vr(10, fake, fake, fake, fake, 100, 0, None, None, fake, None) == E["SGP4_E_ARG"]
    assert vr(0, None, None, None, None, 0, 0, None, None, None, None) == 0
    assert jr(10, fake, fake, fake, fake, 100, 1, fake, None) == E["SGP4_E_PRECISION"]
    assert jr(10, fake, fake, fake, fake, 2**60, 0, fake, None) == E["SGP4_E_SIZE"]
    assert jr(10, fake, fake, fake, None, 100, 0, fake, None) == E["SGP4_E_ARG"]
    assert jr(10, fake, fake, fake, fake, 0, 0, None, None) == 0
    # null pointers
    assert L.sgp4_propagate(None, 10, fake, 10, 0, fake, fake, fake, None) == E["SGP4_E_ARG"]
    assert L.sgp4_propagate(fake, 10, fake, 10, 0, fake, None, fake, None) == E["SGP4_E_ARG"]
    # block size
    assert L.sgp4_propagate_ex(fake, 10, fake, 10, 0, fake, fake, fake, 96, None) == E["SGP4_E_ARG"]
    # one-wavefront-per-tile mapping: scalar constants only, not persistent, unknown bits rejected
    assert L.sgp4_propagate_ex(fake, 10, fake, 10, 0, fake, fake, fake, 256 | 0x40000, None) == E["SGP4_E_ARG"]
    assert L.sgp4_propagate_ex(fake, 10, fake, 10, 0, fake, fake, fake, 256 | 0x10000 | 0x40000 | 0x20000 | (4 << 20),
                               None) == E["SGP4_E_ARG"]
    assert L.sgp4_propagate_ex(fake, 10, fake, 10, 0, fake, fake, fake, 256 | 0x8000, None) == E["SGP4_E_ARG"]
    # more 64-time tiles than 32-bit tile indices address
    assert L.sgp4_propagate_ex(fake, 2**31 - 1, fake, 64 * 4, 0, fake, fake, fake, 256 | 0x10000 | 0x40000,
                               None) == E["SGP4_E_SIZE"]
    # empty batches are valid no-ops
    assert L.sgp4_propagate(fake, 0, fake, 10, 0, fake, fake, fake, None) == 0
    assert L.sgp4_propagate(fake, 10, fake, 0, 0, fake, fake, fake, None) == 0
    assert L.sgp4_propagate_ragged(fake, 10, fake, fake, 0, 0, fake, fake, fake, None, None) == 0
    # points with no satellite
    assert L.sgp4_propagate_ragged(fake, 0, fake, fake, 5, 0, fake, fake, fake, None, None) == E["SGP4_E_OFFSETS"]
    # gravity: J3 without J2, non-positive mu
    g = (ctypes.c_double * 5)(398600.8, 6378.135, 0.0, -2.5e-6, 0.0)
    assert L.sgp4_init(g, 10, fake, fake, None, None) == E["SGP4_E_GRAVITY"]
    g = (ctypes.c_double * 5)(0.0, 6378.135, 1e-3, 0.0, 0.0)
    assert L.sgp4_init(g, 10, fake, fake, None, None) == E["SGP4_E_GRAVITY"]
    assert L.sgp4_init(None, -5, fake, fake, None, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_init(None, 5, None, fake, None, None) == E["SGP4_E_ARG"]
    # plan creation
    out = ctypes.c_void_p()
    assert L.sgp4_plan_create(None, fake, 10, fake, fake, 10, 0, fake, fake, fake, 0, None) == E["SGP4_E_ARG"]
    assert L.sgp4_plan_create(ctypes.byref(out), fake, 10, fake, fake, 10, 7, fake, fake, fake, 0,
                              None) == E["SGP4_E_PRECISION"]
    # unknown ragged mapping, bad workgroup size
    assert L.sgp4_plan_create_config(ctypes.byref(out), fake, 10, fake, fake, 10, 0, fake, fake, fake, 2, 256, 0, 0,
                                     None) == E["SGP4_E_ARG"]
    assert L.sgp4_plan_create_config(ctypes.byref(out), fake, 10, fake, fake, 10, 0, fake, fake, fake, 1, 96, 0, 0,
                                     None) == E["SGP4_E_ARG"]
    assert L.sgp4_plan_launch(None, None) == E["SGP4_E_ARG"]
    L.sgp4_plan_destroy(None)


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2603_27830_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_elements_to_states_and_flat_config_reject_bad_arguments():
    """sgp4_propagate_elements and the flat dense flag: errors before any launch."""
    L = _native.lib()
    E = {v: k for k, v in _native.ERRORS.items()}
    fake = ctypes.c_void_p(0x1000)
    pe = L.sgp4_propagate_elements
    assert pe(None, 10, fake, fake, 5, 3, fake, fake, fake, None, None, 0, None) == E["SGP4_E_PRECISION"]
    assert pe(None, -1, fake, fake, 5, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_SIZE"]
    assert pe(None, 10, fake, fake, -5, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_SIZE"]
    assert pe(None, 2**40, fake, fake, 2**30, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_SIZE"]
    assert pe(None, 10, None, fake, 5, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_ARG"]
    assert pe(None, 10, fake, fake, 5, 0, None, fake, fake, None, None, 0, None) == E["SGP4_E_ARG"]
    small = L.sgp4_consts_bytes(10) - 1
    assert pe(None, 10, fake, fake, 5, 0, fake, fake, fake, None, fake, small, None) == E["SGP4_E_WORKSPACE"]
    # a fused launch covers ceil(T / 16) <= 65535 workgroups in y; beyond that a workspace is required
    assert pe(None, 10, fake, fake, 65535 * 16 + 1, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_WORKSPACE"]
    bad = (ctypes.c_double * 5)(398600.8, -1.0, 0.0, 0.0, 0.0)
    assert pe(bad, 10, fake, fake, 5, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_GRAVITY"]
    # empty batches launch nothing and succeed, even with null buffers
    assert pe(None, 0, None, None, 5, 0, None, None, None, None, None, 0, None) == 0
    assert pe(None, 10, None, None, 0, 0, None, None, None, None, None, 0, None) == 0
    assert L.sgp4_strerror(E["SGP4_E_WORKSPACE"]).decode().startswith("workspace")
    px = L.sgp4_propagate_ex
    FLAT = 0x80000
    for cfg in (256 | FLAT | 0x10000, 256 | FLAT | 0x40000 | 0x10000, 256 | FLAT | 0x20000 | (2 << 20), 96 | FLAT):
        assert px(fake, 10, fake, 10, 0, fake, fake, fake, cfg, None) == E["SGP4_E_ARG"], hex(cfg)
    assert px(fake, 2**31 - 1, fake, 2**9, 0, fake, fake, fake, 64 | FLAT, None) == E["SGP4_E_SIZE"]


def test_launch_extent_limits_are_checked_on_the_host():
    """A dispatch spans fewer than 2^32 lanes per grid dimension: calls whose
    grid would exceed it return SGP4_E_SIZE before any launch."""
    L = _native.lib()
    E = {v: k for k, v in _native.ERRORS.items()}
    fake = ctypes.c_void_p(0x1000)
    SCALAR, TILES, FLAT = 0x10000, 0x40000, 0x80000
    px = L.sgp4_propagate_ex
    # one 256-lane workgroup per satellite: n < 2^24
    assert L.sgp4_vjp(2**24, fake, fake, fake, 1, 0, fake, None, fake, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_jacobian(2**24, fake, fake, fake, 1, 0, fake, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_vjp_ragged(2**24, fake, fake, fake, fake, 1, 0, fake, None, fake, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_jacobian_ragged(2**24, fake, fake, fake, fake, 1, 0, fake, None) == E["SGP4_E_SIZE"]
    # 2^26 tiles of 64 lanes = 2^32 lanes
    assert px(fake, 2**26, fake, 64, 0, fake, fake, fake, 256 | SCALAR | TILES, None) == E["SGP4_E_SIZE"]
    # satellite-by-time grid: n workgroups of 256 lanes
    assert px(fake, 2**24, fake, 10, 0, fake, fake, fake, 256 | SCALAR, None) == E["SGP4_E_SIZE"]
    # flat grid: 2^32 points in 256-lane workgroups
    assert px(fake, 2**22, fake, 2**10, 0, fake, fake, fake, 256 | FLAT, None) == E["SGP4_E_SIZE"]
    # fused grid: ceil(n / 64) workgroups of 64 x 16 lanes
    pe = L.sgp4_propagate_elements
    assert pe(None, 2**28, fake, fake, 16, 0, fake, fake, fake, None, None, 0, None) == E["SGP4_E_SIZE"]


def test_double_sincos_table_is_correctly_rounded():
    """The device table of sin and cos at j pi / 64 (j = -64 .. 64) holds the
    doubles nearest the exact values (checked in 50-digit arithmetic)."""
    import mpmath
    src = open(os.path.join(os.path.dirname(_native.__file__), "csrc", "sgp4mi_math.h")).read()
    body = src[src.index("kSinCos64[258] = {"):]
    body = body[body.index("{") + 1:body.index("};")]
    vals = [float(x) for x in body.replace("\n", " ").split(",") if x.strip()]
    assert len(vals) == 258
    mpmath.mp.dps = 50
    for j in range(-64, 65):
        a = mpmath.mpf(j) * mpmath.pi / 64
        s_exact, c_exact = mpmath.sin(a), mpmath.cos(a)
        s_tab, c_tab = vals[2 * (j + 64)], vals[2 * (j + 64) + 1]
        assert abs(mpmath.mpf(s_tab) - s_exact) <= abs(mpmath.mpf(math.ulp(s_tab))) / 2 + mpmath.mpf(10) ** -45, j
        assert abs(mpmath.mpf(c_tab) - c_exact) <= abs(mpmath.mpf(math.ulp(c_tab))) / 2 + mpmath.mpf(10) ** -45, j
