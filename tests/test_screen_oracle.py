"""The conjunction-screening oracle pinned to closed forms: event counts on a
cubic lattice (nearest neighbours, face and body diagonals), the strict
threshold, permutation invariance and the exclusion of invalid points.
Also the C ABI's argument checks for sgp4_screen (no GPU needed)."""
import ctypes
import itertools
import math

import numpy as np
import pytest

from oracle import screen as osc


def lattice(m, s=1.0, origin=(7000.0, -300.0, 40.0)):
    g = np.array(list(itertools.product(range(m), repeat=3)), dtype=np.float64) * s
    return (g + np.array(origin)).T.copy()  # [3, m^3]


@pytest.mark.parametrize("m", [2, 3, 5])
def test_lattice_counts(m):
    s = 3.0
    p = lattice(m, s)[:, :, None]
    nn = 3 * m * m * (m - 1)                 # axis neighbours at distance s
    face = 6 * m * (m - 1) ** 2              # face diagonals at s*sqrt(2)
    body = 4 * (m - 1) ** 3                  # body diagonals at s*sqrt(3)
    assert len(osc.screen(p, 1.01 * s)[0]) == nn
    assert len(osc.screen(p, 1.5 * s)[0]) == nn + face
    assert len(osc.screen(p, 1.8 * s)[0]) == nn + face + body
    assert len(osc.screen(p, 0.99 * s)[0]) == 0
    ev, d = osc.screen(p, 1.01 * s)
    assert np.all(np.abs(d - s) <= 1e-12) and np.all(ev[:, 0] < ev[:, 1])


def test_threshold_is_strict():
    p = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 2.0]])[:, :, None]  # d(0,1) = 1 exactly
    ev, d = osc.screen(p, 1.0)
    assert len(ev) == 0
    ev, d = osc.screen(p, np.nextafter(1.0, 2.0))
    assert ev.tolist() == [[0, 1, 0]] and d.tolist() == [1.0]


def test_permutation_invariance_and_invalid_points():
    rng = np.random.default_rng(3)
    n, T = 400, 3
    p = rng.normal(0.0, 30.0, (3, n, T))
    ev, d = osc.screen(p, 8.0)
    perm = rng.permutation(n)
    ev2, d2 = osc.screen(p[:, perm, :], 8.0)   # satellite a of the permuted batch is satellite perm[a]
    mapped = np.stack([perm[ev2[:, 0]], perm[ev2[:, 1]], ev2[:, 2]], axis=1)
    mapped[:, :2] = np.sort(mapped[:, :2], axis=1)
    key = lambda e: sorted(map(tuple, e.tolist()))  # noqa: E731
    assert key(mapped) == key(ev) and len(ev) > 50
    err = np.zeros((n, T), np.uint8)
    err[::7] = 4
    p2 = p.copy()
    p2[:, 3::11, 1] = np.nan
    ev3, _ = osc.screen(p2, 8.0, err=err)
    bad = set(range(0, n, 7))
    for i, j, k in ev3.tolist():
        assert i not in bad and j not in bad
        if k == 1:
            assert i % 11 != 3 and j % 11 != 3
    keep = [e for e in ev.tolist() if e[0] not in bad and e[1] not in bad and not (e[2] == 1 and (e[0] % 11 == 3 or e[1] % 11 == 3))]
    assert sorted(map(tuple, keep)) == key(ev3)


def test_screen_argument_errors():
    from paper_2603_27830_amd import _native
    L = _native.lib()
    E = {v: k for k, v in _native.ERRORS.items()}
    fake = ctypes.c_void_p(0x1000)
    sc = L.sgp4_screen
    sx = L.sgp4_screen_ex
    assert sx(fake, 0, None, 12289, 10, 5.0, 10, fake, fake, fake, fake, 1 << 40, 1, None) == E["SGP4_E_SIZE"]
    assert sx(fake, 0, None, 100, 10, 5.0, 10, fake, fake, fake, fake, 1 << 40, 3, None) == E["SGP4_E_ARG"]
    assert sx(fake, 0, None, 2**31, 2**20, 5.0, 10, fake, fake, fake, fake, 1 << 62, 2, None) == E["SGP4_E_SIZE"]
    assert sc(fake, 0, None, -1, 10, 5.0, 10, fake, fake, fake, fake, 1 << 40, None) == E["SGP4_E_SIZE"]
    assert sc(fake, 0, None, 10, 10, 5.0, -1, fake, fake, fake, fake, 1 << 40, None) == E["SGP4_E_SIZE"]
    assert sc(fake, 5, None, 10, 10, 5.0, 10, fake, fake, fake, fake, 1 << 40, None) == E["SGP4_E_PRECISION"]
    for bad in (0.0, -1.0, math.inf, math.nan):
        assert sc(fake, 0, None, 10, 10, bad, 10, fake, fake, fake, fake, 1 << 40, None) == E["SGP4_E_ARG"]
    assert sc(fake, 0, None, 10, 10, 5.0, 10, fake, fake, None, fake, 1 << 40, None) == E["SGP4_E_ARG"]
    assert sc(fake, 0, None, 10, 10, 5.0, 10, None, fake, fake, fake, 1 << 40, None) == E["SGP4_E_ARG"]
    assert sc(None, 0, None, 10, 10, 5.0, 10, fake, fake, fake, fake, 1 << 40, None) == E["SGP4_E_ARG"]
    assert sc(fake, 0, None, 10, 10, 5.0, 10, fake, fake, fake, None, 0, None) == E["SGP4_E_WORKSPACE"]
    need = L.sgp4_screen_workspace_bytes(10, 10)
    assert need >= 12 * 10 * 10
    assert sc(fake, 0, None, 10, 10, 5.0, 10, fake, fake, fake, fake, need - 1, None) == E["SGP4_E_WORKSPACE"]
    assert L.sgp4_screen_workspace_bytes(-1, 10) == 0
