"""The allocation-free screening entry point (sgp4_screen_noalloc) against the
allocating one (sgp4_screen) on the same positions: identical event sets and
distances, on two calls in a row, the second with a smaller batch (the
library's fixed per-GPU workspace keeps the first call's contents, which the
second must not see).  The first batch takes the device-memory bucket path
(n > 12,288), the second the on-chip path."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2603_27830_amd as sg
from paper_2603_27830_amd import _native
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def events(pairs, dist):
    p = pairs.cpu().numpy().astype(np.int64)
    d = dist.cpu().numpy()
    order = np.lexsort((p[:, 2], p[:, 1], p[:, 0]))
    return p[order], d[order]


def positions(n, T, seed, prec):
    el = synth.shell_elements(n, seed)
    t = torch.from_numpy(np.linspace(0.0, 1440.0, T)).to(DEV)
    rec = sg.init(torch.from_numpy(el).to(DEV))
    r, _, err = sg.propagate(rec, t, prec)
    return r.contiguous(), err.contiguous()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_screen_matches_allocating_screen_twice(prec):
    cap = 1 << 21
    pairs = torch.empty((cap, 3), dtype=torch.int32, device=DEV)
    dist = torch.empty(cap, dtype=torch.float64, device=DEV)
    count = torch.empty(1, dtype=torch.int64, device=DEV)
    for n, T, D, seed in ((14000, 300, 40.0, 11), (3000, 120, 60.0, 12)):
        say(f"[gpu] screen_noalloc {prec} n={n} T={T} D={D}")
        L = _native.lib()
        assert L.sgp4_screen_workspace_bytes(n, T) <= sg.NOALLOC_SCREEN_BYTES
        r, err = positions(n, T, seed, prec)
        p0, d0, tot0 = sg.screen(r, D, err, capacity=cap)
        e0 = events(p0, d0)
        p1, d1, tot1 = sg.screen_noalloc(r, D, err, pairs=pairs, dist=dist, count=count)
        torch.cuda.synchronize()
        e1 = events(p1, d1)
        assert tot0 == tot1 and tot0 > 100, (tot0, tot1)
        assert np.array_equal(e0[0], e1[0])
        assert np.array_equal(e0[1], e1[1])


def test_noalloc_screen_rejects_batches_beyond_its_workspace():
    L = _native.lib()
    E = {v: k for k, v in _native.ERRORS.items()}
    fake = ctypes.c_void_p(0x1000)
    n, T = 9341, 1000  # about 122 MB of workspace, above the 64 MiB array
    assert L.sgp4_screen_workspace_bytes(n, T) > sg.NOALLOC_SCREEN_BYTES
    assert L.sgp4_screen_noalloc(fake, 0, None, n, T, 10.0, 16, fake, fake, fake, None) == E["SGP4_E_SIZE"]
    assert L.sgp4_screen_noalloc(fake, 0, None, 100, 100, -1.0, 16, fake, fake, fake, None) == E["SGP4_E_ARG"]
