"""GPU parity of conjunction screening (sgp4_screen) against the brute-force
oracle: the event sets (i, j, k) identical and distances equal to rounding
(both sides compute d^2 in double from the same stored positions with the same
operation order; the decision d^2 < D^2 is taken in the same precision).

Inputs are synthetic: points on LEO-like spherical shells with planted close
pairs, cubic lattices with closed-form counts, and the oracle's own
propagation of the 9,341-satellite catalogue (never a GPU output)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_27830_amd as sg
import synth
from oracle import screen as osc
from test_gpu_parity import DEV, NTHREADS, dev, say

pytestmark = pytest.mark.gpu


def shell_points(n, T, seed, planted=40, radius=6900.0, thick=40.0):
    """Random points on a shell at T times, plus `planted` pairs placed 0-30 km apart."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, n, T))
    v /= np.linalg.norm(v, axis=0)
    r = v * (radius + rng.uniform(-thick / 2, thick / 2, (n, T)))
    for _ in range(planted):
        i, j = rng.choice(n, 2, replace=False)
        k = rng.integers(0, T)
        r[:, j, k] = r[:, i, k] + rng.normal(size=3) * rng.uniform(0.0, 17.0)
    return r


def gpu_events(r, D, err=None, cap=1 << 20, mode=0):
    pairs, dist, total = sg.screen(dev(r), D, None if err is None else dev(err), capacity=cap, mode=mode)
    torch.cuda.synchronize()
    p = pairs.cpu().numpy().astype(np.int64)
    d = dist.cpu().numpy()
    order = np.lexsort((p[:, 1], p[:, 0], p[:, 2]))
    return p[order], d[order], total


def check(r, D, err=None, times=None, mode=0):
    ev, d, total = gpu_events(r, D, err, mode=mode)
    eo, do = osc.screen(r, D, err=err, times=None if times is None else sorted(times))
    if times is not None:
        keep = np.isin(ev[:, 2], np.asarray(list(times)))
        ev, d = ev[keep], d[keep]
    else:
        assert total == len(eo)
    assert np.array_equal(ev, eo), (len(ev), len(eo))
    assert np.allclose(d, do, rtol=1e-15, atol=0.0)
    return len(eo)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,T", [(2, 3), (63, 5), (3000, 16), (1025, 9)])
def test_shell_points_match_oracle(n, T, dtype, mode):
    """Both paths: on-chip buckets (mode 1) and device-memory buckets (mode 2)."""
    r = shell_points(n, T, seed=n + T).astype(dtype)
    say(f"[gpu] screen shell n={n} T={T} {np.dtype(dtype).name} mode={mode}")
    m = check(r, 25.0, mode=mode)
    say(f"  events {m}")


@pytest.mark.parametrize("mode", [1, 2])
def test_invalid_points_excluded(mode):
    n, T = 2000, 6
    r = shell_points(n, T, seed=9, planted=200)
    err = np.zeros((n, T), np.uint8)
    rng = np.random.default_rng(1)
    err[rng.random((n, T)) < 0.1] = 4
    err[rng.random((n, T)) < 0.05] = 6          # decayed points still count
    r[:, rng.random(n) < 0.03, :] = np.nan      # NaN states without a code
    say(f"[gpu] screen with codes and NaN states mode={mode}")
    m = check(r, 25.0, err=err, mode=mode)
    assert m > 100


@pytest.mark.parametrize("m", [3, 8])
def test_lattice_closed_form_counts(m):
    import itertools
    g = np.array(list(itertools.product(range(m), repeat=3)), dtype=np.float64) * 4.0 + [6500.0, 100.0, -50.0]
    r = np.repeat(g.T[:, :, None], 2, axis=2).copy()
    nn, face, body = 3 * m * m * (m - 1), 6 * m * (m - 1) ** 2, 4 * (m - 1) ** 3
    say(f"[gpu] screen lattice m={m}")
    for D, want in ((4.04, nn), (6.0, nn + face), (7.2, nn + face + body)):
        for mode in (1, 2):
            ev, _, total = gpu_events(r, D, mode=mode)
            assert total == 2 * want and len(ev) == 2 * want
            check(r, D, mode=mode)


def test_capacity_smaller_than_the_events():
    r = shell_points(1500, 8, seed=4, planted=300)
    eo, _ = osc.screen(r, 25.0)
    pairs, dist, total = sg.screen(dev(r), 25.0, capacity=50)
    torch.cuda.synchronize()
    assert total == len(eo) and len(pairs) == 50
    got = set(map(tuple, pairs.cpu().numpy().astype(np.int64).tolist()))
    assert got <= set(map(tuple, eo.tolist()))


def test_maximum_satellites_and_empty():
    r = shell_points(12288, 2, seed=5, planted=100)
    say("[gpu] screen n=12288 (maximum)")
    check(r, 20.0)
    for shape in ((3, 0, 4), (3, 1, 4), (3, 5, 0)):
        _, _, total = sg.screen(torch.zeros(shape, dtype=torch.float64, device=DEV), 10.0)
        assert total == 0


def test_catalogue_propagated_by_the_oracle_sampled_times():
    """9,341 satellites x 1,000 times as the benchmark screens them (positions
    from the oracle's FP64 propagation, D = 10 km), FP64 and float32 storage;
    10 sampled times compared with the oracle event by event."""
    cat = synth.config1()
    say("[gpu] screen 9341 x 1000 (oracle positions), sampled times")
    r, _, e = oracle.propagate(cat.elem, cat.t, nthreads=NTHREADS)
    r = r.reshape(3, cat.n, cat.T)
    e = e.reshape(cat.n, cat.T)
    times = list(np.random.default_rng(8).choice(cat.T, 10, replace=False))
    for dtype in (np.float64, np.float32):
        m = check(r.astype(dtype), 10.0, err=e, times=times)
        total = gpu_events(r.astype(dtype), 10.0, err=e)[2]
        say(f"  {np.dtype(dtype).name}: {m} events at the sampled times, {total} over all 1,000")
        assert m > 0 and total > m


def test_beyond_on_chip_size_matches_oracle():
    """20,000 satellites (over the on-chip limit, so the automatic choice takes
    the device-memory path), float32 storage, every event against the oracle."""
    r = shell_points(20000, 3, seed=77, planted=200).astype(np.float32)
    say("[gpu] screen n=20000 T=3 (device-memory buckets)")
    m = check(r, 15.0)
    assert m > 200


def test_mega_constellation_snapshot_sound_and_complete_on_a_subset():
    """100,000 satellites at 2 times: every reported event is a true event
    (distance recomputed from the positions), and on the first 15,000
    satellites the events are exactly the oracle's."""
    n, D = 100_000, 8.0
    r = shell_points(n, 2, seed=99, planted=500)
    say("[gpu] screen n=100000 T=2")
    ev, d, total = gpu_events(r, D)
    assert total == len(ev) and total > 500
    i, j, k = ev[:, 0], ev[:, 1], ev[:, 2]
    dd = np.sqrt(((r[:, j, k] - r[:, i, k]) ** 2).sum(axis=0))
    assert np.all(i < j) and np.all(dd < D) and np.allclose(dd, d, rtol=1e-12)
    sub = 15000
    eo, _ = osc.screen(r[:, :sub, :], D)
    mine = ev[(i < sub) & (j < sub)]
    assert np.array_equal(mine, eo)


def test_device_memory_path_many_times():
    """12,000 satellites x 1,000 times (the on-chip path's largest n, and a
    device-memory layout of 1,000 time rows): the device-memory path's events
    equal the on-chip path's over all times, and the oracle's at sampled
    times."""
    n, T, D = 12_000, 1000, 12.0
    r = shell_points(n, T, seed=123, planted=600).astype(np.float32)
    say(f"[gpu] screen n={n} T={T}: device-memory path against the on-chip path")
    ev2, d2, tot2 = gpu_events(r, D, mode=2)
    ev1, d1, tot1 = gpu_events(r, D, mode=1)
    say(f"  events {tot2} (device memory), {tot1} (on chip)")
    assert tot1 == tot2 == len(ev1) and tot1 > 600
    assert np.array_equal(ev1, ev2) and np.array_equal(d1, d2)
    times = [0, 1, 429, 430, 431, 859, 860, 861, 999]
    m = check(r, D, times=set(times), mode=2)
    assert m > 0
