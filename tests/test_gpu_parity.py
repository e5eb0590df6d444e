"""GPU parity: the HIP path against the CPU oracle, element by element.

FP64: |dr| <= 1e-6 km and |dv| <= 1e-9 km/s, codes bit-exact, NaN where the
code says so.  FP32-mixed: <= 10 m and <= 1e-2 m/s out to 7 days, codes exact
except at threshold ties (a decision variable within the path's error bound of
its threshold, reported separately).  All inputs come from the seeded
generators; every expected value comes from the oracle.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2603_27830_amd as sg
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
NTHREADS = max(1, min(16, os.cpu_count() or 1))
RE = 6378.135


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(*ts):
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in ts]


def say(msg):
    print(msg, flush=True)


def gpu_dense(elem, t, prec="fp64", block=None, grav=None):
    rec = sg.init(dev(elem), grav)
    r, v, err = sg.propagate(rec, dev(t), prec, block=block)
    return host(r, v, err)


def check_fp64(r, v, err, ro, vo, eo, tol_r=1e-6, tol_v=1e-9):
    r = r.reshape(3, -1); v = v.reshape(3, -1); err = err.reshape(-1)
    ro = ro.reshape(3, -1); vo = vo.reshape(3, -1); eo = eo.reshape(-1)
    assert np.array_equal(err, eo), f"codes differ at {np.flatnonzero(err != eo)[:10]}"
    ok = (eo == 0) | (eo == 6)
    assert np.all(np.isnan(r[:, ~ok])) and np.all(np.isnan(v[:, ~ok]))
    if ok.any():
        dr = np.max(np.abs(r[:, ok] - ro[:, ok]))
        dv = np.max(np.abs(v[:, ok] - vo[:, ok]))
        assert dr <= tol_r and dv <= tol_v, (dr, dv)
        return dr, dv
    return 0.0, 0.0


# ------------------------------------------------------------------- FP64 --
SCALAR, PERSIST, TILES = 0x10000, 0x20000, 0x40000
CONFIGS = [64, 128, 256, 512, 256 | SCALAR, 512 | SCALAR, 256 | PERSIST | (4 << 20),
           512 | SCALAR | PERSIST | (8 << 20), 64 | SCALAR | PERSIST | (1 << 20),
           64 | SCALAR | TILES, 256 | SCALAR | TILES, 512 | SCALAR | TILES]


@pytest.mark.parametrize("cfg", CONFIGS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_smoke_grid_every_launch_config(cfg, prec):
    cat = synth.config0()
    say(f"[gpu] c0 64x100 {prec} config={cfg:#x}")
    r, v, err = gpu_dense(cat.elem, cat.t, prec, cfg)
    ro, vo, eo = oracle.propagate(cat.elem, cat.t)
    if prec == "fp64":
        check_fp64(r, v, err, ro, vo, eo)
    else:
        assert np.array_equal(err, eo)
        dr, dv = _errors(r.reshape(3, -1), v.reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
        assert dr.max() <= 0.010 and dv.max() <= 1e-5


def test_starlink_grid_fp64_full_size():
    """9,341 x 1,000 in the benchmark's launch configuration, every point."""
    cat = synth.config1()
    say("[gpu] c1 9341x1000 fp64 full grid")
    r, v, err = gpu_dense(cat.elem, cat.t, "fp64")
    ro, vo, eo = oracle.propagate(cat.elem, cat.t, nthreads=NTHREADS)
    dr, dv = check_fp64(r, v, err, ro, vo, eo)
    say(f"  max |dr| {dr:.3e} km, max |dv| {dv:.3e} km/s")


@pytest.mark.parametrize("n,T", [(1, 1), (1, 63), (3, 65), (130, 1), (17, 257), (5, 1025), (64, 7)])
def test_tail_shapes_fp64(n, T):
    elem = synth.shell_elements(n, 40 + n)
    t = np.sort(np.random.default_rng(T).uniform(-500.0, 9000.0, T))
    say(f"[gpu] tail shape n={n} T={T}")
    for block in (64, 256, 512 | SCALAR, 256 | PERSIST | (2 << 20)):
        r, v, err = gpu_dense(elem, t, "fp64", block)
        ro, vo, eo = oracle.propagate(elem, t)
        check_fp64(r, v, err, ro, vo, eo)


def crafted_elements():
    """Edge cases: invalid epoch eccentricity, non-positive mean motion,
    deep space, simplified drag, exact circular, the 1e-4 eccentricity gate,
    heavy drag (decay and eccentricity below -0.001), NaN drag term, and
    near-parabolic sets that make p_L negative."""
    ke = 60.0 / math.sqrt(RE ** 3 / 398600.8)
    cols = []

    def add(n0=0.065, e0=1e-3, inc=0.9, node=0.1, argp=0.2, mo=0.3, bstar=1e-4, epoch=0.0):
        cols.append([n0, e0, inc, node, argp, mo, bstar, epoch])

    add(e0=1.2); add(e0=-0.1); add(n0=-0.06); add(n0=0.0); add(n0=2 * math.pi / 300.0)
    add(n0=ke * ((RE + 200.0) / RE) ** -1.5, e0=1e-3)           # simplified drag (perigee < 220 km)
    add(n0=ke * ((RE + 120.0) / RE) ** -1.5, e0=1e-4)           # perigee < 156 km and < 98 km branches
    add(e0=0.0); add(e0=1e-4); add(e0=1.0001e-4); add(e0=9.999e-5)
    add(n0=ke * ((RE + 300.0) / RE) ** -1.5, e0=2e-4, bstar=0.05)
    add(n0=ke * ((RE + 400.0) / RE) ** -1.5, e0=3e-4, bstar=0.5)
    add(bstar=float("nan"))
    add(inc=math.pi)                                              # retrograde equatorial (1 + cos i guard)
    add(inc=0.0)
    add(n0=2 * math.pi / 1436.0, e0=2e-4, inc=0.01)                # resonant deep space (24 h)
    add(n0=2 * math.pi / 718.0, e0=0.7, inc=1.1)                   # resonant deep space (12 h, e >= 0.5)
    return np.array(cols, dtype=np.float64).T.copy()


def near_parabolic_elements(n=60):
    """Mean eccentricity 0.99-0.9999: outside the model's domain (its series
    in J2 diverge there), used only to reach a negative semi-latus rectum."""
    rng = np.random.default_rng(13)
    el = np.empty((8, n))
    el[0] = rng.uniform(0.03, 0.06, n)
    el[1] = rng.uniform(0.99, 0.9999, n)
    el[2] = rng.uniform(0.3, 2.8, n)
    el[3:6] = rng.uniform(0, 6.28, (3, n))
    el[6] = 0.0
    el[7] = 0.0
    return el


def conditioning(el, t, trials=6, rels=(1e-15, 1e-13, 1e-11)):
    """Oracle-only conditioning of each point: perturb the seven elements by
    +-rel (relative) and record which codes the oracle reaches and how far the
    state moves.  A decision that flips under a few-ulp perturbation (the
    smallest rel) is a threshold tie of the FP64 computation itself; the codes
    reached under all perturbations are the valid outcomes at such a tie."""
    ro, vo, eo = oracle.propagate(el, t)
    rng = np.random.default_rng(0)
    reach = [eo]
    stable = np.ones(eo.shape, bool)
    move = np.zeros(eo.shape)
    vmove = np.zeros(eo.shape)
    for rel in rels:
        for _ in range(trials):
            pert = el.copy()
            pert[:7] *= 1 + rel * rng.choice([-1.0, 1.0], size=(7, el.shape[1]))
            r2, v2, e2 = oracle.propagate(pert, t)
            reach.append(e2)
            if rel == rels[0]:
                stable &= e2 == eo
                move = np.maximum(move, np.nan_to_num(np.max(np.abs(r2 - ro), axis=0), nan=np.inf))
                vmove = np.maximum(vmove, np.nan_to_num(np.max(np.abs(v2 - vo), axis=0), nan=np.inf))
    return ro, vo, eo, np.stack(reach), stable, np.maximum(move, 1e3 * vmove)


def test_edge_cases_and_error_codes_fp64():
    """Crafted element sets: codes bit-exact wherever the FP64 decision is
    well conditioned; at ties the GPU's code must be one the oracle reaches
    under a 1e-15 relative perturbation.  States are compared (1e-6 km,
    1e-9 km/s) where the oracle's state moves by less than 1e-7 km and 1e-10
    km/s under that perturbation."""
    el = crafted_elements()
    t = np.linspace(-1440.0, 10080.0, 97)
    say(f"[gpu] crafted edge cases n={el.shape[1]} fp64")
    r, v, err = gpu_dense(el, t, "fp64")
    ro, vo, eo, codes, stable, move = conditioning(el, t)
    say(f"  threshold ties: {int((~stable).sum())} of {stable.size} points")
    assert (~stable).sum() <= 0.02 * stable.size
    assert np.array_equal(err[stable], eo[stable])
    tie_ok = np.any(codes == err[None], axis=0)
    say(f"  GPU codes outside the oracle's reachable set at ties: {int((~tie_ok).sum())}")
    # every GPU code at a tie is one the oracle reaches under the perturbations
    assert (~tie_ok).sum() == 0
    bad = (err != 0) & (err != 6)
    assert np.all(np.isnan(r[:, bad])) and np.all(np.isnan(v[:, bad]))
    well = stable & ((eo == 0) | (eo == 6)) & (move < 1e-7)
    assert well.sum() >= 500
    # the ordinary element sets among the crafted ones are all well conditioned
    assert np.all(well[[5, 6, 7, 9, 10, 15]] | ~((eo[[5, 6, 7, 9, 10, 15]] == 0) | (eo[[5, 6, 7, 9, 10, 15]] == 6)))
    assert np.max(np.abs(r[:, well] - ro[:, well])) <= 1e-6
    assert np.max(np.abs(v[:, well] - vo[:, well])) <= 1e-9
    assert {0, 1, 2, 6} <= set(np.unique(eo).tolist())


def test_negative_semilatus_rectum_code4():
    """Near-parabolic sets: where the oracle's p_L is negative by a margin far
    above rounding (p_L < -1e-3 a), the GPU must return code 4 with a NaN
    state; codes decided before p_L (1, 2, 7) must match; elsewhere these
    ill-conditioned sets need only valid codes (sets whose recovered period
    reaches 225 min are deep space, where 3 is possible)."""
    el = near_parabolic_elements()
    t = np.linspace(-1440.0, 10080.0, 97)
    say(f"[gpu] near-parabolic sets n={el.shape[1]}")
    r, v, err = gpu_dense(el, t, "fp64")
    sat = np.repeat(np.arange(el.shape[1]), t.shape[0])
    _, _, eo, d = oracle.propagate_points(el, sat, np.tile(t, el.shape[1]), detail=True)
    err = err.reshape(-1)
    robust4 = (eo == 4) & (d["pL"] < -1e-3 * d["a"])
    assert robust4.sum() >= 50
    assert np.all(err[robust4] == 4)
    early = np.isin(eo, [1, 2, 7])
    assert np.array_equal(err[early], eo[early])
    assert set(np.unique(err).tolist()) <= {0, 1, 2, 3, 4, 6, 7}
    bad = (err != 0) & (err != 6)
    assert np.all(np.isnan(r.reshape(3, -1)[:, bad]))


def test_two_body_gravity_fp64():
    el = synth.shell_elements(200, 77)
    el[6] = 0.0
    grav = (398600.8, 6378.135, 0.0, 0.0, 0.0)
    t = np.linspace(0.0, 2880.0, 50)
    say("[gpu] two-body gravity fp64")
    r, v, err = gpu_dense(el, t, "fp64", grav=grav)
    ro, vo, eo = oracle.propagate(el, t, grav)
    check_fp64(r, v, err, ro, vo, eo)


def test_maximum_sizes_64bit_offsets_and_time_loop():
    """Component arrays above 4 GiB (64-bit store offsets: 40,000 x 27,500 =
    1.1e9 points, FP64 and mixed) and more times than one grid row of
    workgroups covers (1 satellite x 34,000,000 times: the looping kernel),
    checked on sampled points against the oracle."""
    rng = np.random.default_rng(99)
    for n, T in ((40_000, 27_500), (1, 34_000_000)):
        el = synth.shell_elements(n, 500 + n)
        t = np.linspace(0.0, 10080.0, T)
        k = 4000
        sat = rng.integers(0, n, k)
        col = rng.integers(0, T, k)
        col[:2] = [0, T - 1]
        ro, vo, eo = oracle.propagate_points(el, sat, t[col])
        rec = sg.init(dev(el))
        dt = dev(t)
        flat = dev(sat.astype(np.int64) * T + col)
        for prec in ("fp64", "mixed"):
            say(f"[gpu] maximum size n={n} T={T} {prec}")
            r, v, err = sg.propagate(rec, dt, prec)
            rs = r.reshape(3, -1).index_select(1, flat)
            vs = v.reshape(3, -1).index_select(1, flat)
            es = err.reshape(-1).index_select(0, flat)
            rs, vs, es = host(rs, vs, es)
            del r, v, err
            torch.cuda.empty_cache()
            if prec == "fp64":
                check_fp64(rs, vs, es, ro, vo, eo)
            else:
                assert np.array_equal(es, eo)
                dr, dv = _errors(rs, vs, ro, vo)
                assert dr.max() <= 0.010 and dv.max() <= 1e-5


def test_empty_batches():
    el = synth.shell_elements(4, 5)
    rec = sg.init(dev(el))
    r, v, err = sg.propagate(rec, torch.empty(0, dtype=torch.float64, device=DEV), "fp64")
    assert r.shape == (3, 4, 0)
    rec0 = sg.init(torch.empty((8, 0), dtype=torch.float64, device=DEV))
    r, v, err = sg.propagate(rec0, dev(np.arange(5.0)), "mixed")
    torch.cuda.synchronize()
    assert r.shape == (3, 0, 5)


# --------------------------------------------------------- reduced precision --
def _errors(r, v, ro, vo):
    dr = np.linalg.norm(r.astype(np.float64) - ro, axis=0)
    dv = np.linalg.norm(v.astype(np.float64) - vo, axis=0)
    return dr, dv


def test_mixed_precision_within_10m_to_7_days():
    """100k-satellite elements, 7-day horizon at 10-minute steps, on a seeded
    1% satellite sample: max position error <= 10 m, velocity <= 1e-2 m/s in
    every one-day bin of |time since epoch| (max and RMS reported per bin,
    beside plain FP32 on the same points)."""
    cat = synth.config2("7d", n=100_000)
    idx = synth.sample_satellites(cat.n, 0.01, 2)
    el = cat.elem[:, idx]
    say(f"[gpu] mixed precision 7d sample n={el.shape[1]} T={cat.T}")
    ro, vo, eo = oracle.propagate(el, cat.t, nthreads=NTHREADS)
    tsince = np.abs(cat.t[None, :] - 1440.0 * el[7][:, None]).reshape(-1)
    bins = np.minimum((tsince // 1440).astype(int), 9)
    say("  |t - epoch| bin (days)   mixed max dr (m)  rms dr (m)  max dv (mm/s)   fp32 max dr (m)  rms dr (m)")
    res = {}
    for prec in ("mixed", "fp32"):
        r, v, err = gpu_dense(el, cat.t, prec)
        assert np.array_equal(err, eo)
        res[prec] = _errors(r.reshape(3, -1), v.reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
    for b in range(bins.max() + 1):
        m = bins == b
        if not m.any():
            continue
        dr, dv = res["mixed"][0][m], res["mixed"][1][m]
        fr = res["fp32"][0][m]
        say(f"  [{b}, {b + 1})                 {dr.max() * 1e3:8.3f}      {np.sqrt(np.mean(dr ** 2)) * 1e3:7.3f}"
            f"     {dv.max() * 1e6:8.4f}       {fr.max() * 1e3:10.1f}     {np.sqrt(np.mean(fr ** 2)) * 1e3:8.1f}")
        assert dr.max() <= 0.010 and dv.max() <= 1e-5, b


def test_mixed_precision_one_day_grid_and_starlink():
    for cat in (synth.config2("1d", n=2000), synth.config1()):
        say(f"[gpu] mixed precision {cat.name}")
        r, v, err = gpu_dense(cat.elem, cat.t, "mixed")
        ro, vo, eo = oracle.propagate(cat.elem, cat.t, nthreads=NTHREADS)
        assert np.array_equal(err, eo)
        dr, dv = _errors(r.reshape(3, -1), v.reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
        say(f"  max dr {dr.max() * 1e3:.3f} m, max dv {dv.max() * 1e6:.4f} mm/s")
        assert dr.max() <= 0.010 and dv.max() <= 1e-5


def test_plain_fp32_reproduces_the_papers_error_growth():
    """Plain FP32 (every quantity in float, time since epoch included) drifts
    with the horizon (section 4): metres near epoch, hundreds of metres after
    days, bounded by a few km over 7 days; the mixed path does not drift."""
    cat = synth.config2("7d", n=300)
    cat.elem[7] = 0.0
    say("[gpu] plain fp32 error growth")
    r, v, err = gpu_dense(cat.elem, cat.t, "fp32")
    ro, vo, eo = oracle.propagate(cat.elem, cat.t, nthreads=NTHREADS)
    dr, _ = _errors(r.reshape(3, -1), v.reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
    dr = dr.reshape(cat.n, cat.T)
    early = np.median(dr[:, :6])          # first hour
    late = np.median(dr[:, -144:])        # last day
    say(f"  median first hour {early * 1e3:.2f} m, last day {late * 1e3:.1f} m, max {dr.max():.3f} km")
    assert early < 0.01
    assert late > 5 * early
    assert dr.max() < 5.0


# ------------------------------------------------------------------ ragged --
# Agreement between ragged mappings (km, km/s): one sub-tolerance Kepler step.
MAPPING_TOL = {"fp64": (1e-8, 1e-11), "mixed": (1e-3, 1e-6)}


def small_ragged(n=700, seed=21):
    """Short lognormal lists (several tiles per list, ragged tails), 5% heavy
    drag, and empty lists at the start, middle and end."""
    el = synth.shell_elements(n, seed)
    hot = np.random.default_rng(seed).random(n) < 0.05
    el[6, hot] *= 100.0
    off0, t0 = synth.ragged_lists(n, seed, median=40.0, sigma=1.2, max_len=300)
    L = np.diff(off0)
    drop = np.zeros(n, bool)
    drop[[0, n // 2, n - 1]] = True
    keep = ~np.repeat(drop, L)
    L[drop] = 0
    off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    return el, off, t0[keep]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_all_mappings_match_oracle(prec):
    el, off, t = small_ragged()
    say(f"[gpu] ragged n={el.shape[1]} nnz={t.shape[0]} {prec}")
    rec = sg.init(dev(el))
    doff, dt = dev(off), dev(t)
    ro, vo, eo = oracle.propagate_ragged(el, off, t)
    results = {}
    results["search"] = host(*sg.propagate_ragged(rec, doff, dt, prec))
    for autotune, graph in [(False, False), (True, False), (True, True)]:
        plan = sg.RaggedPlan(rec, doff, dt, prec, autotune=autotune, graph=graph)
        results[f"plan{autotune}{graph}"] = host(*plan.launch())
        say(f"  plan {plan.describe()}")
        plan.close()
    for name, (r, v, err) in results.items():
        if prec == "fp64":
            check_fp64(r, v, err, ro, vo, eo)
        else:
            assert np.array_equal(err, eo), name
            ok = (eo == 0) | (eo == 6)
            dr, dv = _errors(r[:, ok], v[:, ok], ro[:, ok], vo[:, ok])
            assert dr.max() <= 0.010 and dv.max() <= 1e-5, (name, dr.max(), dv.max())
    # Mappings agree to the Kepler tolerance: the loop stops when every lane
    # of a wavefront has converged, so whether a lane takes one more
    # (sub-tolerance) step depends on which points share its wavefront; a
    # step below 1e-12 rad (FP64) or 1e-7 rad (float) moves r by < 7e-9 km or
    # 7e-4 km and v by < 8e-12 km/s or 8e-7 km/s.
    base = results["search"]
    tol_r, tol_v = MAPPING_TOL[prec]
    for name, (r, v, err) in results.items():
        assert np.array_equal(err, base[2])
        ok = (err == 0) | (err == 6)
        assert np.max(np.abs(r[:, ok].astype(np.float64) - base[0][:, ok])) <= tol_r, name
        assert np.max(np.abs(v[:, ok].astype(np.float64) - base[1][:, ok])) <= tol_v, name


def test_ragged_tile_and_flat_modes_explicitly():
    """Every (mapping, workgroup, grid) configuration the autotuner may pick
    gives the same codes and states equal to rounding (1e-8 km, 1e-11 km/s)."""
    el, off, t = small_ragged(300, 5)
    rec = sg.init(dev(el))
    doff, dt = dev(off), dev(t)
    ref = host(*sg.propagate_ragged(rec, doff, dt, "fp64"))
    for mode in (0, 1):
        for block in (64, 128, 256, 512):
            for per_cu in (0, 1, 8):
                plan = sg.RaggedPlan(rec, doff, dt, "fp64", autotune=False, graph=False, config=(mode, block, per_cu))
                out = host(*plan.launch())
                plan.close()
                assert np.array_equal(out[2], ref[2]), (mode, block, per_cu)
                ok = (ref[2] == 0) | (ref[2] == 6)
                assert np.all(np.isnan(out[0][:, ~ok]))
                assert np.max(np.abs(out[0][:, ok] - ref[0][:, ok])) <= 1e-8
                assert np.max(np.abs(out[1][:, ok] - ref[1][:, ok])) <= 1e-11


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_long_lists_every_mapping(prec):
    """Lists of 0 to 5,000 points (several tiles, ragged tails, empty lists):
    one wavefront per tile, the persistent tile loop and the flat mapping match
    the oracle, and the two tile mappings (same 64-point chunks) agree to the
    Kepler tolerance."""
    lens = [0, 1, 63, 64, 65, 127, 128, 129, 1023, 1024, 1025, 2047, 2048, 2049, 3000, 4096, 5000, 0, 700]
    n = len(lens)
    el = synth.shell_elements(n, 31)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    rng = np.random.default_rng(31)
    t = np.concatenate([np.sort(rng.uniform(0.0, 10080.0, L)) for L in lens])
    say(f"[gpu] ragged long lists {prec} nnz={t.shape[0]}")
    rec = sg.init(dev(el))
    doff, dt = dev(off), dev(t)
    ro, vo, eo = oracle.propagate_ragged(el, off, t)
    outs = []
    for cfg in [(0, 256, 0), (0, 256, 1), (1, 128, 0)]:
        plan = sg.RaggedPlan(rec, doff, dt, prec, autotune=False, graph=False, config=cfg)
        r, v, err = host(*plan.launch())
        plan.close()
        if prec == "fp64":
            check_fp64(r, v, err, ro, vo, eo)
        else:
            assert np.array_equal(err, eo), cfg
            ok = (eo == 0) | (eo == 6)
            dr, dv = _errors(r[:, ok], v[:, ok], ro[:, ok], vo[:, ok])
            assert dr.max() <= 0.010 and dv.max() <= 1e-5, (cfg, dr.max(), dv.max())
        outs.append((r, v, err))
    (r, v, err), (r1, v1, e1) = outs[0], outs[1]
    assert np.array_equal(err, e1)
    ok = (err == 0) | (err == 6)
    tol_r, tol_v = MAPPING_TOL[prec]
    assert np.max(np.abs(r[:, ok].astype(np.float64) - r1[:, ok])) <= tol_r
    assert np.max(np.abs(v[:, ok].astype(np.float64) - v1[:, ok])) <= tol_v


def test_ragged_graph_replays_match_eager():
    """A captured plan replayed several times, with eager work between the
    replays, reproduces the plan's direct (uncaptured) launch bit for bit."""
    el, off, t = small_ragged(400, 9)
    rec = sg.init(dev(el))
    doff, dt = dev(off), dev(t)
    plan = sg.RaggedPlan(rec, doff, dt, "fp64", autotune=False, graph=True)
    assert '"graph": true' in plan.describe()
    direct = host(*sg.propagate_ragged(rec, doff, dt, "fp64", plan=plan))
    direct = [x.copy() for x in direct]
    for k in range(4):
        for x in plan.out:
            x.zero_()
        _ = torch.ones(1000, device=DEV).sum()  # unrelated eager work between replays
        out = host(*plan.launch())
        assert np.array_equal(out[2], direct[2]), k
        np.testing.assert_array_equal(np.nan_to_num(out[0], nan=7.0), np.nan_to_num(direct[0], nan=7.0))
        np.testing.assert_array_equal(np.nan_to_num(out[1], nan=7.0), np.nan_to_num(direct[1], nan=7.0))
    plan.close()


def test_ragged_malformed_offsets_rejected():
    el = synth.shell_elements(4, 3)
    rec = sg.init(dev(el))
    t = dev(np.arange(10.0))
    for bad in ([0, 3, 2, 8, 10], [1, 3, 5, 8, 10], [0, 3, 5, 8, 9]):
        with pytest.raises(sg.SGP4Error) as e:
            sg.RaggedPlan(rec, dev(np.array(bad, np.int64)), t, "fp64")
        assert e.value.code == -3


def test_ragged_no_plan_malformed_offsets_give_code_8():
    """Without a plan the offsets are not checked on the host (the search's
    bounds and termination are proven on the CPU in test_ragged_search_cpu):
    a point that the offsets place in no satellite's list gets code 8 and NaN,
    every other point the state of a satellite whose list holds it."""
    el = synth.shell_elements(4, 3)
    rec = sg.init(dev(el))
    tt = np.arange(10.0)
    t = dev(tt)
    ro, vo, eo = oracle.propagate(el, tt)  # [3, 4, 10]: every satellite at every time
    cases = {(0, 3, 2, 8, 10): [], (1, 3, 5, 8, 10): [0], (0, 3, 5, 8, 9): [9], (5, 5, 5, 5, 5): list(range(10)),
             (0, 3, 5, 8, 10): []}
    for bad, unowned in cases.items():
        say(f"[gpu] ragged without plan, offsets {bad}")
        off = np.array(bad, np.int64)
        for prec in ("fp64", "mixed"):
            r, v, err = host(*sg.propagate_ragged(rec, dev(off), t, prec))
            assert sorted(np.flatnonzero(err == 8).tolist()) == unowned, (bad, prec, err)
            assert np.all(np.isnan(r[:, err == 8])) and np.all(np.isnan(v[:, err == 8]))
            for p in np.flatnonzero(err != 8):
                owners = [i for i in range(4) if off[i] <= p < off[i + 1]]
                tol = 1e-6 if prec == "fp64" else 0.010
                match = [i for i in owners
                         if err[p] == eo[i, p] and np.max(np.abs(r[:, p] - ro[:, i, p])) <= tol]
                assert match, (bad, prec, p, owners)


def test_full_size_mega_constellation_sampled():
    """100,000 x 1,440 (the 1-day mega-constellation grid) in FP64 and mixed;
    a 1% satellite sample checked against the oracle at every time."""
    cat = synth.config2("1d")
    idx = synth.sample_satellites(cat.n, 0.01, 2)
    say("[gpu] c2 100000x1440 full size, 1% sample")
    rec = sg.init(dev(cat.elem))
    dt = dev(cat.t)
    ro, vo, eo = oracle.propagate(cat.elem[:, idx], cat.t, nthreads=NTHREADS)
    di = dev(idx)
    for prec in ("fp64", "mixed"):
        r, v, err = sg.propagate(rec, dt, prec)
        rs, vs, es = host(r.index_select(1, di), v.index_select(1, di), err.index_select(0, di))
        del r, v, err
        if prec == "fp64":
            check_fp64(rs, vs, es, ro, vo, eo)
        else:
            assert np.array_equal(es, eo)
            dr, dv = _errors(rs.reshape(3, -1), vs.reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
            assert dr.max() <= 0.010 and dv.max() <= 1e-5


# Where a float path takes a code decision the oracle takes in double, the two
# may differ only when the decision variable lies within the path's error of
# its threshold: the radius r_k within 2e-6 earth radii (13 m) of 1 for code
# 6, the mean eccentricity within 1e-7 of -0.001 for code 1 (the float drag
# term bC5 (sin M - sin M0) rounds at ~1e-7 relative).
MIXED_RK_TIE = 2e-6
MIXED_E_TIE = 1e-7


def test_full_size_ragged_catalogue_codes_and_sample():
    """1,000,000 satellites with lognormal time lists (nnz ~ 4.2e8), 5% high drag,
    one autotuned graph-captured launch per precision.  Codes are compared at
    EVERY point against the oracle (codes-only pass over the whole catalogue);
    the states of every point with a non-zero oracle code, and of 20,000 random
    points, are checked against the oracle one by one."""
    cat = synth.config3()
    say(f"[gpu] c3 ragged full size nnz={cat.nnz}: oracle codes over every point")
    eo_all = oracle.codes_ragged(cat.elem, cat.offsets, cat.t, nthreads=NTHREADS)
    nz = np.flatnonzero(eo_all != 0)
    kinds = {int(c): int((eo_all == c).sum()) for c in np.unique(eo_all)}
    say(f"  oracle codes: {kinds}")
    assert {0, 1, 6} <= set(kinds), kinds
    rng = np.random.default_rng(33)
    pts = np.union1d(np.sort(rng.choice(cat.nnz, 20000, replace=False)), nz)
    sat = np.searchsorted(cat.offsets, pts, side="right") - 1
    ro, vo, eo, det = oracle.propagate_points(cat.elem, sat, cat.t[pts], detail=True)
    assert np.array_equal(eo, eo_all[pts])
    # Conditioning of the sampled points (as for the crafted edge cases): the
    # oracle's state at elements perturbed by 1e-15 relative.  States are
    # compared where it moves by less than 1e-7 km and 1e-10 km/s; beyond that
    # the FP64 state itself is ill conditioned (the decay tail of B* ~ 0.6
    # satellites, where the model's semi-major axis reaches 0.004 earth radii
    # and speeds of thousands of km/s: rounding of the mean anomaly's n t
    # alone moves the state by more than the bars).
    prng = np.random.default_rng(0)
    move = np.zeros(pts.size)
    vmove = np.zeros(pts.size)
    for _ in range(6):
        pert = cat.elem.copy()
        pert[:7] *= 1 + 1e-15 * prng.choice([-1.0, 1.0], size=(7, cat.n))
        r2, v2, _ = oracle.propagate_points(pert, sat, cat.t[pts])
        move = np.maximum(move, np.nan_to_num(np.max(np.abs(r2 - ro), axis=0), nan=np.inf))
        vmove = np.maximum(vmove, np.nan_to_num(np.max(np.abs(v2 - vo), axis=0), nan=np.inf))
    well = (move < 1e-7) & (vmove < 1e-10)
    valid = (eo == 0) | (eo == 6)
    say(f"  {int((valid & ~well).sum())} of {int(valid.sum())} valid sampled states ill conditioned "
        f"(all code 6: {bool(np.all(eo[valid & ~well] == 6))})")
    assert np.all(well[eo == 0])
    rec = sg.init(dev(cat.elem))
    doff, dt = dev(cat.offsets), dev(cat.t)
    dp = dev(pts)
    for prec in ("fp64", "mixed"):
        plan = sg.RaggedPlan(rec, doff, dt, prec, autotune=True, graph=True)
        say(f"  {prec} plan {plan.describe()}")
        r, v, err = plan.launch()
        rs, vs, es = host(r.index_select(1, dp), v.index_select(1, dp), err.index_select(0, dp))
        del r, v
        e_all, = host(err)
        plan.close()
        del err
        diff = np.flatnonzero(e_all != eo_all)
        if prec == "fp64":
            assert diff.size == 0, f"{diff.size} codes differ, first at {diff[:10]}"
            assert np.array_equal(es, eo)
            assert np.all(np.isnan(rs[:, ~valid])) and np.all(np.isnan(vs[:, ~valid]))
            dr = np.max(np.abs(rs[:, well] - ro[:, well]))
            dv = np.max(np.abs(vs[:, well] - vo[:, well]))
            say(f"  fp64 max |dr| {dr:.2e} km, |dv| {dv:.2e} km/s over {int(well.sum())} points")
            assert dr <= 1e-6 and dv <= 1e-9
            continue
        # mixed: every code difference must be a threshold tie
        if diff.size:
            dsat = np.searchsorted(cat.offsets, diff, side="right") - 1
            _, _, _, dd = oracle.propagate_points(cat.elem, dsat, cat.t[diff], detail=True)
            tie6 = np.abs(dd["rk"] - 1.0) <= MIXED_RK_TIE
            tie1 = np.abs(dd["emargin"]) <= MIXED_E_TIE
            assert np.all(tie6 | tie1), f"non-tie code differences at {diff[~(tie6 | tie1)][:10]}"
            say(f"  mixed code ties: {int(tie6.sum())} at r_k = 1, {int(tie1.sum())} at e = -0.001")
        same = es == eo
        ok = same & valid & well
        assert np.all(np.isnan(rs[:, same & ~valid]))
        dr, dv = _errors(rs[:, ok], vs[:, ok], ro[:, ok], vo[:, ok])
        say(f"  mixed max |dr| {dr.max() * 1e3:.3f} m, |dv| {dv.max() * 1e6:.3f} mm/s over {int(ok.sum())} points")
        assert dr.max() <= 0.010 and dv.max() <= 1e-5
