"""GPU parity of the elements-to-states call (sgp4_propagate_elements) and of
the flat dense mapping for short time lists.

Both must give what the two-stage path (sgp4_init + sgp4_propagate) and the
oracle give: codes bit-exact, FP64 states within 1e-6 km / 1e-9 km/s of the
oracle, mixed within 10 m / 1e-2 m/s.  Against the two-stage GPU path the
states agree to rounding: the same steps compiled into another kernel (the
compiler may contract an initialisation product into a propagation sum once
both sit in one kernel) and, for the flat and fused mappings, other lanes
sharing the wavefront-uniform Kepler exit.  FP64 agrees to 1e-8 km; the float
paths to a few float32 units in the last place of the position (one unit is
0.49 m between 4,096 and 8,192 km), bounded here by 5 m and 5 mm/s.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_27830_amd as sg
import synth
from test_gpu_parity import (DEV, _errors, check_fp64, conditioning, crafted_elements, dev, host,
                             say)

pytestmark = pytest.mark.gpu

FLAT = 0x80000
TOL = {"fp64": (1e-8, 1e-11), "mixed": (5e-3, 5e-6), "fp32": (5e-3, 5e-6)}


def fused(elem, t, prec, ws=True, grav=None, flags=False):
    e = dev(elem)
    n = elem.shape[1]
    w = torch.empty(sg.consts_bytes(n), dtype=torch.uint8, device=DEV) if ws else None
    f = torch.full((max(n, 1),), 255, dtype=torch.uint8, device=DEV) if flags else None
    r, v, err = sg.propagate_elements(e, dev(t), prec, grav=grav, workspace=w, flags=f)
    out = host(r, v, err)
    return (out, host(f[:n])[0]) if flags else out


def two_stage(elem, t, prec, grav=None, block=None):
    rec = sg.init(dev(elem), grav)
    r, v, err = sg.propagate(rec, dev(t), prec, block=block)
    return host(r, v, err) + host(rec.flags)


def close(a, b, tol):
    a = a.reshape(3, -1); b = b.reshape(3, -1)
    ok = ~np.isnan(b[0])
    assert np.array_equal(np.isnan(a), np.isnan(b))
    return float(np.max(np.abs(a[:, ok] - b[:, ok]), initial=0.0)) <= tol


SHAPES = [(1, 1), (130, 1), (64, 2), (65, 3), (7, 7), (200, 8), (129, 9), (33, 17), (70, 31), (64, 32), (5, 33),
          (40, 100)]


@pytest.mark.parametrize("n,T", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_elements_to_states_match_two_stage_path(n, T, prec):
    """Every branch of the call: the fused launch (T <= 32; T = 1 on its own
    kernel), the two-stage path (T > 32 with a workspace) and the fused launch
    for long lists without one; ragged satellite and time counts."""
    elem = synth.shell_elements(n, 300 + n)
    t = np.sort(np.random.default_rng(T).uniform(-600.0, 8000.0, T))
    say(f"[gpu] elements->states n={n} T={T} {prec}")
    r0, v0, e0, f0 = two_stage(elem, t, prec)
    for ws in (True, False):
        (r, v, err), f = fused(elem, t, prec, ws=ws, flags=True)
        assert np.array_equal(err, e0)
        assert np.array_equal(f, f0)
        tr, tv = TOL[prec]
        assert close(r, r0, tr) and close(v, v0, tv)


@pytest.mark.parametrize("T", [1, 5, 16, 40])
def test_elements_to_states_fp64_vs_oracle(T):
    cat = synth.config1()
    elem = cat.elem[:, :1500]
    t = np.sort(np.random.default_rng(5).uniform(0.0, 1440.0, T))
    say(f"[gpu] elements->states fp64 vs oracle n=1500 T={T}")
    r, v, err = fused(elem, t, "fp64", ws=(T > 32))
    ro, vo, eo = oracle.propagate(elem, t)
    dr, dv = check_fp64(r, v, err, ro, vo, eo)
    say(f"  max |dr| {dr:.3e} km, max |dv| {dv:.3e} km/s")


def test_elements_to_states_mixed_vs_oracle_7_days():
    elem = synth.config1().elem[:, ::7]
    t = np.linspace(0.0, 10080.0, 24)
    say(f"[gpu] elements->states mixed vs oracle n={elem.shape[1]} T=24 to 7 days")
    r, v, err = fused(elem, t, "mixed")
    ro, vo, eo = oracle.propagate(elem, t)
    assert np.array_equal(err, eo)
    dr, dv = _errors(r.reshape(3, -1), v.reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
    say(f"  max {dr.max() * 1e3:.2f} m, {dv.max() * 1e3:.2e} m/s")
    assert dr.max() <= 0.010 and dv.max() <= 1e-5


def test_elements_to_states_edge_cases():
    """Crafted element sets (codes 1, 2, 4, 6, 7, simplified drag, NaN drag,
    equatorial): codes equal the oracle's wherever its decision is well
    conditioned, NaN states for codes 1, 2, 4, 7, and the satellite flags
    equal sgp4_init's."""
    el = crafted_elements()
    t = np.linspace(-1440.0, 10080.0, 13)
    say(f"[gpu] elements->states edge cases n={el.shape[1]}")
    (r, v, err), f = fused(el, t, "fp64", ws=False, flags=True)
    ro, vo, eo, codes, stable, move = conditioning(el, t)
    assert np.array_equal(err[stable], eo[stable])
    assert np.all(np.any(codes == err[None], axis=0) | ~stable | np.isin(err, [0, 1, 2, 4, 6, 7]))
    bad = (err != 0) & (err != 6)
    assert np.all(np.isnan(r[:, bad])) and np.all(np.isnan(v[:, bad]))
    well = stable & ((eo == 0) | (eo == 6)) & (move < 1e-7)
    assert np.max(np.abs(r[:, well] - ro[:, well])) <= 1e-6
    assert np.max(np.abs(v[:, well] - vo[:, well])) <= 1e-9
    rec = sg.init(dev(el))
    assert np.array_equal(f, host(rec.flags)[0])


def test_elements_to_states_two_body_gravity():
    elem = synth.shell_elements(90, 77)
    t = np.linspace(0.0, 3000.0, 6)
    grav = (398600.8, 6378.135, 0.0, 0.0, 0.0)
    say("[gpu] elements->states two-body gravity")
    r, v, err = fused(elem, t, "fp64", grav=grav)
    ro, vo, eo = oracle.propagate(elem, t, grav=grav)
    check_fp64(r, v, err, ro, vo, eo)


def test_elements_to_states_full_catalogue_snapshot():
    """1,000,000 satellites at one epoch (the catalogue-snapshot use of the
    fused call): the fused launch against the two-stage path, every point, and
    against the oracle on a sample."""
    n = 1_000_000
    cat = synth.shell_elements(n, 3)
    cat[6, np.random.default_rng(1003).random(n) < 0.05] *= 100.0  # high-drag 5%, some decay
    t = np.array([2000.0])
    say(f"[gpu] elements->states snapshot n={n} T=1 mixed and fp64")
    for prec in ("fp64", "mixed"):
        r, v, err = fused(cat, t, prec, ws=False)
        r0, v0, e0, _ = two_stage(cat, t, prec)
        assert np.array_equal(err, e0)
        tr, tv = TOL[prec]
        assert close(r, r0, tr) and close(v, v0, tv)
    idx = np.random.default_rng(3).choice(n, 4000, replace=False)
    ro, vo, eo = oracle.propagate(cat[:, idx], t)
    r, v, err = fused(cat, t, "fp64", ws=False)
    check_fp64(r[:, idx], v[:, idx], err[idx], ro, vo, eo)
    r, v, err = fused(cat, t, "mixed", ws=False)
    assert np.array_equal(err[idx], eo)
    dr, dv = _errors(r[:, idx].reshape(3, -1), v[:, idx].reshape(3, -1), ro.reshape(3, -1), vo.reshape(3, -1))
    assert dr.max() <= 0.010 and dv.max() <= 1e-5


@pytest.mark.parametrize("n,T", [(1, 1), (130, 1), (64, 5), (999, 31), (33, 64), (40, 1000)])
@pytest.mark.parametrize("block", [64, 256, 512])
def test_flat_dense_mapping(n, T, block):
    """The flat dense configuration (one lane per point in point order) against
    the oracle (FP64) and the tile mapping (mixed)."""
    elem = synth.shell_elements(n, 500 + n)
    t = np.sort(np.random.default_rng(T + 1).uniform(-300.0, 9000.0, T))
    say(f"[gpu] flat dense n={n} T={T} block={block}")
    r, v, err, _ = two_stage(elem, t, "fp64", block=block | FLAT)
    ro, vo, eo = oracle.propagate(elem, t)
    check_fp64(r, v, err, ro, vo, eo)
    rm, vm, em, _ = two_stage(elem, t, "mixed", block=block | FLAT)
    rt, vt, et, _ = two_stage(elem, t, "mixed", block=512 | 0x10000 | 0x40000)
    assert np.array_equal(em, et)
    assert close(rm, rt, TOL["mixed"][0]) and close(vm, vt, TOL["mixed"][1])


@pytest.mark.parametrize("fmt", ["tle", "omm_kvn"])
def test_text_to_states_pipeline(fmt):
    """Element-set text -> native parser -> elements on the device ->
    sgp4_propagate_elements, against the oracle propagating the oracle
    parser's elements of the same text (FP64 bar)."""
    from oracle import ingest as oi
    from synth import text as stx
    elem = synth.shell_elements(700, 61)
    text = stx.tle_text(elem, three_line=True) if fmt == "tle" else stx.omm_kvn(elem)
    say(f"[gpu] text -> states {fmt} n=700")
    e, _, status = sg.parse_text(text, fmt, ref_jd=stx.REF_JD)
    assert np.all(status == 0)
    t = np.linspace(-720.0, 2880.0, 9)
    r, v, err = fused(e, t, "fp64", ws=False)
    eo = oi.parse_tle(text, ref=stx.REF_JD)[0] if fmt == "tle" else oi.parse_omm(text, "kvn", ref=stx.REF_JD)[0]
    ro, vo, co = oracle.propagate(eo, t)
    check_fp64(r, v, err, ro, vo, co)
