"""Seeded generators are deterministic and shaped like the workloads; the oracle
still reproduces its stored regression fixture."""
import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_generators_are_deterministic_and_shaped():
    a, b = synth.config0(), synth.config0()
    assert np.array_equal(a.elem, b.elem) and np.array_equal(a.t, b.t)
    assert a.elem.shape == (8, 64) and a.t.shape == (100,) and a.t[0] == 0.0 and a.t[-1] == 1440.0
    revs = a.elem[0] * 1440 / (2 * np.pi)
    assert revs.min() >= 14.8 and revs.max() <= 15.3
    assert a.elem[1].min() >= 1e-5 and a.elem[1].max() <= 2e-3
    assert set(np.round(np.rad2deg(a.elem[2]), 6)) <= {43.0, 53.0, 70.0, 97.6}
    c = synth.config1(2000, 10)
    assert np.all(np.abs(c.elem[7]) <= 3.0)
    inc = np.round(np.rad2deg(c.elem[2]), 6)
    frac = {d: np.mean(inc == d) for d in (53.0, 53.2, 70.0, 97.6, 43.0)}
    assert abs(frac[53.0] - 0.40) < 0.04 and abs(frac[97.6] - 0.10) < 0.03
    revs = c.elem[0] * 1440 / (2 * np.pi)
    assert revs.min() > 14.8 and revs.max() < 15.3


def test_ragged_lists_sorted_and_bounded():
    off, t = synth.ragged_lists(3000, 3)
    L = np.diff(off)
    assert off[0] == 0 and off[-1] == t.shape[0] and L.min() >= 1 and L.max() <= 4096
    assert 200 < np.median(L) < 320
    assert t.min() >= 0 and t.max() <= 10080
    for i in range(0, 3000, 37):
        assert np.all(np.diff(t[off[i]:off[i + 1]]) >= 0)
    off2, t2 = synth.ragged_lists(3000, 3)
    assert np.array_equal(off, off2) and np.array_equal(t, t2)


def test_oracle_reproduces_regression_fixture():
    rows = np.loadtxt(os.path.join(HERE, "golden", "c0_oracle_sample.txt"))
    cat = synth.config0()
    sat = rows[:, 0].astype(np.int64)
    r, v, err = oracle.propagate_points(cat.elem, sat, rows[:, 1])
    assert np.array_equal(err, rows[:, 2].astype(np.uint8))
    assert np.max(np.abs(r.T - rows[:, 3:6])) <= 1e-9
    assert np.max(np.abs(v.T - rows[:, 6:9])) <= 1e-12
