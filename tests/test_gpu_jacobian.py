"""GPU Jacobian d(r, v)/d(elements) per point against the CPU dual-number oracle,
the GPU VJP (its contraction) and between precisions.

Bars: FP64 vs the oracle's forward-mode (dual-number) Jacobian to 1e-8 of each
(component, element) column's scale; NaN exactly where the oracle's code is 1,
2, 4 or 7; the Jacobian contracted with a cotangent equals the VJP to 1e-10;
FP32-mixed vs FP64 to 1e-4 of the column scale (the mixed forward state carries
~1e-7 relative error; measured ~2e-6).  Deep-space satellites are not
differentiated (NaN).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_27830_amd as sg
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def gpu_jacobian(elem, t, prec):
    rec = sg.init(dev(elem))
    J = sg.jacobian(rec, dev(t), prec)
    torch.cuda.synchronize()
    return J.cpu().numpy()  # [6, 7, n, T]


def oracle_jacobian(elem, t):
    n, T = elem.shape[1], t.shape[0]
    sat = np.repeat(np.arange(n), T)
    J, r, v, err = oracle.jacobian_points(elem, sat, np.tile(t, n))
    return np.transpose(J, (1, 2, 0)).reshape(6, 7, n, T), err.reshape(n, T)


def column_error(J, ref, valid):
    """max over (component, element) of max |J - ref| / max |ref| over the valid points."""
    d = np.abs(J - ref)[:, :, valid]
    s = np.abs(ref)[:, :, valid].max(axis=2, keepdims=True) + 1e-300
    return float((d / s).max())


def test_jacobian_fp64_matches_dual_oracle():
    cat = synth.config1(24, 30)
    say("[gpu] jacobian fp64 24 x 30")
    J = gpu_jacobian(cat.elem, cat.t, "fp64")
    ref, err = oracle_jacobian(cat.elem, cat.t)
    valid = (err == 0) | (err == 6)
    assert valid.all()
    e = column_error(J, ref, valid)
    say(f"  max column-relative error {e:.3e}")
    assert e <= 1e-8


def test_jacobian_edge_sets_nan_where_no_state():
    el = synth.shell_elements(20, 8)
    ke = 60.0 / np.sqrt(6378.135 ** 3 / 398600.8)
    el[0, :4] = ke * ((6378.135 + 200.0) / 6378.135) ** -1.5      # perigee below 220 km
    el[6, 4:8] = 2e-3                                              # heavy drag
    el[0, 8:10] = 2 * np.pi / 300.0                                # deep space: not differentiated
    el[1, 10:12] = 1.5                                             # invalid eccentricity: code 1
    t = np.linspace(0.0, 10080.0, 40)
    say("[gpu] jacobian fp64 edge sets")
    J = gpu_jacobian(el, t, "fp64")
    ref, err = oracle_jacobian(el, t)
    valid = (err == 0) | (err == 6)
    valid[8:10] = False
    assert np.array_equal(np.isnan(J).all(axis=(0, 1)), ~valid)
    assert np.isfinite(J[:, :, valid]).all()
    assert column_error(J, ref, valid) <= 1e-7


def test_jacobian_contracts_to_the_vjp():
    cat = synth.config1(40, 50)
    rng = np.random.default_rng(9)
    gr = rng.normal(size=(3, cat.n, cat.T))
    gv = rng.normal(size=(3, cat.n, cat.T)) * 1e3
    say("[gpu] jacobian contracted vs vjp")
    rec = sg.init(dev(cat.elem))
    J = sg.jacobian(rec, dev(cat.t), "fp64").cpu().numpy()
    g = sg.vjp(rec, dev(cat.t), dev(gr), dev(gv), "fp64").cpu().numpy()
    cot = np.concatenate([gr, gv])                               # [6, n, T]
    contracted = np.einsum("cmit,cit->mi", J, cot)
    scale = np.abs(g).max(axis=1, keepdims=True) + 1e-300
    e = float((np.abs(contracted - g) / scale).max())
    say(f"  max relative difference {e:.3e}")
    assert e <= 1e-10


def test_jacobian_mixed_matches_fp64():
    cat = synth.config1(64, 40)
    say("[gpu] jacobian mixed vs fp64")
    J64 = gpu_jacobian(cat.elem, cat.t, "fp64")
    J32 = gpu_jacobian(cat.elem, cat.t, "mixed")
    valid = np.ones((cat.n, cat.T), bool)
    e = column_error(J32, J64, valid)
    say(f"  max column-relative difference {e:.3e}")
    assert e <= 1e-4


def test_jacobian_rejects_plain_fp32():
    rec = sg.init(dev(synth.config0().elem))
    with pytest.raises(Exception):
        sg.jacobian(rec, dev(synth.config0().t), "fp32")


def test_jacobian_ragged_oracle_dense_and_vjp():
    """Jacobian over per-satellite time lists (empty lists and a deep-space
    satellite among them): FP64 against the oracle's dual-number Jacobian at
    the same points to 1e-8 of each column's scale, mixed against FP64 to
    1e-4, NaN at every point of the deep-space satellite; contracted with a
    cotangent it equals sgp4_vjp_ragged to 1e-10; a dense grid given as lists
    equals sgp4_jacobian bit for bit."""
    cat = synth.config1(50, 1)
    el = cat.elem.copy()
    el[:, 9] = synth.config5(12, 1).elem[:, 2]
    el[7, 9] = 0.0
    rng = np.random.default_rng(41)
    lens = rng.integers(0, 40, el.shape[1])
    lens[[0, 20]] = 0
    offsets = np.zeros(el.shape[1] + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    nnz = int(offsets[-1])
    t = np.concatenate([np.sort(rng.uniform(-300.0, 3000.0, L)) for L in lens])
    say(f"[gpu] jacobian ragged n={el.shape[1]} nnz={nnz}")
    rec = sg.init(dev(el))
    J64 = sg.jacobian_ragged(rec, dev(offsets), dev(t), "fp64").cpu().numpy()
    J32 = sg.jacobian_ragged(rec, dev(offsets), dev(t), "mixed").cpu().numpy()
    sat = np.repeat(np.arange(el.shape[1]), lens)
    ref, _, _, err = oracle.jacobian_points(el, sat, t)
    ref = np.transpose(ref, (1, 2, 0))  # [6, 7, nnz]
    deep = sat == 9
    assert deep.sum() > 0 and np.all(np.isnan(J64[:, :, deep])) and np.all(np.isnan(J32[:, :, deep]))
    valid = ((err == 0) | (err == 6)) & ~deep
    e64 = column_error(J64, ref, valid)
    e32 = column_error(J32, J64, valid)
    say(f"  fp64 vs oracle {e64:.2e}, mixed vs fp64 {e32:.2e}")
    assert e64 <= 1e-8 and e32 <= 1e-4
    # the contraction with a cotangent is the ragged VJP
    gr = rng.normal(size=(3, nnz))
    gv = rng.normal(size=(3, nnz)) * 1e3
    g = sg.vjp_ragged(rec, dev(offsets), dev(t), dev(gr), dev(gv), "fp64").cpu().numpy()
    Jv = np.where(np.isnan(J64), 0.0, J64)
    contr = np.einsum("cmp,cp->mp", Jv[:3], gr) + np.einsum("cmp,cp->mp", Jv[3:], gv)
    want = np.zeros((7, el.shape[1]))
    np.add.at(want.T, sat, contr.T)
    keep = np.ones(el.shape[1], bool)
    keep[9] = False
    scale = np.abs(want[:, keep]).max(axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(g[:, keep] - want[:, keep]) / scale) <= 1e-10
    # a dense grid given as lists
    d = synth.config1(20, 33)
    recd = sg.init(dev(d.elem))
    dense = sg.jacobian(recd, dev(d.t), "fp64")
    lists = sg.jacobian_ragged(recd, dev(np.arange(d.n + 1, dtype=np.int64) * d.T), dev(np.tile(d.t, d.n)), "fp64")
    torch.cuda.synchronize()
    assert torch.equal(dense.reshape(6, 7, -1), lists)
