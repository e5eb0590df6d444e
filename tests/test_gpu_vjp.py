"""GPU VJP against the CPU dual-number oracle, central finite differences and
the autograd wrapper.

Bars: FP64 VJP vs the oracle's forward-mode (dual-number) VJP to 1e-8
relative per satellite (both differentiate the same function; the oracle
iterates Newton with duals, the kernel uses the implicit-function theorem at
the root); FP32-mixed vs FP64 and vs the dual oracle for the same cotangent
to 1e-4 relative (the forward state of the mixed path carries ~1e-7 relative
error; measured ~2e-6); the VJP of a least-squares loss vs central
differences of that loss to 1e-5 relative (FP64), and for the mixed path vs
central differences of the mixed loss to 2% plus its rounding noise.
"""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def rel_err_per_sat(g, ref):
    """max over satellites of |g - ref| / |ref| (norms over the 7 elements, each
    element scaled by its column's typical size so angles and B* compare fairly)."""
    scale = np.median(np.abs(ref), axis=1, keepdims=True) + 1e-300
    d = np.linalg.norm((g - ref) / scale, axis=0)
    n = np.linalg.norm(ref / scale, axis=0) + 1e-300
    return np.max(d / n)


def gpu_vjp(elem, t, gr, gv, prec):
    rec = sg.init(dev(elem))
    dt = torch.float64 if prec == "fp64" else torch.float32
    g = sg.vjp(rec, dev(t), dev(gr).to(dt), None if gv is None else dev(gv).to(dt), prec)
    torch.cuda.synchronize()
    return g.cpu().numpy()


@pytest.mark.parametrize("with_gv", [False, True])
def test_vjp_fp64_matches_dual_oracle(with_gv):
    cat = synth.config1(96, 37)
    rng = np.random.default_rng(5)
    gr = rng.normal(size=(3, cat.n, cat.T))
    gv = rng.normal(size=(3, cat.n, cat.T)) * 1e3 if with_gv else None
    say(f"[gpu] vjp fp64 96 x 37 gv={with_gv}")
    g = gpu_vjp(cat.elem, cat.t, gr, gv, "fp64")
    ref = oracle.vjp(cat.elem, cat.t, gr, gv)
    err = rel_err_per_sat(g, ref)
    say(f"  max relative error per satellite {err:.3e}")
    assert err <= 1e-8


def test_vjp_simplified_drag_and_invalid_points():
    """Low-perigee (simplified drag) and heavy-drag sets differentiate like the
    oracle; invalid element sets (code 1 at every point) get a zero gradient;
    deep-space sets are not differentiated by the library (NaN)."""
    el = synth.shell_elements(40, 8)
    ke = 60.0 / np.sqrt(6378.135 ** 3 / 398600.8)
    el[0, :8] = ke * ((6378.135 + 200.0) / 6378.135) ** -1.5      # perigee below 220 km
    el[6, 8:16] = 2e-3                                              # heavy drag (20x the median)
    el[0, 16:18] = 2 * np.pi / 300.0                                # deep space: not differentiated
    el[1, 18:20] = 1.5                                              # invalid eccentricity: code 1
    t = np.linspace(0.0, 10080.0, 64)
    rng = np.random.default_rng(6)
    gr = rng.normal(size=(3, el.shape[1], t.shape[0]))
    say("[gpu] vjp fp64 edge sets")
    g = gpu_vjp(el, t, gr, None, "fp64")
    ref = oracle.vjp(el, t, gr, None)
    assert np.all(np.isnan(g[:, 16:18]))
    assert np.all(g[:, 18:20] == 0.0) and np.all(ref[:, 18:20] == 0.0)
    keep = np.ones(el.shape[1], bool)
    keep[16:20] = False
    assert np.all(np.isfinite(g[:, keep]))
    assert rel_err_per_sat(g[:, keep], ref[:, keep]) <= 1e-7


def test_vjp_mixed_matches_fp64_for_the_same_cotangent():
    cat = synth.config1(200, 50)
    rng = np.random.default_rng(7)
    gr = rng.normal(size=(3, cat.n, cat.T)).astype(np.float32).astype(np.float64)
    say("[gpu] vjp mixed vs fp64")
    g64 = gpu_vjp(cat.elem, cat.t, gr, None, "fp64")
    g32 = gpu_vjp(cat.elem, cat.t, gr, None, "mixed")
    err = rel_err_per_sat(g32, g64)
    say(f"  mixed vs fp64 max relative error per satellite {err:.3e}")
    assert err <= 1e-4


def test_vjp_mixed_matches_dual_oracle():
    """The mixed VJP against the FP64 dual-number oracle on the same (float-
    representable) cotangent: within 1e-4 per satellite, the forward mixed
    state's relative error carried through the sweep."""
    cat = synth.config1(40, 50)
    rng = np.random.default_rng(11)
    gr = rng.normal(size=(3, cat.n, cat.T)).astype(np.float32).astype(np.float64)
    say("[gpu] vjp mixed vs dual oracle")
    g32 = gpu_vjp(cat.elem, cat.t, gr, None, "mixed")
    ref = oracle.vjp(cat.elem, cat.t, gr, None)
    err = rel_err_per_sat(g32, ref)
    say(f"  max relative error per satellite {err:.3e}")
    assert err <= 1e-4


def _loss_and_grad(cat, r_obs, prec):
    elem = dev(cat.elem).requires_grad_(True)
    r, v, err = sg.SGP4Function.apply(elem, dev(cat.t), prec)
    loss = ((r.double() - dev(r_obs)) ** 2).sum()
    loss.backward()
    return loss.item(), elem.grad.cpu().numpy()


def test_least_squares_gradient_matches_central_differences():
    """Loss = sum |r(theta) - r_obs|^2 with observations from perturbed truth
    elements plus 10 m noise (the differentiation workload's recipe): the
    autograd gradient (hand-written VJP) equals central differences of the
    loss evaluated by the FP64 forward kernel."""
    cat, truth, noise = synth.config4(24, 40)
    ro, _, eo = oracle.propagate(truth, cat.t)
    r_obs = ro + noise
    assert np.all(eo == 0)
    say("[gpu] least-squares gradient vs central differences")
    loss, grad = _loss_and_grad(cat, r_obs, "fp64")
    assert np.all(grad[7] == 0.0)
    steps = [1e-9, 1e-7, 1e-7, 1e-7, 1e-7, 1e-7, 1e-7]
    for m, h in enumerate(steps):
        for i in (0, 7, 19):
            def L(delta):
                el = cat.elem.copy()
                el[m, i] += delta
                rec = sg.init(dev(el))
                r, _, _ = sg.propagate(rec, dev(cat.t), "fp64")
                return float(((r - dev(r_obs)) ** 2).sum().item())
            fd = (L(h) - L(-h)) / (2 * h)
            assert abs(fd - grad[m, i]) <= 1e-5 * abs(grad[m, i]) + 1e-6 * abs(loss) / max(abs(cat.elem[m, i]), 1e-3), \
                (m, i, fd, grad[m, i])


def test_mixed_least_squares_gradient_matches_central_differences():
    """The same loss evaluated by the mixed forward kernel: its autograd gradient
    (the mixed VJP) against central differences of the mixed loss, with steps
    that move the positions by tens of metres so that the float rounding of the
    states (a few decimetres, ~1e-3 km^2 in the loss) stays below the
    difference; bar 2% of the gradient plus that noise over the step."""
    cat, truth, noise = synth.config4(24, 40)
    ro, _, eo = oracle.propagate(truth, cat.t)
    r_obs = ro + noise
    say("[gpu] mixed least-squares gradient vs central differences of the mixed loss")
    loss, grad = _loss_and_grad(cat, r_obs, "mixed")
    steps = [1e-8, 1e-5, 1e-5, 1e-5, 1e-5, 1e-5, 1e-5]
    worst = 0.0
    for m, h in enumerate(steps):
        for i in (0, 7, 19):
            def L(delta):
                el = cat.elem.copy()
                el[m, i] += delta
                rec = sg.init(dev(el))
                r, _, _ = sg.propagate(rec, dev(cat.t), "mixed")
                return float(((r.double() - dev(r_obs)) ** 2).sum().item())
            fd = (L(h) - L(-h)) / (2 * h)
            bar = 2e-2 * abs(grad[m, i]) + 2e-3 / (2 * h)
            worst = max(worst, abs(fd - grad[m, i]) / bar)
            assert abs(fd - grad[m, i]) <= bar, (m, i, fd, grad[m, i])
    say(f"  worst |fd - grad| / bar = {worst:.3f}")


def test_autograd_gradient_equals_direct_vjp_call():
    cat = synth.config1(30, 20)
    rng = np.random.default_rng(3)
    w = dev(rng.normal(size=(3, cat.n, cat.T)))
    elem = dev(cat.elem).requires_grad_(True)
    r, v, _ = sg.SGP4Function.apply(elem, dev(cat.t), "fp64")
    (r * w).sum().backward()
    rec = sg.init(dev(cat.elem))
    g = sg.vjp(rec, dev(cat.t), w, None, "fp64")
    torch.cuda.synchronize()
    assert torch.equal(elem.grad[:7], g)
    assert torch.all(elem.grad[7] == 0)


def test_vjp_repeatable_bit_for_bit():
    cat = synth.config1(64, 300)
    gr = np.random.default_rng(11).normal(size=(3, cat.n, cat.T))
    a = gpu_vjp(cat.elem, cat.t, gr, None, "fp64")
    b = gpu_vjp(cat.elem, cat.t, gr, None, "fp64")
    assert np.array_equal(a, b)


def test_vjp_full_size_differentiation_workload():
    """9,341 x 1,000 (config-1 elements), observations from the perturbed truth
    plus 10 m noise, g_r = 2 (r - r_obs): FP64 and mixed VJPs on the whole grid;
    a seeded sample of 40 satellites checked against the dual-number oracle."""
    cat, truth, noise = synth.config4()
    say("[gpu] full-size differentiation workload 9341 x 1000")
    ro, _, _ = oracle.propagate(truth, cat.t, nthreads=NTHREADS)
    r_obs = ro + noise
    rec = sg.init(dev(cat.elem))
    r, _, _ = sg.propagate(rec, dev(cat.t), "fp64")
    gr = 2.0 * (r - dev(r_obs))
    g64 = sg.vjp(rec, dev(cat.t), gr, None, "fp64").cpu().numpy()
    r32, _, _ = sg.propagate(rec, dev(cat.t), "mixed")
    g32 = sg.vjp(rec, dev(cat.t), 2.0 * (r32.double() - dev(r_obs)).float(), None, "mixed").cpu().numpy()
    idx = synth.sample_satellites(cat.n, 40 / cat.n, 4)
    gr_s = gr.cpu().numpy()[:, idx, :]
    ref = oracle.vjp(cat.elem[:, idx], cat.t, gr_s, None)
    err = rel_err_per_sat(g64[:, idx], ref)
    say(f"  fp64 vs oracle on 40 satellites: {err:.3e}")
    assert err <= 1e-8
    assert np.all(np.isfinite(g32))
    # the residuals differ between the paths (mixed positions carry ~1 m); the
    # gradients agree to the residual's relative difference
    err32 = rel_err_per_sat(g32[:, idx], g64[:, idx])
    say(f"  mixed vs fp64 (own residuals) on 40 satellites: {err32:.3e}")
    assert err32 <= 0.2
    # the same cotangent for both paths (the FP64 residuals rounded to float):
    # the gradients then agree to the mixed forward state's relative error
    g32s = sg.vjp(rec, dev(cat.t), gr.float(), None, "mixed").cpu().numpy()
    g64s = sg.vjp(rec, dev(cat.t), gr.float().double(), None, "fp64").cpu().numpy()
    err_same = rel_err_per_sat(g32s, g64s)
    say(f"  mixed vs fp64 (same cotangent) on all satellites: {err_same:.3e}")
    assert err_same <= 1e-4


def test_vjp_ragged_matches_dual_oracle_dense_and_clamped_offsets():
    """VJP over per-satellite time lists (empty lists, a deep-space satellite
    and a simplified-drag set among them): FP64 against the oracle's ragged
    dual-number VJP to 1e-8 relative per satellite, FP32-mixed against FP64
    for the same cotangent to 1e-4; empty lists give zero columns, the
    deep-space satellite NaN; a dense grid given as lists equals sgp4_vjp bit
    for bit; malformed offsets give the gradient of the clamped lists."""
    cat = synth.config1(80, 1)
    el = cat.elem.copy()
    el[:, 7] = synth.config5(8, 1).elem[:, 3]
    el[7, 7] = 0.0
    ke = oracle.ke()
    el[0, 11] = ke * ((6378.135 + 200.0) / 6378.135) ** -1.5     # perigee below 220 km: simplified drag
    rng = np.random.default_rng(31)
    lens = rng.integers(0, 60, el.shape[1])
    lens[[0, 5, 40]] = 0
    offsets = np.zeros(el.shape[1] + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    nnz = int(offsets[-1])
    t = np.concatenate([np.sort(rng.uniform(-500.0, 4000.0, L)) for L in lens])
    gr = rng.normal(size=(3, nnz))
    gv = rng.normal(size=(3, nnz)) * 1e3
    say(f"[gpu] vjp ragged n={el.shape[1]} nnz={nnz}")
    rec = sg.init(dev(el))
    g64 = sg.vjp_ragged(rec, dev(offsets), dev(t), dev(gr), dev(gv), "fp64").cpu().numpy()
    g32 = sg.vjp_ragged(rec, dev(offsets), dev(t), dev(gr).float(), dev(gv).float(), "mixed").cpu().numpy()
    want = oracle.vjp_ragged(el, offsets, t, gr, gv)
    deep = np.zeros(el.shape[1], bool)
    deep[7] = True
    assert np.all(np.isnan(g64[:, deep])) and np.all(np.isnan(g32[:, deep]))
    empty = lens == 0
    assert np.all(g64[:, empty] == 0.0) and np.all(g32[:, empty] == 0.0)
    use = ~deep & ~empty
    e64 = rel_err_per_sat(g64[:, use], want[:, use])
    e32 = rel_err_per_sat(g32[:, use], g64[:, use])
    say(f"  fp64 vs oracle {e64:.2e}, mixed vs fp64 {e32:.2e}")
    assert e64 <= 1e-8 and e32 <= 1e-4
    # a dense grid given as lists: the dense kernel's result, bit for bit
    d = synth.config1(32, 20)
    gd = rng.normal(size=(3, d.n, d.T))
    recd = sg.init(dev(d.elem))
    dense = sg.vjp(recd, dev(d.t), dev(gd), None, "fp64")
    lists = sg.vjp_ragged(recd, dev(np.arange(d.n + 1, dtype=np.int64) * d.T), dev(np.tile(d.t, d.n)),
                          dev(gd.reshape(3, -1)), None, "fp64")
    torch.cuda.synchronize()
    assert torch.equal(dense, lists)
    # malformed offsets (decreasing, negative, past nnz): each satellite's
    # clamped range, never an out-of-range read
    bad = offsets.copy()
    bad[3] = bad[5] + 7          # decreasing afterwards
    bad[10] = -40
    bad[50] = nnz + 100
    gb = sg.vjp_ragged(rec, dev(bad), dev(t), dev(gr), dev(gv), "fp64").cpu().numpy()
    for i in range(el.shape[1]):
        lo = min(max(int(bad[i]), 0), nnz)
        hi = min(max(int(bad[i + 1]), lo), nnz)
        if deep[i]:
            assert np.all(np.isnan(gb[:, i]))
            continue
        wi = oracle.vjp_ragged(el[:, i:i + 1], np.array([0, hi - lo]), t[lo:hi], gr[:, lo:hi], gv[:, lo:hi])[:, 0]
        if hi == lo:
            assert np.all(gb[:, i] == 0.0)
        else:
            assert rel_err_per_sat(gb[:, i:i + 1], wi[:, None]) <= 1e-8, i


def test_ragged_autograd_gradient_equals_direct_vjp_call():
    """SGP4RaggedFunction: a loss on the ragged states, backward through the
    ragged VJP, equals the direct sgp4_vjp_ragged call for the same cotangent,
    bit for bit, in both precisions."""
    cat = synth.config1(40, 1)
    rng = np.random.default_rng(13)
    lens = rng.integers(0, 30, cat.n)
    offsets = np.zeros(cat.n + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    t = np.concatenate([np.sort(rng.uniform(0.0, 2880.0, L)) for L in lens])
    for prec in ("fp64", "mixed"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        w = dev(rng.normal(size=(3, t.size))).to(dt)
        elem = dev(cat.elem).requires_grad_(True)
        r, v, _ = sg.SGP4RaggedFunction.apply(elem, dev(offsets), dev(t), prec)
        (r * w).sum().backward()
        g = sg.vjp_ragged(sg.init(dev(cat.elem)), dev(offsets), dev(t), w, None, prec)
        torch.cuda.synchronize()
        assert torch.equal(elem.grad[:7], g) and torch.all(elem.grad[7] == 0), prec
