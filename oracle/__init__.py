"""SGP4 near-Earth oracle: TEST INFRASTRUCTURE ONLY.

A plain serial FP64 CPU implementation (``sgp4_oracle.cpp``) of the model the
paper re-implements (section 2.1: SGP4 of Hoots & Roehrich 1980 / Hoots et al.
2004 / Vallado et al. 2006, WGS72 constants).  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It shares no
code with the GPU library, and the GPU library never calls it.

Array conventions (all numpy, C-contiguous):
  elem   float64 [8, n]: no_kozai (rad/min), ecco, inclo, nodeo, argpo, mo (rad),
         bstar (1/earth radii), epoch (days after the caller's reference)
  t      float64 minutes after the reference (time since epoch = t - 1440*epoch)
  r, v   float64 [3, P] km and km/s (TEME); err uint8 [P]
  grav   None (WGS72) or 5 floats {mu km^3/s^2, R km, J2, J3, J4}
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
ND = 35  # intermediate values per point (oracle_detail_count)
DETAIL_NAMES = [
    "M", "argp", "node", "a", "n", "e", "L", "axn", "ayn", "LT", "U", "psi", "iters", "resid",
    "ecE", "esE", "eL2", "pL", "r", "rdot", "rfdot", "betaL", "sinu", "cosu", "u",
    "k1", "k2", "rk", "uk", "nodek", "ik", "rdotk", "rfdotk", "code", "emargin",
]
INIT_NAMES = [
    "cosi", "sini", "beta0sq", "beta0", "c41", "x1", "x7", "n0pp", "a0pp", "rp", "hp", "s", "q4",
    "xi", "eta", "C1", "C2", "C3", "C4", "C5", "Mdot", "argpdot", "nodedot", "nodedot1",
    "argpcof", "Mcof", "nodecf", "t2cof", "aycof", "Lcof", "dM0", "sinM0",
    "D2", "D3", "D4", "t3cof", "t4cof", "t5cof", "isimp", "deep", "epoch_code", "ke", "j3oj2", "vkms",
    "resonant", "dedt", "didt", "dMdt", "dnodedt", "dargpdt", "Msun0", "Mmoon0",
] + [f"{name}_{body}" for body in ("sun", "moon")
     for name in ("pe2", "pe3", "pi2", "pi3", "pl2", "pl3", "pl4", "pgh2", "pgh3", "pgh4", "ph2", "ph3")] + [
    "irez", "xlamo", "xfact", "gsto"] + [f"res{k}" for k in range(10)]
RES_F = ["F311", "F220", "F330", "F221", "F321", "F322", "F441", "F442", "F522", "F523", "F542", "F543"]
RES_G = ["G310s", "G200", "G300", "G201", "G211", "G310", "G322", "G410", "G422", "G520", "G532", "G521", "G533"]
WGS72 = (398600.8, 6378.135, 0.001082616, -0.00000253881, -0.00000165597)

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    global _LIB
    if _LIB is None:
        # SGP4_ORACLE_LIB lets the mutation tests load a deliberately broken build.
        path = os.environ.get("SGP4_ORACLE_LIB", _build.LIB)
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.oracle_propagate.argtypes = [_dp, ctypes.c_int64, _dp, _dp, ctypes.c_int64, _dp, _dp, _u8p, ctypes.c_int]
        L.oracle_propagate_ragged.argtypes = [_dp, ctypes.c_int64, _dp, _i64p, _dp, ctypes.c_int64, _dp, _dp, _u8p,
                                              ctypes.c_int]
        L.oracle_codes_ragged.argtypes = [_dp, ctypes.c_int64, _dp, _i64p, _dp, ctypes.c_int64, _u8p, ctypes.c_int]
        L.oracle_propagate_points.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _i64p, _dp, _dp, _dp, _u8p, _dp]
        L.oracle_init.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
        L.oracle_jacobian_points.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _i64p, _dp, _dp, _dp, _dp, _u8p]
        L.oracle_vjp.argtypes = [_dp, ctypes.c_int64, _dp, _dp, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int]
        L.oracle_vjp_ragged.argtypes = [_dp, ctypes.c_int64, _dp, _i64p, _dp, ctypes.c_int64, _dp, _dp, _dp,
                                        ctypes.c_int]
        L.oracle_count_ops.argtypes = [_dp, _dp, ctypes.c_double, _u64p]
        L.oracle_set_reference_jd.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_reference_jd.restype = ctypes.c_double
        L.oracle_resonance_functions.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_resonance_constants.argtypes = [_dp]
        L.oracle_gmst.argtypes = [ctypes.c_double]
        L.oracle_gmst.restype = ctypes.c_double
        L.oracle_resonance_rates.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_resonance_integrate.argtypes = [_dp, _dp, ctypes.c_double, _dp]
        L.oracle_ke.argtypes = [_dp]
        L.oracle_ke.restype = ctypes.c_double
        assert L.oracle_detail_count() == ND
        assert L.oracle_init_count() == len(INIT_NAMES)
        _LIB = L
    return _LIB


def _p(a, typ=_dp):
    return None if a is None else a.ctypes.data_as(typ)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grav(grav):
    return None if grav is None else _f64(grav)


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle call failed with code {rc}")


def propagate(elem, t, grav=None, nthreads=1):
    """Dense grid: returns r[3, n, T], v[3, n, T], err[n, T]."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    n, T = elem.shape[1], t.shape[0]
    r = np.empty((3, n * T)); v = np.empty((3, n * T)); err = np.empty(n * T, np.uint8)
    _check(lib().oracle_propagate(_p(g), n, _p(elem), _p(t), T, _p(r), _p(v), _p(err, _u8p), int(nthreads)))
    return r.reshape(3, n, T), v.reshape(3, n, T), err.reshape(n, T)


def propagate_ragged(elem, offsets, t, grav=None, nthreads=1):
    """CSR lists: returns r[3, nnz], v[3, nnz], err[nnz]."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n, nnz = elem.shape[1], t.shape[0]
    r = np.empty((3, nnz)); v = np.empty((3, nnz)); err = np.empty(nnz, np.uint8)
    _check(lib().oracle_propagate_ragged(_p(g), n, _p(elem), _p(offsets, _i64p), _p(t), nnz, _p(r), _p(v),
                                         _p(err, _u8p), int(nthreads)))
    return r, v, err


def codes_ragged(elem, offsets, t, grav=None, nthreads=1):
    """CSR lists, codes only: err[nnz] (states computed and dropped)."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n, nnz = elem.shape[1], t.shape[0]
    err = np.empty(nnz, np.uint8)
    _check(lib().oracle_codes_ragged(_p(g), n, _p(elem), _p(offsets, _i64p), _p(t), nnz, _p(err, _u8p),
                                     int(nthreads)))
    return err


def propagate_points(elem, sat, t, grav=None, detail=False):
    """Individual points (sat[k], t[k]); returns r[3, K], v[3, K], err[K] (+ detail dict)."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    sat = np.ascontiguousarray(sat, dtype=np.int64)
    K = t.shape[0]
    r = np.empty((3, K)); v = np.empty((3, K)); err = np.empty(K, np.uint8)
    det = np.empty((K, ND)) if detail else None
    _check(lib().oracle_propagate_points(_p(g), elem.shape[1], _p(elem), K, _p(sat, _i64p), _p(t), _p(r), _p(v),
                                         _p(err, _u8p), _p(det)))
    if detail:
        return r, v, err, {name: det[:, k] for k, name in enumerate(DETAIL_NAMES)}
    return r, v, err


def init_constants(elem, grav=None):
    """Per-satellite initialisation constants as a dict of float64 [n] arrays."""
    elem = _f64(elem); g = _grav(grav)
    n = elem.shape[1]
    rec = np.empty((n, len(INIT_NAMES)))
    _check(lib().oracle_init(_p(g), n, _p(elem), _p(rec)))
    return {name: rec[:, k] for k, name in enumerate(INIT_NAMES)}


def jacobian_points(elem, sat, t, grav=None):
    """Dual-number Jacobian J[K, 6, 7] of (r, v) w.r.t. (n0, e0, i0, node0, argp0, M0, bstar)."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    sat = np.ascontiguousarray(sat, dtype=np.int64)
    K = t.shape[0]
    J = np.empty((K, 6, 7)); r = np.empty((3, K)); v = np.empty((3, K)); err = np.empty(K, np.uint8)
    _check(lib().oracle_jacobian_points(_p(g), elem.shape[1], _p(elem), K, _p(sat, _i64p), _p(t), _p(J), _p(r),
                                        _p(v), _p(err, _u8p)))
    return J, r, v, err


def vjp(elem, t, gr, gv=None, grav=None, nthreads=1):
    """Dual-number VJP over a dense grid: gelem[7, n]."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    n, T = elem.shape[1], t.shape[0]
    gr = _f64(gr).reshape(3, n * T)
    gv = None if gv is None else _f64(gv).reshape(3, n * T)
    out = np.empty((7, n))
    _check(lib().oracle_vjp(_p(g), n, _p(elem), _p(t), T, _p(gr), _p(gv), _p(out), int(nthreads)))
    return out


def vjp_ragged(elem, offsets, t, gr, gv=None, grav=None, nthreads=1):
    """Dual-number VJP over CSR time lists: gelem[7, n]; gr, gv [3, nnz]."""
    elem = _f64(elem); t = _f64(t); g = _grav(grav)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n, nnz = elem.shape[1], t.shape[0]
    gr = _f64(gr).reshape(3, nnz)
    gv = None if gv is None else _f64(gv).reshape(3, nnz)
    out = np.empty((7, n))
    _check(lib().oracle_vjp_ragged(_p(g), n, _p(elem), _p(offsets, _i64p), _p(t), nnz, _p(gr), _p(gv), _p(out),
                                   int(nthreads)))
    return out


def count_ops(elem1, tmin, grav=None):
    """Arithmetic performed by the definition for one point (init excluded)."""
    e = _f64(elem1); g = _grav(grav)
    out = np.zeros(8, np.uint64)
    lib().oracle_count_ops(_p(g), _p(e), float(tmin), _p(out, _u64p))
    keys = ["add", "mul", "div", "sqrt", "cbrt", "trig", "atan2", "floor"]
    return {k: int(x) for k, x in zip(keys, out)}


class reference_jd:
    """Context manager: the reference instant (Julian date, whole + fraction) of
    the elements' epoch row and the times while the block runs (the deep-space
    model's lunar and solar arguments need absolute time); J2000.0 otherwise."""

    def __init__(self, whole, frac=0.0):
        self.whole, self.frac = float(whole), float(frac)

    def __enter__(self):
        L = lib()
        self.saved = L.oracle_reference_jd()
        L.oracle_set_reference_jd(self.whole, self.frac)
        return self

    def __exit__(self, *exc):
        lib().oracle_set_reference_jd(self.saved, 0.0)
        return False


def ke(grav=None):
    g = _grav(grav)
    return lib().oracle_ke(_p(g))


def resonance_functions(e, inc):
    """The model's inclination and eccentricity functions of the resonant
    terms at (e, i): two dicts keyed by RES_F and RES_G names."""
    out = np.empty(len(RES_F) + len(RES_G))
    lib().oracle_resonance_functions(float(e), float(inc), _p(out))
    return dict(zip(RES_F, out[:len(RES_F)])), dict(zip(RES_G, out[len(RES_F):]))


def resonance_constants():
    """Earth rotation rate (rad/min), step (min), and the 24 h / 12 h term
    tables as lists of dicts (j, k, l, phase, J)."""
    out = np.empty(2 + 5 * 13)
    m = lib().oracle_resonance_constants(_p(out))
    assert m == out.size
    terms = [dict(zip(("j", "k", "l", "phase", "J"), out[2 + 5 * i:7 + 5 * i])) for i in range(13)]
    return float(out[0]), float(out[1]), terms[:3], terms[3:]


def gmst(jd):
    """Greenwich mean sidereal angle (rad) at Julian date jd (UT1)."""
    return lib().oracle_gmst(float(jd))


def resonance_rates(elem1, xli, xni, atime, grav=None):
    """(dn/dt, d2n/dt2, dlambda/dt) of one element set's resonance, and its class."""
    e = _f64(elem1).reshape(-1); g = _grav(grav)
    out = np.empty(3)
    cls = lib().oracle_resonance_rates(_p(g), _p(e), float(xli), float(xni), float(atime), _p(out))
    return out, cls


def resonance_integrate(elem1, t, grav=None):
    """(lambda, n, time of the last step) integrated to t minutes after epoch, and the class."""
    e = _f64(elem1).reshape(-1); g = _grav(grav)
    out = np.empty(3)
    cls = lib().oracle_resonance_integrate(_p(g), _p(e), float(t), _p(out))
    return out, cls
