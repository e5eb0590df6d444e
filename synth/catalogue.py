"""Synthetic Starlink-shaped catalogues.

The paper's workloads use the CelesTrak Starlink element sets of 13 January
2026 (9,341 satellites, section 3.1), a tiled catalogue of up to ~1.8 million
satellites (section 3.2) and 100 element sets propagated over two weeks
(section 4).  Those data are not available here, so every workload is a seeded
synthetic catalogue with the same shapes: near-circular LEO orbits at
Starlink shell inclinations and altitudes, lognormal B*, epochs spread over
+-3 days, 1-day and 7-day horizons.

Element rows (float64 [8, n]):
  0 no_kozai rad/min, 1 ecco, 2 inclo rad, 3 nodeo rad, 4 argpo rad, 5 mo rad,
  6 bstar 1/earth-radii, 7 epoch days after the reference instant.
Times are float64 minutes after the reference instant.

Streams: numpy PCG64 with independent children of SeedSequence(seed), one per
quantity, so changing one quantity's recipe does not shift the others.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Catalogue", "Ragged", "ELEMENT_ROWS", "config0", "config1", "config2", "config3", "config4",
    "uniform_elements", "shell_elements", "sample_satellites", "ragged_lists", "deep_elements", "config5",
    "DEEP_REF_JD",
]

ELEMENT_ROWS = ("no_kozai", "ecco", "inclo", "nodeo", "argpo", "mo", "bstar", "epoch")

# Kepler's third law is only used to turn a shell altitude into a plausible
# mean motion for synthetic inputs (WGS72 mu and equatorial radius).
_MU_KM3_S2 = 398600.8
_RE_KM = 6378.135

# (fraction, inclination deg, altitude km): Starlink-like shells.
SHELLS = ((0.40, 53.0, 550.0), (0.25, 53.2, 540.0), (0.15, 70.0, 570.0), (0.10, 97.6, 560.0), (0.10, 43.0, 530.0))


@dataclasses.dataclass
class Catalogue:
    elem: np.ndarray          # float64 [8, n]
    t: np.ndarray             # float64 [T] minutes after the reference
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.elem.shape[1])

    @property
    def T(self) -> int:
        return int(self.t.shape[0])


@dataclasses.dataclass
class Ragged:
    elem: np.ndarray          # float64 [8, n]
    offsets: np.ndarray       # int64 [n + 1], offsets[0] = 0, offsets[n] = nnz
    t: np.ndarray             # float64 [nnz] minutes after the reference, sorted within each list
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.elem.shape[1])

    @property
    def nnz(self) -> int:
        return int(self.t.shape[0])


def _streams(seed: int, k: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(k)]


def _angles_bstar(rng: np.random.Generator, n: int):
    node = rng.uniform(0.0, 2.0 * math.pi, n)
    argp = rng.uniform(0.0, 2.0 * math.pi, n)
    mo = rng.uniform(0.0, 2.0 * math.pi, n)
    ecc = rng.uniform(1e-5, 2e-3, n)
    bstar = 1e-4 * np.exp(rng.normal(0.0, 1.0, n))
    return node, argp, mo, ecc, bstar


def uniform_elements(n: int, seed: int) -> np.ndarray:
    """Mean motion U(14.8, 15.3) rev/day, inclination from {43, 53, 70, 97.6} deg, epoch 0."""
    r_el, r_inc, r_ang = _streams(seed, 3)
    revs = r_el.uniform(14.8, 15.3, n)
    inc = np.deg2rad(np.array([43.0, 53.0, 70.0, 97.6]))[r_inc.integers(0, 4, n)]
    node, argp, mo, ecc, bstar = _angles_bstar(r_ang, n)
    elem = np.empty((8, n))
    elem[0] = revs * 2.0 * math.pi / 1440.0
    elem[1] = ecc
    elem[2] = inc
    elem[3], elem[4], elem[5], elem[6] = node, argp, mo, bstar
    elem[7] = 0.0
    return elem


def shell_elements(n: int, seed: int, epoch_days: float = 3.0) -> np.ndarray:
    """Starlink-like shells (multinomial fractions), +-5 km altitude jitter, epochs U(-3, +3) days."""
    r_shell, r_alt, r_ang, r_ep = _streams(seed, 4)
    frac = np.array([s[0] for s in SHELLS])
    counts = r_shell.multinomial(n, frac)
    shell = np.repeat(np.arange(len(SHELLS)), counts)
    r_shell.shuffle(shell)
    inc = np.deg2rad(np.array([s[1] for s in SHELLS]))[shell]
    alt = np.array([s[2] for s in SHELLS])[shell] + r_alt.uniform(-5.0, 5.0, n)
    a_km = _RE_KM + alt
    n_rad_s = np.sqrt(_MU_KM3_S2 / a_km ** 3)
    node, argp, mo, ecc, bstar = _angles_bstar(r_ang, n)
    elem = np.empty((8, n))
    elem[0] = n_rad_s * 60.0
    elem[1] = ecc
    elem[2] = inc
    elem[3], elem[4], elem[5], elem[6] = node, argp, mo, bstar
    elem[7] = r_ep.uniform(-epoch_days, epoch_days, n)
    return elem


def config0() -> Catalogue:
    """64 satellites x 100 times over 0-1440 min (ends included), seed 0."""
    return Catalogue(uniform_elements(64, 0), np.linspace(0.0, 1440.0, 100), "c0: 64 x 100 FP64 smoke grid")


def config1(n: int = 9341, T: int = 1000) -> Catalogue:
    """9,341 Starlink-shaped satellites x 1,000 times over 0-1440 min, seed 1."""
    return Catalogue(shell_elements(n, 1), np.linspace(0.0, 1440.0, T), f"c1: {n} x {T} Starlink-shaped dense grid")


def config2(horizon: str = "1d", n: int = 100_000) -> Catalogue:
    """100k satellites; 1-day horizon at 1-min steps (1,440 times) or 7 days at 10-min steps (1,008)."""
    elem = shell_elements(n, 2)
    if horizon == "1d":
        t = np.arange(1440, dtype=np.float64)
    elif horizon == "7d":
        t = 10.0 * np.arange(1008, dtype=np.float64)
    else:
        raise ValueError(horizon)
    return Catalogue(elem, t, f"c2: {n} x {t.shape[0]} mega-constellation ({horizon})")


_CHUNK = 65536  # satellites per time-generation chunk (fixed: part of the recipe)


def ragged_lists(n: int, seed: int, median: float = 256.0, sigma: float = 1.0, max_len: int = 4096,
                 horizon_min: float = 10080.0):
    """Lognormal list lengths clip(round(median*exp(sigma*Z)), 1, max_len); times sorted U(0, horizon).

    Sorted uniforms per list are the normalised partial sums of L+1 standard
    exponentials (order statistics of the uniform distribution).  Generated in
    fixed chunks of satellites, each chunk with its own child stream, so memory
    stays bounded and the result does not depend on the machine.
    """
    ss_len, ss_t = np.random.SeedSequence(seed).spawn(2)
    r_len = np.random.Generator(np.random.PCG64(ss_len))
    lengths = np.clip(np.rint(median * np.exp(sigma * r_len.normal(0.0, 1.0, n))), 1, max_len).astype(np.int64)
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(lengths, out=offsets[1:])
    t = np.empty(int(offsets[-1]), np.float64)
    nchunks = (n + _CHUNK - 1) // _CHUNK
    for c, ss in zip(range(nchunks), ss_t.spawn(nchunks)):
        lo, hi = c * _CHUNK, min(n, (c + 1) * _CHUNK)
        L = lengths[lo:hi]
        m = hi - lo
        gaps = np.random.Generator(np.random.PCG64(ss)).standard_exponential(int(L.sum()) + m)
        csum = np.cumsum(gaps)
        starts = np.zeros(m, np.int64)
        np.cumsum(L[:-1] + 1, out=starts[1:])
        ends = starts + L                      # index of each list's closing gap
        base = np.where(starts > 0, csum[starts - 1], 0.0)
        total = csum[ends] - base
        keep = np.ones(csum.shape[0], bool)
        keep[ends] = False
        owner = np.repeat(np.arange(m), L)
        t[offsets[lo]:offsets[hi]] = (csum[keep] - base[owner]) / total[owner] * horizon_min
    return offsets, t


def config3(n: int = 1_000_000, high_drag_frac: float = 0.05) -> Ragged:
    """Ragged catalogue: lognormal list lengths (median 256, sigma 1, 1..4096), 7-day
    horizon, 5% of satellites with B* x 100, seed 3."""
    r_drag, = _streams(1003, 1)
    elem = shell_elements(n, 3)
    hot = r_drag.random(n) < high_drag_frac
    elem[6, hot] *= 100.0
    offsets, t = ragged_lists(n, 3)
    return Ragged(elem, offsets, t, f"c3: {n} satellites ragged, nnz={t.shape[0]}")


def config4(n: int = 9341, T: int = 1000):
    """Differentiation workload: config-1 elements theta, perturbed truth theta' =
    theta * (1 + 1e-5 z) on the seven differentiated rows, and 10 m position noise.
    Returns (catalogue, theta_true[8, n], noise_km[3, n, T])."""
    cat = config1(n, T)
    r_pert, r_noise = _streams(1004, 2)
    truth = cat.elem.copy()
    truth[:7] *= 1.0 + 1e-5 * r_pert.normal(0.0, 1.0, (7, n))
    noise = 0.01 * r_noise.normal(0.0, 1.0, (3, n, T))
    return Catalogue(cat.elem, cat.t, f"c4: {n} x {T} differentiation"), truth, noise


def sample_satellites(n: int, frac: float, seed: int) -> np.ndarray:
    """Seeded sorted sample of satellite indices (at least one)."""
    rng, = _streams(seed + 7919, 1)
    k = max(1, int(round(n * frac)))
    return np.sort(rng.choice(n, size=k, replace=False))


# Reference instant of the deep-space catalogue: 2026 January 13 0h UT (the
# date of the paper's element sets), as a Julian date.
DEEP_REF_JD = 2461053.5

# (fraction, semi-major axis km, eccentricity range, inclination deg range):
# navigation-constellation MEO, transfer orbits (low inclinations included, so
# that the deep-space model's low-inclination form is met), other non-resonant
# high orbits, and the two resonant classes of the deep-space model (24 h:
# near-geosynchronous; 12 h with e >= 0.5: Molniya-type).
DEEP_CLASSES = (
    (0.25, 26560.0, (0.0, 0.02), (54.0, 56.0)),      # GPS-like 12 h, e < 0.5: not resonant
    (0.15, 29600.0, (0.0, 0.01), (55.0, 57.0)),      # Galileo-like
    (0.10, 25510.0, (0.0, 0.01), (64.0, 65.6)),      # GLONASS-like
    (0.20, 24400.0, (0.70, 0.72), (0.5, 28.5)),      # transfer orbits, perigee 450-1050 km
    (0.15, 12500.0, (0.0, 0.3), (10.0, 120.0)),      # 232-min and longer periods
    (0.10, 42164.0, (0.0, 0.001), (0.0, 3.0)),       # near-geosynchronous: 24 h resonance
    (0.05, 26600.0, (0.68, 0.74), (62.0, 64.0)),     # Molniya-type: 12 h resonance
)


def deep_elements(n: int, seed: int, epoch_days: float = 3.0) -> np.ndarray:
    """Deep-space catalogue (periods of 225 min or more) by DEEP_CLASSES, B* =
    1e-5 exp(N(0, 1)), epochs U(-3, +3) days after DEEP_REF_JD."""
    r_cls, r_shape, r_ang, r_ep = _streams(seed, 4)
    frac = np.array([c[0] for c in DEEP_CLASSES])
    counts = r_cls.multinomial(n, frac / frac.sum())
    cls = np.repeat(np.arange(len(DEEP_CLASSES)), counts)
    r_cls.shuffle(cls)
    a_km = np.array([c[1] for c in DEEP_CLASSES])[cls] * (1.0 + r_shape.uniform(-0.002, 0.002, n))
    e_lo = np.array([c[2][0] for c in DEEP_CLASSES])[cls]
    e_hi = np.array([c[2][1] for c in DEEP_CLASSES])[cls]
    i_lo = np.array([c[3][0] for c in DEEP_CLASSES])[cls]
    i_hi = np.array([c[3][1] for c in DEEP_CLASSES])[cls]
    ecc = e_lo + (e_hi - e_lo) * r_shape.random(n)
    inc = np.deg2rad(i_lo + (i_hi - i_lo) * r_shape.random(n))
    node = r_ang.uniform(0.0, 2.0 * math.pi, n)
    argp = r_ang.uniform(0.0, 2.0 * math.pi, n)
    mo = r_ang.uniform(0.0, 2.0 * math.pi, n)
    bstar = 1e-5 * np.exp(r_ang.normal(0.0, 1.0, n))
    elem = np.empty((8, n))
    elem[0] = np.sqrt(_MU_KM3_S2 / a_km ** 3) * 60.0
    elem[1] = ecc
    elem[2] = inc
    elem[3], elem[4], elem[5], elem[6] = node, argp, mo, bstar
    elem[7] = r_ep.uniform(-epoch_days, epoch_days, n)
    return elem


def config5(n: int = 4096, T: int = 1008) -> Catalogue:
    """Deep-space catalogue, n satellites x T times at 10-minute steps over 7 days
    after the reference DEEP_REF_JD, seed 5."""
    return Catalogue(deep_elements(n, 5), 10.0 * np.arange(T), f"c5: {n} x {T} deep-space catalogue")
