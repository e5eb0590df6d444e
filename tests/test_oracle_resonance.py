"""Pins of the oracle's resonant deep-space terms (12 h and 24 h classes).

The resonance of the deep-space model (Hoots & Roehrich 1980, revised by
Vallado et al. 2006; the paper's section 6 names deep space as the variant it
leaves out) integrates the mean motion n and the resonant mean longitude
lambda under the tesseral harmonics J_lm of the geopotential.  Per term,
Lagrange's equation gives dn/dt = 3 n^2 (R/a)^l k F_lmp(i) G_lpq(e) J_lm sin psi
with psi = (l-2p) w + k M + m (node - theta) - m lambda_lm, k = l - 2p + q.
What pins the oracle's version, each against something other than itself:

* the inclination functions against Kaula's closed general formula (exact);
* the eccentricity functions against Hansen coefficients computed by
  quadrature: the 24 h series to their first dropped power of e, the 12 h
  polynomial fits to a few per cent over the Molniya range;
* the 24 h rates, harmonic by harmonic, against the along-track force of a
  published geopotential's (2,2), (3,1), (3,3) tesseral terms on a
  geostationary orbit, and the stable longitudes that force produces;
* the 12 h rates against the resonant arguments the tesseral terms select
  for an orbit at twice the Earth's rotation rate;
* the integrator against a fine numerical solution of its own equations,
  and its continuity across its 720-minute steps;
* the sidereal time against its J2000.0 value and rate;
* end to end, a geostationary satellite's Earth-fixed longitude: its drift
  rate and acceleration over 60 days.

The tesseral magnitudes and phases of degrees 3 to 5 of the 12 h class, the
720-minute step and the 12 h fits' eccentricity ranges are model definitions
(parity unpinned).
"""
import math

import numpy as np
from scipy.integrate import solve_ivp

import oracle

MU, RE = 398600.8, 6378.135
KE = 60.0 / math.sqrt(RE ** 3 / MU)


def elem(a_km, e, inc, node, argp, M, bstar=0.0, epoch=0.0):
    n = math.sqrt(MU / a_km ** 3) * 60.0
    return np.array([[n], [e], [inc], [node], [argp], [M], [bstar], [epoch]], dtype=np.float64)


def kaula_F(l, m, p, inc):
    """Kaula's inclination function F_lmp(i) (Kaula 1966, eq. 3.60), summed
    exactly as written."""
    k = (l - m) // 2
    ci, si = math.cos(inc), math.sin(inc)
    total = 0.0
    for t in range(0, min(p, k) + 1):
        a = math.factorial(2 * l - 2 * t) / (math.factorial(t) * math.factorial(l - t) *
                                             math.factorial(l - m - 2 * t) * 2 ** (2 * l - 2 * t))
        ssum = 0.0
        for s in range(0, m + 1):
            csum = 0
            for c in range(0, l - m - 2 * t + s + 1):
                d = p - t - c
                if 0 <= d <= m - s:
                    csum += math.comb(l - m - 2 * t + s, c) * math.comb(m - s, d) * (-1) ** (c - k)
            ssum += math.comb(m, s) * ci ** s * csum
        total += a * si ** (l - m - 2 * t) * ssum
    return total


def hansen_G(l, p, q, e, N=100000):
    """Eccentricity function G_lpq(e): the mean over the mean anomaly of
    (a/r)^(l+1) cos((l-2p) f - (l-2p+q) M) (midpoint rule, which converges
    geometrically for this smooth periodic integrand)."""
    M = (np.arange(N) + 0.5) * 2 * np.pi / N
    E = M + e * np.sin(M)
    for _ in range(50):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    f = 2 * np.arctan2(np.sqrt(1 + e) * np.sin(E / 2), np.sqrt(1 - e) * np.cos(E / 2))
    r = 1 - e * np.cos(E)
    return float(np.mean(r ** -(l + 1) * np.cos((l - 2 * p) * f - (l - 2 * p + q) * M)))


F_LMP = {"F311": (3, 1, 1), "F220": (2, 2, 0), "F330": (3, 3, 0), "F221": (2, 2, 1), "F321": (3, 2, 1),
         "F322": (3, 2, 2), "F441": (4, 4, 1), "F442": (4, 4, 2), "F522": (5, 2, 2), "F523": (5, 2, 3),
         "F542": (5, 4, 2), "F543": (5, 4, 3)}
# the 12 h terms as (l, m, p, q) in the oracle's order, with their F and G
TERMS12 = [((2, 2, 0, -1), "F220", "G201"), ((2, 2, 1, 1), "F221", "G211"), ((3, 2, 1, 0), "F321", "G310"),
           ((3, 2, 2, 2), "F322", "G322"), ((4, 4, 1, 0), "F441", "G410"), ((4, 4, 2, 2), "F442", "G422"),
           ((5, 2, 2, 0), "F522", "G520"), ((5, 2, 3, 2), "F523", "G532"), ((5, 4, 2, 1), "F542", "G521"),
           ((5, 4, 3, 3), "F543", "G533")]

# EGM96 (Lemoine et al. 1998), unnormalised tesseral coefficients C_lm, S_lm.
EGM96 = {(2, 2): (1.5744603e-6, -9.0380381e-7), (3, 1): (2.1926385e-6, 2.6842489e-7),
         (3, 3): (1.0038827e-7, 1.9722137e-7)}
# Geodesy Legendre functions at the equator (no Condon-Shortley phase).
P_LM_EQUATOR = {(2, 2): 3.0, (3, 1): -1.5, (3, 3): 15.0}


def iau82_gmst(jd):
    """Greenwich mean sidereal time, IAU 1982 (Aoki et al. 1982), radians."""
    T = (jd - 2451545.0) / 36525.0
    sec = 67310.54841 + (876600.0 * 3600.0 + 8640184.812866) * T + 0.093104 * T * T - 6.2e-6 * T ** 3
    return (sec % 86400.0) * (2 * math.pi / 86400.0)


def test_inclination_functions_are_kaulas():
    for inc in (0.0, 0.1, 0.7, 1.107, 1.5, 2.0, 2.9):
        F, _ = oracle.resonance_functions(0.6, inc)
        for name, (l, m, p) in F_LMP.items():
            want = kaula_F(l, m, p, inc)
            # the model prints 1/3 (times coefficients up to ~80) and two
            # coefficients to 8-9 digits
            assert abs(F[name] - want) <= 5e-7 * max(abs(want), 1.0), (name, inc, F[name], want)


def test_24h_eccentricity_functions_are_the_series_of_the_hansen_coefficients():
    """G310 = 1 + 2 e^2 (next term -239/64 e^4), G200 to e^4 (next ~0.12 e^6),
    G300 to e^4 (next ~1.9 e^6): each within its first dropped power."""
    for e in (0.01, 0.05, 0.1, 0.15, 0.2):
        _, G = oracle.resonance_functions(e, 0.3)
        assert abs(G["G310s"] - hansen_G(3, 1, 0, e)) <= 4.5 * e ** 4, e
        assert abs(G["G200"] - hansen_G(2, 0, 0, e)) <= 0.2 * e ** 6, e
        assert abs(G["G300"] - hansen_G(3, 0, 0, e)) <= 2.5 * e ** 6, e


def test_12h_eccentricity_fits_follow_the_hansen_coefficients():
    """The model's polynomial fits against quadrature over the eccentricities
    of 12-hour resonant orbits: within 6% (the fits' own accuracy)."""
    for e in np.linspace(0.55, 0.75, 9):
        _, G = oracle.resonance_functions(e, 0.3)
        for (l, m, p, q), _, gname in TERMS12:
            want = hansen_G(l, p, q, e)
            assert abs(G[gname] - want) <= 0.06 * max(abs(want), 0.3), (gname, e, G[gname], want)


def _geo(lon0_deg=0.0, e=1e-4, inc=0.0):
    el = elem(42164.2, e, inc, 0.0, 0.0, 0.0)
    gsto = oracle.gmst(2451545.0)  # epoch row 0 at the default reference, J2000.0
    el[5, 0] = (math.radians(lon0_deg) + gsto) % (2 * math.pi)
    return el


def test_24h_rates_are_the_tesseral_force_on_a_geostationary_orbit():
    """For a circular equatorial orbit the (l, m) tesseral term's along-track
    force gives dn/dt = 3 n^2 (R/a)^l m P_lm(0) J_lm sin(m (lambda - lambda_lm)).
    Harmonic by harmonic, the oracle's dn/dt(lambda) must match that force
    computed from EGM96 (the model's older field differs by a few per cent)."""
    el = _geo()
    c = oracle.init_constants(el)
    assert c["irez"][0] == 1
    n = c["n0pp"][0]
    ra = (n / KE) ** (2.0 / 3.0)
    N = 64
    lam = 2 * np.pi * np.arange(N) / N
    nd = np.array([oracle.resonance_rates(el[:, 0], x, n, 0.0)[0][0] for x in lam])
    X = np.fft.fft(nd) / N
    for (l, m), (C, S) in EGM96.items():
        J, lam_lm = math.hypot(C, S), math.atan2(S, C) / m
        amp = 3.0 * n * n * ra ** l * m * P_LM_EQUATOR[(l, m)] * J
        # A sin(m lambda - phi) has the m-th Fourier coefficient (A / 2i) exp(-i phi)
        want = amp / 2j * np.exp(-1j * m * lam_lm)
        got = X[m]
        assert abs(got - want) <= 0.05 * abs(want), ((l, m), got, want)
    # no other harmonics
    assert np.max(np.abs(X[4:N // 2])) < 1e-6 * np.max(np.abs(X))


def test_24h_stable_longitudes():
    """Geostationary satellites drift toward the stable points of the
    tesseral field, near 75 E and 255 E (dn/dt = 0 with negative slope)."""
    el = _geo()
    n = oracle.init_constants(el)["n0pp"][0]
    lam = np.radians(np.arange(0.0, 360.0, 0.05))
    nd = np.array([oracle.resonance_rates(el[:, 0], x, n, 0.0)[0][0] for x in lam])
    down = np.where((nd[:-1] > 0) & (nd[1:] <= 0))[0]
    stable = sorted(np.degrees(lam[down]))
    assert len(stable) == 2
    assert abs(stable[0] - 75.1) < 1.5 and abs(stable[1] - 255.1) < 2.0, stable


def test_12h_rates_follow_the_resonant_arguments():
    """At twice the Earth's rotation rate the terms that stay resonant are those
    with k = l - 2p + q = m / 2; their arguments in the model's variables are
    (l - 2p) w + k lambda - m lambda_lm, lambda = M + 2 node - 2 theta.  The
    oracle's dn/dt and d2n/dt2 must be the sum of 3 n^2 (R/a)^l k F G J sin psi
    over the ten terms, with Kaula's F."""
    rate, step, t24, t12 = oracle.resonance_constants()
    assert step == 720.0
    # the (2, 2) harmonic is the same in both classes: magnitude and phase m lambda_22
    assert t12[0]["J"] == t12[1]["J"] == t24[1]["J"]
    assert abs(math.remainder(t12[0]["phase"] - t24[1]["phase"], 2 * math.pi)) < 1e-15
    assert abs(math.remainder(t12[1]["phase"] - t24[1]["phase"], 2 * math.pi)) < 1e-15
    for inc, e in ((1.107, 0.72), (0.9, 0.6), (1.3, 0.68)):
        el = elem(26600.0, e, inc, 0.7, 1.3, 0.2)
        c = oracle.init_constants(el)
        assert c["irez"][0] == 2
        n = c["n0pp"][0]
        ra = (n / KE) ** (2.0 / 3.0)
        _, G = oracle.resonance_functions(e, inc)
        rng = np.random.default_rng(7)
        for xli, xni, atime in zip(rng.uniform(0, 2 * np.pi, 5), n * (1 + rng.uniform(-1e-4, 1e-4, 5)),
                                   rng.uniform(-5000, 5000, 5)):
            w = 1.3 + c["argpdot"][0] * atime
            nd = ndd = 0.0
            for ((l, m, p, q), fname, gname), term in zip(TERMS12, t12):
                j, k = l - 2 * p, l - 2 * p + q
                assert k * 2 == m and term["j"] == j and term["k"] == k and term["l"] == l
                coef = 3.0 * n * n * ra ** l * k * kaula_F(l, m, p, inc) * G[gname] * term["J"]
                psi = j * w + k * xli - term["phase"]
                nd += coef * math.sin(psi)
                ndd += k * coef * math.cos(psi)
            out, cls = oracle.resonance_rates(el[:, 0], xli, xni, atime)
            ldot = xni + c["xfact"][0]
            assert cls == 2 and out[2] == ldot
            scale = sum(abs(3.0 * n * n * ra ** t[0][0] * t[0][1] // 2) for t in TERMS12) * 1e-6
            assert abs(out[0] - nd) <= 1e-7 * abs(nd) + 1e-22, (out[0], nd)
            assert abs(out[1] - ndd * ldot) <= 1e-7 * abs(ndd * ldot) + 1e-28, (out[1], ndd * ldot)


def test_resonant_longitude_rate_at_epoch_is_the_sum_of_the_secular_rates():
    """dlambda/dt at epoch (n + xfact) is the rate of the resonant argument:
    24 h M + w + node - theta, 12 h M + 2 node - 2 theta, each angle at its
    secular rate (gravity and bodies) and theta at the sidereal rate."""
    rate = oracle.resonance_constants()[0]
    sidereal = (iau82_gmst(2451546.0) - iau82_gmst(2451545.0)) % (2 * math.pi) / 1440.0 + 2 * math.pi / 1440.0
    assert abs(rate / sidereal - 1.0) < 1e-6
    for el in (_geo(30.0), elem(26600.0, 0.72, 1.107, 0.7, 1.3, 0.2)):
        c = {k: v[0] for k, v in oracle.init_constants(el).items()}
        out, cls = oracle.resonance_rates(el[:, 0], c["xlamo"], c["n0pp"], 0.0)
        dM, dw, dO = c["Mdot"] + c["dMdt"], c["argpdot"] + c["dargpdt"], c["nodedot"] + c["dnodedt"]
        want = dM + dw + dO - rate if cls == 1 else dM + 2 * (dO - rate)
        assert abs(out[2] - want) < 1e-12, (cls, out[2], want)


def test_sidereal_time_epoch_value_and_rate():
    # 18h 41m 50.54841s at J2000.0 (the 1982 definition), and 360.9856473... deg/day
    assert abs(math.degrees(oracle.gmst(2451545.0)) - 280.46061837504) < 1e-8
    d = (oracle.gmst(2451545.0 + 100.0) - oracle.gmst(2451545.0)) % (2 * math.pi)
    assert abs(math.degrees(d) - (100 * 360.98564736629) % 360.0) < 1e-5
    for jd in (2440000.5, 2451545.0, 2460000.25):
        assert abs(math.remainder(oracle.gmst(jd) - iau82_gmst(jd), 2 * math.pi)) < 1e-12


def test_integrator_matches_a_fine_solution_of_its_equations():
    """720-minute second-order Taylor steps against DOP853 on
    dlambda/dt = n + xfact, dn/dt = ndot(lambda, t): the difference is a small
    fraction of the resonance's own effect (truncation of the steps)."""
    for el in (_geo(30.0), elem(26600.0, 0.72, 1.107, 0.7, 1.3, 0.2)):
        c = oracle.init_constants(el)
        x0, n0, xf = c["xlamo"][0], c["n0pp"][0], c["xfact"][0]
        for T in (700.0, 1000.0, -3000.0, 10080.0, 43200.0):
            (xl, nm, at), cls = oracle.resonance_integrate(el[:, 0], T)
            assert at == 720.0 * math.trunc(T / 720.0)

            def f(t, y):
                out, _ = oracle.resonance_rates(el[:, 0], y[0], y[1], t)
                return [out[2], out[0]]

            sol = solve_ivp(f, (0.0, T), [x0, n0], method="DOP853", rtol=1e-13, atol=1e-16)
            l_ref, n_ref = sol.y[0, -1], sol.y[1, -1]
            dl_res = abs(l_ref - (x0 + (n0 + xf) * T))   # what the resonance changes
            dn_res = abs(n_ref - n0)
            assert dl_res > 1e-7 and dn_res > 1e-9
            assert abs(xl - l_ref) <= 2e-3 * dl_res, (cls, T, xl - l_ref, dl_res)
            assert abs(nm - n_ref) <= 2e-3 * dn_res, (cls, T, nm - n_ref, dn_res)


def test_states_continuous_across_integrator_steps():
    for el in (_geo(30.0), elem(26600.0, 0.72, 1.107, 0.7, 1.3, 0.2)):
        for tb in (720.0, 1440.0, 5040.0, -720.0, -2160.0):
            dt = 1e-3
            t = np.array([tb - dt, tb, tb + dt])
            r, v, err = oracle.propagate(el, t)
            assert np.all(err == 0)
            r = r[:, 0, :]; v = v[:, 0, :]
            # second difference of a smooth path: |r(t-) - 2 r(t) + r(t+)| = |a| (60 dt)^2,
            # |a| the two-body acceleration to within J2 and the bodies
            acc = MU / np.dot(r[:, 1], r[:, 1])
            jump = np.linalg.norm(r[:, 0] - 2 * r[:, 1] + r[:, 2])
            assert abs(jump - acc * (60 * dt) ** 2) < 0.01 * acc * (60 * dt) ** 2, (tb, jump)


def test_geostationary_longitude_drift_end_to_end():
    """A geostationary satellite at 30 E over 60 days.  Its mean Earth-fixed
    longitude (the mean longitude M + w + node less the sidereal time),
    fitted by a quartic in time (the acceleration changes as the satellite
    drifts), accelerates at epoch as the tesseral force at that longitude says
    (EGM96 (2,2), (3,1), (3,3)) and drifts at the rate the secular rates give;
    the longitude of the TEME position follows it to within the lunar-solar
    periodic terms."""
    el = _geo(30.0)
    c = {k: v[0] for k, v in oracle.init_constants(el).items()}
    days = np.arange(0.0, 61.0)
    gmst = np.array([iau82_gmst(2451545.0 + d) for d in days])
    r, _, err, det = oracle.propagate_points(el, np.zeros(days.size, np.int64), 1440.0 * days, detail=True)
    assert np.all(err == 0)
    lon = np.unwrap(det["L"] - gmst)
    true_lon = np.unwrap(np.arctan2(r[1], r[0]) - gmst)
    assert np.max(np.abs(np.remainder(true_lon - lon + np.pi, 2 * np.pi) - np.pi)) < 2e-3
    c4, c3, c2, c1, c0 = np.polyfit(days, lon, 4)
    n = c["n0pp"]
    ra = (n / KE) ** (2.0 / 3.0)

    def ndot(x):
        tot = 0.0
        for (l, m), (C, S) in EGM96.items():
            J, lam_lm = math.hypot(C, S), math.atan2(S, C) / m
            tot += 3.0 * n * n * ra ** l * m * P_LM_EQUATOR[(l, m)] * J * np.sin(m * (x - lam_lm))
        return tot

    want_acc = float(ndot(lon[0])) * 1440.0 ** 2   # rad/day^2 at epoch
    assert abs(2 * c2 - want_acc) <= 0.06 * abs(want_acc), (2 * c2, want_acc)
    sidereal = 2 * math.pi * 1.002737909350795  # rad/day, the IAU 1982 rate at J2000.0
    want_rate = (c["Mdot"] + c["dMdt"] + c["argpdot"] + c["dargpdt"] + c["nodedot"] + c["dnodedt"]) * 1440.0 - sidereal
    assert abs(c1 - want_rate) < 2e-6, (c1, want_rate)   # rad/day
    assert abs(math.degrees(c0) - 30.0) < 1e-3
