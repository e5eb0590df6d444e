"""The oracle's pins must catch plausible mistakes.

Each mutant is the oracle source with one planted mistake (a dropped term, a
flipped sign, a wrong coefficient or power), built on the CPU into a temporary
library and run against the pin tests; at least one pin must fail.  Parts of the
model that no available pin can see are listed in the design notes as parity
unpinned (the J2 bracket of C4, the eccentricity factor of the drag node term,
the low-perigee density parameter and the model's switch thresholds).
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sgp4_oracle.cpp")

MUTANTS = [
    ("short-period radius coefficient", "0.5 * k1 * x1 * cos2u", "0.25 * k1 * x1 * cos2u"),
    ("short-period argument of latitude sign", "u - 0.25 * k2 * x7 * sin2u", "u + 0.25 * k2 * x7 * sin2u"),
    ("short-period node sign", "node + 1.5 * k2 * cosip * sin2u", "node - 1.5 * k2 * cosip * sin2u"),
    ("short-period inclination dropped", "incp + 1.5 * k2 * cosip * sinip * cos2u", "incp + 0.0 * k2"),
    ("short-period radial rate dropped", "rdot - n / g.ke * k1 * x1 * sin2u", "rdot - 0.0 * k1"),
    ("short-period transverse rate coefficient", "(x1 * cos2u + 1.5 * c41)", "(x1 * cos2u + 0.5 * c41)"),
    ("D3 coefficient", "(17.0 * c.a0pp + c.s)", "(16.0 * c.a0pp + c.s)"),
    ("D4 power of a0", "(2.0 / 3.0) * c.a0pp * c.a0pp * c.xi", "(2.0 / 3.0) * c.a0pp * c.xi"),
    ("t4cof coefficient", "12.0 * c.D2 + 10.0 * C1sq", "12.0 * c.D2 + 8.0 * C1sq"),
    ("Kepler residual sign", "(U - ayn * cp + axn * sp - psi)", "(U + ayn * cp + axn * sp - psi)"),
    ("velocity unit", "g->vkms = g->radius * g->ke / 60.0", "g->vkms = g->radius * g->ke / 61.0"),
    ("first-order node rate", "c.nodedot1 = -T1 * c.cosi", "c.nodedot1 = -0.9 * T1 * c.cosi"),
    ("un-Kozai coefficient", "0.75 * J2 * c.c41", "1.5 * J2 * c.c41"),
    ("J3 long-period eccentricity sign", "ayn = e * sin(argp) + tau * aycof;\n    LT = L +",
     "ayn = e * sin(argp) - tau * aycof;\n    LT = L +"),
    ("first-order mean-anomaly rate", "0.5 * T1 * c.beta0 * c.c41", "0.6 * T1 * c.beta0 * c.c41"),
    ("C2 eta-squared coefficient", "(1.0 + 1.5 * eta2 + e0eta", "(1.0 + 2.5 * eta2 + e0eta"),
    ("C4 first-order bracket", "e0 * (0.5 + 2.0 * eta2)", "e0 * (0.5 + 1.0 * eta2)"),
    ("C5 prefactor", "c.C5 = 2.0 * coef1", "c.C5 = 2.5 * coef1"),
    ("drag node coefficient", "c.nodecf = 3.5 * c.beta0sq", "c.nodecf = 3.0 * c.beta0sq"),
    ("J4 perigee polynomial", "T3 * (3.0 - 36.0 * th2 + 49.0 * th4)", "T3 * (3.0 - 36.0 * th2 + 48.0 * th4)"),
    ("J4 node polynomial", "2.0 * T3 * (3.0 - 7.0 * th2)", "2.0 * T3 * (3.0 - 6.0 * th2)"),
    ("J3 long-period longitude polynomial", "(3.0 + 5.0 * c.cosi) / den", "(3.0 + 4.0 * c.cosi) / den"),
    ("J3 long-period eccentricity coefficient", "c.aycof = -0.5 * j3oj2", "c.aycof = -0.45 * j3oj2"),
    ("eccentricity floor of code 1", "if (!(val(e) >= -0.001 && val(e) < 1.0)) return fail(1);",
     "if (!(val(e) >= -0.01 && val(e) < 1.0)) return fail(1);"),
    # J2^2 secular polynomials: each coefficient changed by about 10%
    ("J2^2 node coefficient", "(0.5 * T2 * (4.0 - 19.0 * th2)", "(0.5 * T2 * (4.0 - 17.0 * th2)"),
    ("J2^2 node constant", "(0.5 * T2 * (4.0 - 19.0 * th2)", "(0.5 * T2 * (3.6 - 19.0 * th2)"),
    ("J2^2 perigee quartic", "(7.0 - 114.0 * th2 + 395.0 * th4)", "(7.0 - 114.0 * th2 + 355.0 * th4)"),
    ("J2^2 perigee quadratic", "(7.0 - 114.0 * th2 + 395.0 * th4)", "(7.0 - 103.0 * th2 + 395.0 * th4)"),
    ("J2^2 perigee constant", "(7.0 - 114.0 * th2 + 395.0 * th4)", "(6.3 - 114.0 * th2 + 395.0 * th4)"),
    ("J2^2 mean-anomaly quartic", "(13.0 - 78.0 * th2 + 137.0 * th4)", "(13.0 - 78.0 * th2 + 123.0 * th4)"),
    ("J2^2 mean-anomaly quadratic", "(13.0 - 78.0 * th2 + 137.0 * th4)", "(13.0 - 70.0 * th2 + 137.0 * th4)"),
    ("J2^2 mean-anomaly constant", "(13.0 - 78.0 * th2 + 137.0 * th4)", "(11.7 - 78.0 * th2 + 137.0 * th4)"),
    ("J2^2 rate scale", "S T2 = 0.5 * T1 * J2 / p0sq;", "S T2 = 0.55 * T1 * J2 / p0sq;"),
    # the J2 term of C2
    ("C2 J2 coefficient", "0.375 * J2 * c.xi / q * c.c41", "0.34 * J2 * c.xi / q * c.c41"),
    ("C2 J2 eta polynomial", "(8.0 + 3.0 * eta2 * (8.0 + eta2))", "(8.0 + 2.0 * eta2 * (8.0 + eta2))"),
    # drag on the perigee and the mean anomaly
    ("C3 coefficient", "c.C3 = -2.0 * coef * c.xi", "c.C3 = -1.8 * coef * c.xi"),
    ("C3 inclination factor", "c.n0pp * c.sini / e0", "c.n0pp * c.cosi / e0"),
    ("C3 drag perigee phase", "c.argpcof = c.bstar * c.C3 * cos(c.argp0);",
     "c.argpcof = c.bstar * c.C3 * sin(c.argp0);"),
    ("Mcof coefficient", "-(2.0 / 3.0) * coef * c.bstar / e0eta", "-(0.6) * coef * c.bstar / e0eta"),
    ("Mcof eccentricity factor", "-(2.0 / 3.0) * coef * c.bstar / e0eta", "-(2.0 / 3.0) * coef * c.bstar / c.eta"),
    ("drag periodic power", "S dM = c.Mcof * (cube(1.0 + c.eta * cos(M_df)) - c.dM0);",
     "S dM = c.Mcof * (sq(1.0 + c.eta * cos(M_df)) - c.dM0);"),
    ("drag periodic epoch offset", "c.dM0 = cube(1.0 + c.eta * cos(c.M0));", "c.dM0 = cube(1.0 + c.eta * sin(c.M0));"),
    ("drag eccentricity epoch offset", "c.sinM0 = sin(c.M0);", "c.sinM0 = cos(c.M0);"),
    ("J3 drag term sign in M", "M = M_df + dargp + dM;", "M = M_df - dargp + dM;"),
    # deep space: lunar-solar constants, the averaged-quadrupole algebra, the
    # periodic and body-eccentricity coefficients, the low-inclination form
    ("lunar node rate sign", "4.5236020 - 9.2422029e-4 * day", "4.5236020 + 9.2422029e-4 * day"),
    ("lunar perigee epoch value", "5.8351514 + 0.0019443680 * day", "5.8351614 + 0.0019443680 * day"),
    ("Moon inclination constant", "kMoonCosI0 = 0.91375164", "kMoonCosI0 = 0.91385164"),
    ("solar strength", "{2.9864797e-6, 4.7968065e-7}", "{2.9964797e-6, 4.7968065e-7}"),
    ("quadrupole direction cosine sign", "const S a7 = -cg * sh + sg * ci * ch;", "const S a7 = cg * sh + sg * ci * ch;"),
    ("z31 coefficient", "b.z31 = 12.0 * x1 * x1 - 3.0 * x3 * x3;", "b.z31 = 11.0 * x1 * x1 - 3.0 * x3 * x3;"),
    ("z1 eccentricity-free term", "b.z1 = 2.0 * z1 + beta2 * b.z31;", "b.z1 = 2.0 * z1 + b.z31;"),
    ("s1 coefficient", "b.s1 = -15.0 * e * b.s4;", "b.s1 = -14.0 * e * b.s4;"),
    ("secular M constant", "(q.z1 + q.z3 - 14.0 - 6.0 * e2)", "(q.z1 + q.z3 - 13.0 - 6.0 * e2)"),
    ("secular node-in-perigee term", "c.dargpdt = dgh - cim * dh;", "c.dargpdt = dgh + cim * dh;"),
    ("periodic inclination coefficient", "c.pi3[k] = 2.0 * q.s2 * (q.z13 - q.z11);", "c.pi3[k] = 2.0 * q.s2 * (q.z13 + q.z11);"),
    ("body-eccentricity M term", "(-21.0 - 9.0 * e2) * kEBody[k]", "(-20.0 - 9.0 * e2) * kEBody[k]"),
    ("body-eccentricity perigee term", "c.pgh4[k] = -18.0 * q.s4 * kEBody[k];", "c.pgh4[k] = -16.0 * q.s4 * kEBody[k];"),
    ("low-inclination node component sign", "S alf = sinip * sno + (ph * cno + pinc * cosip * sno);",
     "S alf = sinip * sno + (ph * cno - pinc * cosip * sno);"),
    ("low-inclination longitude term", "(pl + pgh - pinc * node * sinip)", "(pl + pgh + pinc * node * sinip)"),
    ("24 h resonance band", "nv < 0.0052359877 && nv > 0.0034906585", "nv < 0.0052359877 && nv > 0.0044906585"),
    # resonance: inclination and eccentricity functions, the 24 h harmonics,
    # the 12 h arguments, the coefficients' k factor, epoch longitude and
    # rate, the integrator and the sidereal time
    ("F311 second term", "- 0.75 * (1.0 + ci);", "- 0.7 * (1.0 + ci);"),
    ("F442 coefficient", "F[kF442] = 39.375 * s2 * s2;", "F[kF442] = 38.375 * s2 * s2;"),
    ("F523 second coefficient", "6.56250012 * (1.0 + 2.0 * ci - 3.0 * c2)", "6.06250012 * (1.0 + 2.0 * ci - 3.0 * c2)"),
    ("F543 sign", "F[kF543] = 29.53125 * si * (-2.0", "F[kF543] = -29.53125 * si * (-2.0"),
    ("G300 quartic coefficient", "(-6.0 + 6.60937 * e2)", "(-6.0 + 5.60937 * e2)"),
    ("G200 quadratic coefficient", "(-2.5 + 0.8125 * e2)", "(-2.0 + 0.8125 * e2)"),
    ("G201 slope sign", "G[kG201] = -0.306 - (e - 0.64) * 0.440;", "G[kG201] = -0.306 + (e - 0.64) * 0.440;"),
    ("G422 fit coefficient", "- 1629.014 * e2", "- 1529.014 * e2"),
    ("G533 fit coefficient (e >= 0.7)", "+ 109377.94 * e3", "+ 109277.94 * e3"),
    ("24 h (3,1) phase", "{0, 1, 3, 0.13130908, 2.1460748e-6}", "{0, 1, 3, 0.23130908, 2.1460748e-6}"),
    ("24 h (2,2) magnitude", "{0, 2, 2, 2.0 * 2.8843198, 1.7891679e-6}", "{0, 2, 2, 2.0 * 2.8843198, 1.6891679e-6}"),
    ("24 h (3,3) phase", "{0, 3, 3, 3.0 * 0.37448087, 2.2123015e-7}", "{0, 3, 3, 3.0 * 0.47448087, 2.2123015e-7}"),
    ("12 h (3,2,2,2) perigee multiple", "{-1, 1, 3, 0.95240898", "{1, 1, 3, 0.95240898"),
    ("12 h (4,4,2,2) longitude multiple", "{0, 2, 4, 1.8014998", "{0, 1, 4, 1.8014998"),
    ("resonant coefficient k factor", "S coef = base * double(q.k) * q.J * FG;", "S coef = base * q.J * FG;"),
    ("24 h epoch longitude", "c.xlamo = mod2pi(c.M0 + c.node0 + c.argp0 - c.gsto);",
     "c.xlamo = mod2pi(c.M0 + c.node0 + c.argp0 + c.gsto);"),
    ("24 h longitude rate drops the bodies' M rate", "- kEarthRate + c.dMdt + c.dargpdt", "- kEarthRate + c.dargpdt"),
    ("12 h longitude rate", "2.0 * (c.nodedot + c.dnodedt - kEarthRate)", "2.0 * (c.nodedot - kEarthRate)"),
    ("integrator step's second-order term", "xni = xni + ndot * h + nddot * (0.5 * h * h);",
     "xni = xni + ndot * h + nddot * (h * h);"),
    ("integrator remainder's second-order term", "*xl = xli + ldot * ft + ndot * (0.5 * ft * ft);",
     "*xl = xli + ldot * ft + ndot * (0.4 * ft * ft);"),
    ("12 h perigee of the rates", "const S w = c.argp0 + c.argpdot * atime;", "const S w = c.argp0;"),
    ("sidereal time rate", "(876600.0 * 3600.0 + 8640184.812866) * T", "(876600.0 * 3600.0 + 8640194.812866) * T"),
    ("resonant mean anomaly, 12 h", "M = xl - 2.0 * node + 2.0 * theta;", "M = xl - 2.0 * node + theta;"),
]


def _run(mutant, workdir):
    name, old, new = mutant
    src = open(SRC).read()
    assert src.count(old) == 1, name
    cpp = os.path.join(workdir, "m.cpp")
    lib = os.path.join(workdir, "m.so")
    open(cpp, "w").write(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-pthread", "-o", lib, cpp],
                   check=True)
    env = dict(os.environ, SGP4_ORACLE_LIB=lib)
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_deep.py"),
                        os.path.join(ROOT, "tests", "test_oracle_resonance.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return name, p.returncode


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        dirs = []
        for k in range(len(MUTANTS)):
            d = os.path.join(tmp, str(k))
            os.makedirs(d)
            dirs.append(d)
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(_run, MUTANTS, dirs))
    survived = [name for name, rc in results if rc == 0]
    assert not survived, f"mutants not caught by any pin: {survived}"


def test_unmutated_source_passes():
    # guard: the harness itself must not report a failure for the real oracle
    with tempfile.TemporaryDirectory() as tmp:
        name, rc = _run(("identity", "int oracle_abi_version(void) { return 1; }",
                         "int oracle_abi_version(void) { return 1; }"), tmp)
    assert rc == 0
