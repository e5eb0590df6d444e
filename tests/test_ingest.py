"""Ingestion: the oracle's element-set parser pinned to what the formats fix,
and the library's native parser (sgp4_text_count / sgp4_text_parse, host
code, no GPU) against the oracle record by record.

Bar: catalogue numbers and status bits identical; elements bit-identical
(both sides convert the same decimal text with one correct rounding and apply
the same unit conversions), NaN in the same places.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import paper_2603_27830_amd as sg
import synth
from oracle import ingest as oi
from synth import text as st


def _tle(l1_68: str, l2_68: str):
    return l1_68 + str(oi.checksum(l1_68 + "0")), l2_68 + str(oi.checksum(l2_68 + "0"))


# A pair written field by field from the column layout: catalogue 12345,
# epoch 2024 day 61.75 (2024 is a leap year: day 61 is March 1), B* =
# 0.12345e-3, inclination 53 deg, node 120.5 deg, e = 0.0001234, perigee
# 90 deg, mean anomaly 270 deg, 15.1 rev/day.
L1 = "1 12345U 24001A   24061.75000000  .00001234  00000-0  12345-3 0  999"
L2 = "2 12345  53.0000 120.5000 0001234  90.0000 270.0000 15.10000000  777"


# ------------------------------------------------------------ oracle pins --
def test_julian_dates_of_textbook_instants():
    assert oi.jd0(2000, 1, 1) + 0.5 == 2451545.0          # J2000.0 is 2000-01-01 12:00
    assert oi.jd0(1858, 11, 17) == 2400000.5              # origin of the modified Julian date
    assert oi.jd0(1957, 10, 4) == 2436115.5
    assert oi.jd0(2024, 3, 1) - oi.jd0(2024, 2, 28) == 2  # leap day
    assert oi.jd0(2100, 3, 1) - oi.jd0(2100, 2, 28) == 1  # century rule


def test_checksum_definition():
    l1, l2 = _tle(L1, L2)
    assert len(l1) == 69 and len(l2) == 69
    # brute force of the definition on a short string: digits sum, '-' counts one
    assert oi.checksum("1-2-3" + " " * 63) == (1 + 1 + 2 + 1 + 3) % 10
    _, _, s = oi.parse_tle(l1 + "\n" + l2 + "\n")
    assert s[0] == 0
    bad = l1[:30] + str((int(l1[30]) + 1) % 10) + l1[31:]
    _, _, s = oi.parse_tle(bad + "\n" + l2 + "\n")
    assert s[0] == oi.CHECKSUM


def test_hand_written_pair_fields():
    l1, l2 = _tle(L1, L2)
    el, sat, stat = oi.parse_tle("A NAME LINE\n" + l1 + "\n" + l2 + "\n", ref=(oi.jd0(2024, 1, 1), 0.0))
    assert sat[0] == 12345 and stat[0] == 0
    e = el[:, 0]
    assert e[0] == 15.1 / (1440.0 / (2 * math.pi))
    assert e[1] == 0.0001234
    assert e[2] == 53.0 * math.pi / 180 and e[3] == 120.5 * math.pi / 180
    assert e[4] == math.pi / 2 and e[5] == 270.0 * math.pi / 180
    assert e[6] == 0.12345e-3
    assert e[7] == 60.75                                   # day 61.75 is 60.75 days after January 1, 0h


def test_year_pivot_and_alpha5_numbers():
    assert oi.satnum("A0000") == 100000
    assert oi.satnum("H9999") == 179999
    assert oi.satnum("J0000") == 180000                    # I is skipped
    assert oi.satnum("P0000") == 230000                    # O is skipped
    assert oi.satnum("Z9999") == 339999
    assert oi.satnum("I0000") is None and oi.satnum("O1234") is None
    for yy, year in (("57", 1957), ("99", 1999), ("00", 2000), ("56", 2056)):
        l1 = L1[:18] + yy + "001.00000000" + L1[32:]
        el, _, _ = oi.parse_tle("\n".join(_tle(l1, L2)) + "\n", ref=(oi.jd0(year, 1, 1), 0.0))
        assert el[7, 0] == 0.0, yy


def test_assumed_decimal_fields():
    assert oi.assumed_decimal(" 12345-3") == 0.12345e-3
    assert oi.assumed_decimal("-11606-4") == -0.11606e-4
    assert oi.assumed_decimal(" 00000-0") == 0.0
    assert oi.assumed_decimal(" 10000+1") == 1.0
    assert oi.assumed_decimal("  1-x") is None


def test_day_fraction_is_the_correctly_rounded_digit_string():
    digits = "51782528"
    l1 = L1[:18] + "08264." + digits + L1[32:]
    el, _, _ = oi.parse_tle("\n".join(_tle(l1, L2)) + "\n", ref=(oi.jd0(2008, 1, 1), 0.0))
    exact = 263 + oi.exact_day_fraction(digits)
    assert abs(Fraction(el[7, 0]) - exact) <= Fraction(1, 2 ** 44)   # half an ulp of a 263-day value
    assert float(oi.exact_day_fraction(digits)) == float("0." + digits)


def test_iso_epochs():
    base = oi.jd0(2025, 3, 4)
    assert oi.parse_iso("2025-03-04T12:00:00") == (base, 0.5)
    assert oi.parse_iso("2025-03-04T06:00:00.000Z") == (base, 0.25)
    assert oi.parse_iso("2025-063T18:00:00") == (base, 0.75)        # day of year 63 of 2025 is March 4
    w, f = oi.parse_iso("2025-03-04T00:00:00.000000001")
    assert w == base and f == 1 / 86400e9
    assert oi.parse_iso("2025-02-29T00:00:00") is None
    assert oi.parse_iso("2025-03-04 12:00:00") is None


def test_round_trip_through_written_text():
    """Elements written by the synthetic writer parse back to within the
    printed precision (4 decimals of a degree, 8 of a rev/day, 7 of e, 5
    significant digits of B*, 1e-8 day)."""
    elem = synth.shell_elements(400, 11)
    for fmt, text in (("tle", st.tle_text(elem, three_line=True)), ("kvn", st.omm_kvn(elem)),
                      ("csv", st.omm_csv(elem)), ("json", st.omm_json(elem))):
        if fmt == "tle":
            el, sat, stat = oi.parse_tle(text, ref=st.REF_JD)
        else:
            el, sat, stat = oi.parse_omm(text, fmt, ref=st.REF_JD)
        assert el.shape == (8, 400) and np.all(stat == 0), fmt
        assert np.all(sat == np.arange(1, 401)), fmt
        mm = lambda x: x * 1440 / (2 * np.pi)  # noqa: E731
        assert np.max(np.abs(mm(el[0]) - mm(elem[0]))) <= 0.51e-8, fmt
        assert np.max(np.abs(el[1] - elem[1])) <= 0.51e-7, fmt
        assert np.max(np.abs(np.degrees(el[2]) - np.degrees(elem[2]))) <= 0.51e-4, fmt
        ang = lambda a, b: np.abs((np.degrees(a) - np.degrees(b) + 180.0) % 360.0 - 180.0)  # noqa: E731
        for k in (3, 4, 5):
            assert np.max(ang(el[k], elem[k])) <= 0.51e-4, (fmt, k)
        assert np.max(np.abs(el[6] - elem[6]) / np.abs(elem[6])) <= 0.51e-4, fmt
        # printed resolution, plus the writer's own rounding of the Julian date (ulp 4.7e-10 day)
        assert np.max(np.abs(el[7] - elem[7])) <= (0.5e-8 if fmt == "tle" else 0.5e-6 / 86400) + 1e-9, fmt


def test_corrupted_records_flagged():
    elem = synth.shell_elements(300, 12)
    lines = st.corrupt_tle(st.tle_lines(elem), np.random.default_rng(4), frac=0.3)
    text = "\n".join(x for _, a, b in lines for x in (a, b)) + "\n"
    el, sat, stat = oi.parse_tle(text)
    assert np.any(stat & oi.CHECKSUM) and np.any(stat & oi.MISMATCH) and np.any(stat & oi.FIELD)
    assert np.all(np.isnan(el[:, (stat & oi.FIELD) != 0]))
    assert not np.any(np.isnan(el[:, (stat & oi.FIELD) == 0]))


# ----------------------------------------------- native parser vs oracle --
def _same(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return a.shape == b.shape and np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(
        a[~np.isnan(a)], b[~np.isnan(b)])


def _check(text, fmt, ref=None):
    ref_o = oi.J2000 if ref is None else ref
    if fmt == "tle":
        eo, so, to = oi.parse_tle(text, ref=ref_o)
    else:
        eo, so, to = oi.parse_omm(text, fmt[4:], ref=ref_o)
    e, s, t = sg.parse_text(text, fmt, ref_jd=ref, threads=4)
    assert _same(e, eo), fmt
    assert np.array_equal(s, so) and np.array_equal(t, to), fmt
    return e


@pytest.mark.parametrize("three_line,crlf", [(False, False), (True, False), (True, True)])
def test_native_tle_matches_oracle(three_line, crlf):
    elem = synth.shell_elements(3000, 21)
    sat = np.random.default_rng(2).integers(1, 340000, 3000)   # five-digit and alpha-5 numbers
    text = st.tle_text(elem, satnums=sat, three_line=three_line, crlf=crlf)
    e = _check(text, "tle", ref=st.REF_JD)
    assert np.all(np.isfinite(e))
    _check(text, "tle")                                        # default reference J2000


def test_native_tle_corrupted_records_match_oracle():
    elem = synth.shell_elements(2000, 22)
    lines = st.corrupt_tle(st.tle_lines(elem), np.random.default_rng(5), frac=0.3)
    text = "junk line\n" + "\n".join(x for _, a, b in lines for x in (a, b)) + "\n1 short line\n"
    _check(text, "tle", ref=st.REF_JD)


def test_native_tle_large_text_uses_threads_and_keeps_order():
    """Over the multi-threaded size (several MB of text): same records, same
    order, as a single-threaded parse and the oracle."""
    elem = synth.shell_elements(40000, 23)
    text = st.tle_text(elem, three_line=True)
    assert len(text) > 4 << 20
    e1, s1, t1 = sg.parse_text(text, "tle", ref_jd=st.REF_JD, threads=1)
    e8, s8, t8 = sg.parse_text(text, "tle", ref_jd=st.REF_JD, threads=8)
    assert _same(e1, e8) and np.array_equal(s1, s8) and np.array_equal(t1, t8)
    eo, so, to = oi.parse_tle(text, ref=st.REF_JD)
    assert _same(e8, eo) and np.array_equal(s8, so)


@pytest.mark.parametrize("fmt", ["omm_kvn", "omm_csv", "omm_json"])
def test_native_omm_matches_oracle(fmt):
    elem = synth.shell_elements(1500, 24)
    writer = {"omm_kvn": st.omm_kvn, "omm_csv": st.omm_csv, "omm_json": st.omm_json}[fmt]
    e = _check(writer(elem), fmt, ref=st.REF_JD)
    assert np.all(np.isfinite(e))


def test_native_omm_missing_and_bad_fields():
    text = ("CCSDS_OMM_VERS = 2.0\nEPOCH = 2025-01-02T03:04:05.5\nMEAN_MOTION = 15.2\nECCENTRICITY = 0.001\n"
            "INCLINATION = 53\nRA_OF_ASC_NODE = 10\nARG_OF_PERICENTER = 20\nMEAN_ANOMALY = 30\nBSTAR = 1e-4\n"
            "NORAD_CAT_ID = 77\n"
            "CCSDS_OMM_VERS = 2.0\nEPOCH = 2025-02-30T00:00:00\nMEAN_MOTION = 15.2\nECCENTRICITY = 0.001\n"
            "INCLINATION = 53\nRA_OF_ASC_NODE = 10\nARG_OF_PERICENTER = 20\nMEAN_ANOMALY = 30\nBSTAR = 1e-4\n"
            "CCSDS_OMM_VERS = 2.0\nEPOCH = 2025-001T00:00:00Z\nMEAN_MOTION = fast\nECCENTRICITY = 0.001\n"
            "INCLINATION = 53\nRA_OF_ASC_NODE = 10\nARG_OF_PERICENTER = 20\nMEAN_ANOMALY = 30\nBSTAR = 1e-4\n"
            "CCSDS_OMM_VERS = 2.0\nEPOCH = 2025-001T00:00:00Z\nMEAN_MOTION = 15\nECCENTRICITY = 0.001\n"
            "INCLINATION = 53\nRA_OF_ASC_NODE = 10\nARG_OF_PERICENTER = 20\nMEAN_ANOMALY = 30\n")
    e = _check(text, "omm_kvn")
    _, s, t = sg.parse_text(text, "omm_kvn")
    assert list(t) == [0, 4, 4, 4] and list(s) == [77, -1, -1, -1]
    assert np.all(np.isfinite(e[:, 0])) and np.all(np.isnan(e[:, 1:]))


def test_native_parser_argument_errors():
    from paper_2603_27830_amd import _native
    L = _native.lib()
    E = {v: k for k, v in _native.ERRORS.items()}
    import ctypes
    n = ctypes.c_int64(-5)
    assert L.sgp4_text_count(b"", 0, 1, ctypes.byref(n)) == 0 and n.value == 0
    assert L.sgp4_text_count(b"x", 1, 9, ctypes.byref(n)) == E["SGP4_E_ARG"]
    assert L.sgp4_text_count(b"x", 1, 1, None) == E["SGP4_E_ARG"]
    assert L.sgp4_text_count(b"[1,2]", 5, 4, ctypes.byref(n)) == E["SGP4_E_ARG"]
    buf = (ctypes.c_double * 8)()
    l1, l2 = _tle(L1, L2)
    txt = (l1 + "\n" + l2 + "\n").encode()
    assert L.sgp4_text_parse(txt, len(txt), 1, 2, None, buf, None, None, 1) == E["SGP4_E_SIZE"]
    assert L.sgp4_text_parse(txt, len(txt), 1, -1, None, buf, None, None, 1) == E["SGP4_E_SIZE"]
    assert L.sgp4_text_parse(txt, len(txt), 1, 1, None, None, None, None, 1) == E["SGP4_E_ARG"]
    bad_ref = (ctypes.c_double * 2)(float("nan"), 0.0)
    assert L.sgp4_text_parse(txt, len(txt), 1, 1, bad_ref, buf, None, None, 1) == E["SGP4_E_ARG"]
    assert L.sgp4_text_parse(txt, len(txt), 1, 1, None, buf, None, None, 1) == 0
    assert buf[2] == 53.0 * math.pi / 180


def test_parsed_units_agree_with_the_propagated_orbit():
    """The parser's unit conversions checked through the physics, not its own
    formulas: propagating the parsed elements (oracle, FP64) must give an orbit
    whose period is 1440 / (rev/day) minutes, whose maximum |z| / r is sin i and
    whose ascending node lies at the RAAN (to the J2 effects over one orbit),
    and whose epoch is where the text puts it."""
    from oracle import propagate
    l1 = "1 00042U 25001A   25032.25000000  .00000000  00000-0  00000-0 0  999"
    l2 = "2 00042  51.6000  80.0000 0001000  30.0000 200.0000 15.50000000   17"
    l1, l2 = _tle(l1, l2)
    ref = (oi.jd0(2025, 1, 1), 0.0)
    el, _, st = sg.parse_text(l1 + "\n" + l2 + "\n", "tle", ref_jd=ref)
    assert st[0] == 0
    assert el[7, 0] == 31.25                              # day 32.25 of 2025 is 31.25 days after January 1, 0h
    period = 1440.0 / 15.5
    t = 1440.0 * el[7, 0] + np.linspace(0.0, 1.2 * period, 4001)
    r, v, err = propagate(el, t)
    assert np.all(err == 0)
    x, y, z = r[0, 0], r[1, 0], r[2, 0]
    rr = np.sqrt(x * x + y * y + z * z)
    assert abs(np.degrees(np.arcsin(np.max(np.abs(z) / rr))) - 51.6) < 0.05
    # consecutive ascending crossings of the equator: period and node longitude
    up = np.flatnonzero((z[:-1] < 0) & (z[1:] >= 0))
    assert len(up) >= 1
    k = up[0]
    f = -z[k] / (z[k + 1] - z[k])
    tc = t[k] + f * (t[k + 1] - t[k])
    xc, yc = x[k] + f * (x[k + 1] - x[k]), y[k] + f * (y[k + 1] - y[k])
    node = math.degrees(math.atan2(yc, xc)) % 360.0
    assert abs(node - 80.0) < 0.4                          # nodal regression ~5 deg/day: < 0.35 deg in an orbit
    # the satellite starts at u = 30 + 200 deg from the node; it reaches the node after (360 - 230)/360 of an orbit
    assert abs((tc - t[0]) - period * (360.0 - 230.0) / 360.0) < 0.01 * period
