"""Element-set text parser: TEST INFRASTRUCTURE ONLY (oracle of the library's
native ingestion).

Plain Python written from the format definitions, for checking the native
parser record by record; only the tests may call it.

Two-line element sets (the fixed-column layout of the published format):
  line 1: columns 3-7 catalogue number, 19-20 epoch year (57-99 -> 19xx,
          00-56 -> 20xx), 21-32 epoch day of year with fraction (day 1.0 is
          January 1, 0h UTC), 54-61 B* with an assumed leading decimal point
          and a signed exponent, 69 checksum;
  line 2: columns 3-7 catalogue number, 9-16 inclination (deg), 18-25 right
          ascension of the ascending node (deg), 27-33 eccentricity (assumed
          leading decimal point), 35-42 argument of perigee (deg), 44-51 mean
          anomaly (deg), 53-63 mean motion (rev/day), 69 checksum;
  checksum: the sum of the digits of columns 1-68, each '-' counting one,
  modulo 10.  Alpha-5 catalogue numbers put a letter (A = 10 ... Z = 33, I
  and O not used) in place of the ten-thousands digits.
OMM (CCSDS Orbit Mean-elements Message) records carry the same elements under
keyword names, epoch as ISO 8601 UTC.

Output rows as the propagation oracle takes them: no_kozai (rad/min: rev/day
divided by 1440 / 2 pi), ecco, inclo, nodeo, argpo, mo (rad: degrees times
pi / 180), bstar, epoch in days after the reference Julian date
ref = (whole, frac): (JD at 0h of the epoch's day - ref[0]) + (day fraction
- ref[1]).  Status bits: 1 checksum, 2 catalogue numbers differ, 4 a field
missing or not a number (elements NaN).
"""
from __future__ import annotations

import datetime
import json
import math
import re
from fractions import Fraction

import numpy as np

CHECKSUM, MISMATCH, FIELD = 1, 2, 4
J2000 = (2451545.0, 0.0)
RAD_PER_DEG = math.pi / 180.0
MIN_PER_RAD = 1440.0 / (2.0 * math.pi)
_ORDINAL_JD0 = 1721424.5  # JD at 0h of the day before 0001-01-01 (ordinal 0)
ALPHA5 = "ABCDEFGHJKLMNPQRSTUVWXYZ"


def jd0(year: int, month: int, day: int) -> float:
    """Julian date at 0h UTC of a Gregorian calendar date (via date ordinals)."""
    return _ORDINAL_JD0 + datetime.date(year, month, day).toordinal()


def checksum(line: str) -> int:
    total = 0
    for c in line[:68]:
        if "0" <= c <= "9":
            total += ord(c) - ord("0")
        elif c == "-":
            total += 1
    return total % 10


def satnum(field: str):
    f = field.strip()
    if len(f) == 5 and f[0] in ALPHA5:
        if not f[1:].isdigit():
            return None
        return (10 + ALPHA5.index(f[0])) * 10000 + int(f[1:])
    if not f or not f.isdigit():
        return None
    return int(f)


def assumed_decimal(field: str):
    """' 12345-3' -> 0.12345e-3 (the decimal string converted once)."""
    m = re.fullmatch(r"\s*([+-]?)(\d+)(?:([+-])(\d+))?\s*", field)
    if not m:
        return None
    sign, mant, esign, exp = m.groups()
    text = ("-" if sign == "-" else "") + "0." + mant
    if esign:
        text += "e" + esign + exp
    return float(text)


def _number(field: str):
    try:
        s = field.strip()
        if not s or not re.fullmatch(r"[+-]?(\d+\.?\d*|\.\d+)([eE][+-]?\d+)?", s):
            return None
        return float(s)
    except ValueError:
        return None


def _fraction_digits(digits: str):
    if not digits.isdigit():
        return None
    return float("0." + digits[:18])


def parse_tle_record(l1: str, l2: str):
    """Returns (fields dict or None, satnum, status)."""
    status = 0
    n1, n2 = satnum(l1[2:7]), satnum(l2[2:7])
    if n1 is None or n2 is None:
        status |= FIELD
    elif n1 != n2:
        status |= MISMATCH
    if not (l1[68].isdigit() and l2[68].isdigit() and checksum(l1) == int(l1[68]) and checksum(l2) == int(l2[68])):
        status |= CHECKSUM
    sat = n1 if n1 is not None else -1
    try:
        yy = int(l1[18:20])
        if not 0 <= yy <= 99:
            raise ValueError
        year = 2000 + yy if yy < 57 else 1900 + yy
        day_text = l1[20:32].strip()
        whole_day, frac_digits = day_text.split(".")
        doy = int(whole_day)
        frac = _fraction_digits(frac_digits) if frac_digits else 0.0
        ndays = 366 if (year % 4 == 0 and (year % 100 != 0 or year % 400 == 0)) else 365
        if frac is None or not 1 <= doy <= ndays:
            raise ValueError
        whole = jd0(year, 1, 1) + (doy - 1)
        ecc_text = l2[26:33].strip()
        vals = dict(bstar=assumed_decimal(l1[53:61]), incl=_number(l2[8:16]), node=_number(l2[17:25]),
                    ecc=_fraction_digits(ecc_text) if ecc_text else None, argp=_number(l2[34:42]),
                    mo=_number(l2[43:51]), mm=_number(l2[52:63]))
        if any(v is None for v in vals.values()):
            raise ValueError
    except ValueError:
        return None, sat, status | FIELD
    vals["whole"], vals["frac"] = whole, frac
    return vals, sat, status


def _row(vals, ref):
    if vals is None:
        return [math.nan] * 8
    return [vals["mm"] / MIN_PER_RAD, vals["ecc"], vals["incl"] * RAD_PER_DEG, vals["node"] * RAD_PER_DEG,
            vals["argp"] * RAD_PER_DEG, vals["mo"] * RAD_PER_DEG, vals["bstar"],
            (vals["whole"] - ref[0]) + (vals["frac"] - ref[1])]


def _lines(text: str):
    return [l[:-1] if l.endswith("\r") else l for l in text.split("\n")]


def parse_tle(text: str, ref=J2000):
    """All records of a TLE / 3LE text: (elem [8, n], satnum [n], status [n])."""
    lines = _lines(text)
    rows, sats, stats = [], [], []
    k = 0
    while k < len(lines):
        l1 = lines[k]
        if (len(l1) >= 69 and l1[:2] == "1 " and k + 1 < len(lines) and len(lines[k + 1]) >= 69
                and lines[k + 1][:2] == "2 "):
            vals, sat, st = parse_tle_record(l1, lines[k + 1])
            rows.append(_row(vals, ref))
            sats.append(sat)
            stats.append(st)
            k += 2
        else:
            k += 1
    return _pack(rows, sats, stats)


def _pack(rows, sats, stats):
    elem = np.array(rows, dtype=np.float64).reshape(-1, 8).T.copy()
    return elem, np.array(sats, dtype=np.int64), np.array(stats, dtype=np.int32)


def parse_iso(text: str):
    """'YYYY-MM-DDThh:mm:ss[.f]' or 'YYYY-DDDThh:mm:ss[.f]' (UTC, optional Z) ->
    (JD at 0h, day fraction) with the fraction nanoseconds / 86,400e9."""
    m = re.fullmatch(r"\s*(\d{4})-(?:(\d{1,2})-(\d{1,2})|(\d{1,3}))T(\d{2}):(\d{2}):(\d{2})(?:\.(\d*))?[Zz]?\s*", text)
    if not m:
        return None
    y, mo, d, doy, hh, mi, ss, fr = m.groups()
    y = int(y)
    try:
        if doy is not None:
            base = jd0(y, 1, 1) + (int(doy) - 1)
            if int(doy) < 1 or int(doy) > (366 if (y % 4 == 0 and (y % 100 != 0 or y % 400 == 0)) else 365):
                return None
        else:
            base = jd0(y, int(mo), int(d))
    except ValueError:
        return None
    hh, mi, ss = int(hh), int(mi), int(ss)
    if hh > 23 or mi > 59 or ss > 60:
        return None
    ns = int((fr or "")[:9].ljust(9, "0")) if fr is not None else 0
    day_ns = ((hh * 60 + mi) * 60 + ss) * 10 ** 9 + ns
    return base, day_ns / 86400e9


REQUIRED = ("MEAN_MOTION", "ECCENTRICITY", "INCLINATION", "RA_OF_ASC_NODE", "ARG_OF_PERICENTER", "MEAN_ANOMALY",
            "BSTAR")


def _omm_record(rec: dict, ref):
    rec = {k.strip().upper(): (v.strip().strip('"') if isinstance(v, str) else v) for k, v in rec.items()}
    sat = -1
    if "NORAD_CAT_ID" in rec:
        try:
            sat = int(str(rec["NORAD_CAT_ID"]).strip())
        except ValueError:
            sat = -1
    vals = {}
    for k in REQUIRED:
        v = rec.get(k)
        x = _number(str(v)) if v is not None else None
        if x is None:
            return [math.nan] * 8, sat, FIELD
        vals[k] = x
    ep = parse_iso(str(rec.get("EPOCH", "")))
    if ep is None:
        return [math.nan] * 8, sat, FIELD
    row = _row(dict(mm=vals["MEAN_MOTION"], ecc=vals["ECCENTRICITY"], incl=vals["INCLINATION"],
                    node=vals["RA_OF_ASC_NODE"], argp=vals["ARG_OF_PERICENTER"], mo=vals["MEAN_ANOMALY"],
                    bstar=vals["BSTAR"], whole=ep[0], frac=ep[1]), ref)
    return row, sat, 0


def parse_omm(text: str, fmt: str, ref=J2000):
    """fmt: 'kvn', 'csv' or 'json'."""
    recs = []
    if fmt == "kvn":
        cur = {}
        for line in _lines(text):
            s = line.strip()
            if not s or s.startswith("COMMENT") or "=" not in s:
                continue
            k, v = s.split("=", 1)
            k = k.strip()
            v = v.split("[", 1)[0].strip()
            if (k == "CCSDS_OMM_VERS" or k in cur) and cur:
                recs.append(cur)
                cur = {}
            cur[k] = v
        if cur:
            recs.append(cur)
    elif fmt == "csv":
        lines = [l.strip() for l in _lines(text) if l.strip()]
        if lines:
            head = [h.strip().strip('"') for h in lines[0].split(",")]
            for l in lines[1:]:
                recs.append(dict(zip(head, l.split(","))))
    elif fmt == "json":
        data = json.loads(text)
        recs = data if isinstance(data, list) else [data]
        recs = [{k: (v if isinstance(v, str) else json.dumps(v)) for k, v in r.items()} for r in recs]
    else:
        raise ValueError(fmt)
    rows, sats, stats = [], [], []
    for r in recs:
        row, sat, st = _omm_record(r, ref)
        rows.append(row)
        sats.append(sat)
        stats.append(st)
    return _pack(rows, sats, stats)


def exact_day_fraction(digits: str) -> Fraction:
    """The exact rational value of a fraction-of-day digit string (for pins)."""
    return Fraction(int(digits), 10 ** len(digits))
