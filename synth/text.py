"""Synthetic element-set text: seeded catalogues written as two-line element
sets (TLE / 3LE) and as CCSDS OMM records (KVN, CSV, JSON).

No element-set files are available here, so the ingestion path is exercised
on text written from the synthetic catalogues.  The writer follows the
published fixed-column TLE layout (columns 1-69 per line, modulo-10
checksum in column 69) and the OMM keyword names; it rounds each element to
the precision the format prints, so the text, not the float elements, is
the ground truth a parser must reproduce.

Epochs: the catalogue's epoch row is days after a reference instant; the
writer places that reference at REF_JD (a two-part Julian date).
"""
from __future__ import annotations

import datetime as _dt
import json as _json
import math

import numpy as np

__all__ = ["REF_JD", "tle_lines", "tle_text", "omm_kvn", "omm_csv", "omm_json", "corrupt_tle"]

# 2025-01-01 00:00 UTC as (Julian date at 0h, day fraction).
REF_JD = (2460676.5, 0.0)
_JD_ORDINAL0 = 1721424.5  # Julian date at 0h of proleptic Gregorian ordinal 0 (0000-12-31)


def _calendar(epoch_days: float):
    """Absolute epoch as (datetime date, fraction of day) from days after REF_JD."""
    jd = REF_JD[0] + REF_JD[1] + float(epoch_days)
    day0 = math.floor(jd - 0.5)          # JD at 0h is day0 + 0.5
    frac = jd - 0.5 - day0
    date = _dt.date.fromordinal(int(day0 + 0.5 - _JD_ORDINAL0))
    return date, frac


def _checksum(line68: str) -> str:
    s = 0
    for c in line68:
        if c.isdigit():
            s += int(c)
        elif c == "-":
            s += 1
    return str(s % 10)


def _assumed(x: float) -> str:
    """' 12345-3' form: sign, five mantissa digits (assumed leading point), exponent."""
    if x == 0.0 or not math.isfinite(x):
        return " 00000-0"
    sign = "-" if x < 0 else " "
    a = abs(x)
    e = math.floor(math.log10(a)) + 1
    m = int(round(a / 10.0 ** e * 1e5))
    if m >= 100000:
        m //= 10
        e += 1
    e = max(-9, min(9, e))
    return f"{sign}{m:05d}{'-' if e < 0 else '+'}{abs(e)}"


def _satnum(k: int) -> str:
    if k < 100000:
        return f"{k:05d}"
    lead = k // 10000
    letters = "ABCDEFGHJKLMNPQRSTUVWXYZ"  # 10..33, I and O skipped
    return letters[lead - 10] + f"{k % 10000:04d}"


def tle_lines(elem: np.ndarray, satnums=None, names=None):
    """Two-line element sets for the columns of elem ([8, n], catalogue rows);
    returns a list of (name or None, line1, line2)."""
    n = elem.shape[1]
    if satnums is None:
        satnums = np.arange(1, n + 1) % 100000
    out = []
    for i in range(n):
        no, ecc, inc, node, argp, mo, bstar, ep = (float(x) for x in elem[:, i])
        date, frac = _calendar(ep)
        yy = date.year % 100
        doy = date.timetuple().tm_yday
        day = f"{doy:03d}.{int(round(frac * 1e8)):08d}"
        if day.endswith("100000000"):  # the fraction rounded up to a whole day
            day = f"{doy:03d}.99999999"
        sn = _satnum(int(satnums[i]))
        l1 = (f"1 {sn}U 25001A   {yy:02d}{day} {' .00000000':>10} {' 00000-0'} {_assumed(bstar)} 0 "
              f"{(i % 9999) + 1:>4d}")
        mm = no * 1440.0 / (2.0 * math.pi)
        e7 = int(round(ecc * 1e7))
        deg = lambda x: math.degrees(x) % 360.0  # noqa: E731
        l2 = (f"2 {sn} {math.degrees(inc):8.4f} {deg(node):8.4f} {min(e7, 9999999):07d} {deg(argp):8.4f} "
              f"{deg(mo):8.4f} {mm:11.8f}{(i * 7) % 100000:5d}")
        l2 = l2.replace("360.0000", "  0.0000")
        assert len(l1) == 68 and len(l2) == 68, (l1, l2)
        out.append((None if names is None else names[i], l1 + _checksum(l1), l2 + _checksum(l2)))
    return out


def tle_text(elem: np.ndarray, satnums=None, three_line=False, crlf=False) -> str:
    names = [f"SYNTH-{i:06d}" for i in range(elem.shape[1])] if three_line else None
    nl = "\r\n" if crlf else "\n"
    rows = []
    for name, l1, l2 in tle_lines(elem, satnums, names):
        if name is not None:
            rows.append(name)
        rows += [l1, l2]
    return nl.join(rows) + nl


def corrupt_tle(lines, rng: np.random.Generator, frac: float = 0.05):
    """Flip a digit (checksum error), change the second line's catalogue
    number (mismatch) or blank a field (unparsable) in a fraction of records."""
    out = []
    for name, l1, l2 in lines:
        u = rng.random()
        if u < frac / 3:
            k = 20 + int(rng.integers(0, 12))
            c = l1[k]
            if c.isdigit():
                l1 = l1[:k] + str((int(c) + 1) % 10) + l1[k + 1:]
        elif u < 2 * frac / 3:
            l2 = l2[:2] + "99999" + l2[7:]
        elif u < frac:
            l2 = l2[:8] + "   x.xxx" + l2[16:]
        out.append((name, l1, l2))
    return out


def _omm_fields(elem: np.ndarray, i: int):
    no, ecc, inc, node, argp, mo, bstar, ep = (float(x) for x in elem[:, i])
    date, frac = _calendar(ep)
    us = int(round(frac * 86400e6))
    us = min(us, 86400 * 10 ** 6 - 1)
    t = _dt.datetime(date.year, date.month, date.day) + _dt.timedelta(microseconds=us)
    return {
        "OBJECT_NAME": f"SYNTH-{i:06d}",
        "NORAD_CAT_ID": str(i + 1),
        "EPOCH": t.strftime("%Y-%m-%dT%H:%M:%S.%f"),
        "MEAN_MOTION": f"{no * 1440.0 / (2.0 * math.pi):.8f}",
        "ECCENTRICITY": f"{ecc:.7f}",
        "INCLINATION": f"{math.degrees(inc):.4f}",
        "RA_OF_ASC_NODE": f"{math.degrees(node) % 360.0:.4f}",
        "ARG_OF_PERICENTER": f"{math.degrees(argp) % 360.0:.4f}",
        "MEAN_ANOMALY": f"{math.degrees(mo) % 360.0:.4f}",
        "BSTAR": f"{bstar:.8e}",
        "MEAN_MOTION_DOT": "0",
        "MEAN_MOTION_DDOT": "0",
    }


def omm_kvn(elem: np.ndarray) -> str:
    out = []
    for i in range(elem.shape[1]):
        f = _omm_fields(elem, i)
        out.append("CCSDS_OMM_VERS = 2.0")
        out.append("COMMENT synthetic element set")
        for k, v in f.items():
            unit = " [rev/day]" if k == "MEAN_MOTION" else (" [deg]" if k in ("INCLINATION", "MEAN_ANOMALY") else "")
            out.append(f"{k} = {v}{unit}")
        out.append("")
    return "\n".join(out)


def omm_csv(elem: np.ndarray) -> str:
    rows = [_omm_fields(elem, i) for i in range(elem.shape[1])]
    keys = list(rows[0].keys()) if rows else []
    return "\n".join([",".join(keys)] + [",".join(r[k] for k in keys) for r in rows]) + "\n"


def omm_json(elem: np.ndarray) -> str:
    rows = []
    for i in range(elem.shape[1]):
        f = _omm_fields(elem, i)
        rows.append({k: (v if k in ("OBJECT_NAME", "EPOCH") else (int(v) if k == "NORAD_CAT_ID" else float(v)))
                     for k, v in f.items()})
    return _json.dumps(rows)
