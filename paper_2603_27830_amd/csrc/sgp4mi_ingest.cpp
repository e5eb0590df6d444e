// Ingestion: element-set text (two-line element sets, CCSDS OMM in KVN, CSV
// or JSON form) to the model's elements, on the host.
//
// jaxsgp4 takes its satellites from two-line element sets through the
// reference implementation's parser (paper section 2.1) and notes that a
// 32-bit Julian-date epoch loses precision (section 4).  Here every epoch is
// split into a whole-day part (a Julian date at 0h, exact in double) and a day
// fraction parsed from its decimal digits, and the element row carries the
// epoch as days after a caller-chosen reference given the same way, so the
// difference keeps the full resolution of the text (1e-8 day for TLE, 1 ns
// for OMM) whatever the magnitude of the Julian date.
//
// Decimal fields are converted with std::from_chars (correctly rounded,
// locale-independent).  Unit conversions: mean motion rev/day -> rad/min by
// division by 1440 / (2 pi); degrees -> radians by multiplication by pi / 180.
#include <atomic>
#include <charconv>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "sgp4mi.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kDeg2Rad = kPi / 180.0;
constexpr double kMinPerRad = 1440.0 / (2.0 * kPi);  // (rev/day) / (rad/min)
constexpr double kNaN = __builtin_nan("");

struct Fields {
  double no_kozai, ecco, inclo, nodeo, argpo, mo, bstar;
  double jd_whole, jd_frac;  // epoch: Julian date at 0h of the day, day fraction
  int64_t satnum;
  int32_t status;
};

// ------------------------------------------------------------ primitives --
bool is_digit(char c) { return c >= '0' && c <= '9'; }

// Trimmed view [b, e) of s.
void trim(const char*& b, const char*& e) {
  while (b < e && (*b == ' ' || *b == '\t')) ++b;
  while (e > b && (e[-1] == ' ' || e[-1] == '\t' || e[-1] == '\r')) --e;
}

// A decimal number (optional sign, digits, point, exponent); false unless the
// whole trimmed field is one number.
bool parse_double(const char* b, const char* e, double* out) {
  trim(b, e);
  if (b == e) return false;
  if (*b == '+') ++b;  // from_chars accepts '-' but not '+'
  const auto r = std::from_chars(b, e, *out, std::chars_format::general);
  return r.ec == std::errc() && r.ptr == e && std::isfinite(*out);
}


bool parse_int(const char* b, const char* e, int64_t* out) {
  trim(b, e);
  if (b == e) return false;
  if (*b == '+') ++b;
  const auto r = std::from_chars(b, e, *out);
  return r.ec == std::errc() && r.ptr == e;
}

// A non-empty run of decimal digits only (no sign, no blanks).
bool fixed_digits(const char* b, const char* e, int64_t* out) {
  for (const char* p = b; p < e; ++p)
    if (!is_digit(*p)) return false;
  return b < e && parse_int(b, e, out);
}

// Julian date at 0h of the proleptic Gregorian date y-m-d (years >= 1): the
// day count from 0000-03-01 (years taken from March, so that the leap day
// ends the year) plus that origin's Julian date.
double jd_at_0h(int64_t y, int64_t m, int64_t d) {
  const int64_t a = m <= 2 ? 1 : 0;
  const int64_t yy = y - a;
  const int64_t mm = m + 12 * a - 3;  // 0 = March ... 11 = February
  const int64_t days = 365 * yy + yy / 4 - yy / 100 + yy / 400 + (153 * mm + 2) / 5 + d - 1;
  // days counts from 0000-03-01; 0000-03-01 is JD 1721119.5 at 0h
  return 1721119.5 + double(days);
}

bool leap(int64_t y) { return (y % 4 == 0 && y % 100 != 0) || y % 400 == 0; }

// Fraction digits "ddd..." (at most 18) -> value / 10^len, correctly rounded.
bool digits_fraction(const char* b, const char* e, double* out) {
  if (e - b > 18) e = b + 18;
  if (b == e) { *out = 0.0; return true; }
  std::string s = "0.";
  for (const char* p = b; p < e; ++p) {
    if (!is_digit(*p)) return false;
    s.push_back(*p);
  }
  const auto r = std::from_chars(s.data(), s.data() + s.size(), *out);
  return r.ec == std::errc();
}

// ------------------------------------------------------------------- TLE --
// Assumed-decimal field with exponent, e.g. " 12345-3" = 0.12345e-3,
// "-11606-4" = -0.11606e-4, " 00000+0" = 0.
bool parse_assumed(const char* b, const char* e, double* out) {
  trim(b, e);
  if (b == e) return false;
  std::string s;
  if (*b == '-' || *b == '+') { if (*b == '-') s.push_back('-'); ++b; }
  // mantissa digits, then an exponent sign and digits
  const char* m = b;
  while (b < e && is_digit(*b)) ++b;
  if (b == m) return false;
  s += "0.";
  s.append(m, b);
  if (b < e) {
    if (*b != '-' && *b != '+') return false;
    s.push_back('e');
    s.push_back(*b++);
    if (b == e) return false;
    const char* x = b;
    while (b < e && is_digit(*b)) ++b;
    if (b != e || b == x) return false;
    s.append(x, e);
  }
  const auto r = std::from_chars(s.data(), s.data() + s.size(), *out);
  return r.ec == std::errc();
}

// Catalogue number: five digits, or the alpha-5 form (a letter for the
// ten-thousands, A = 10 ... Z = 33 skipping I and O, then four digits).
bool parse_satnum(const char* b, const char* e, int64_t* out) {
  trim(b, e);
  if (b == e) return false;
  if (*b >= 'A' && *b <= 'Z') {
    const char c = *b;
    if (c == 'I' || c == 'O' || e - b != 5) return false;
    int64_t v = 10 + (c - 'A');
    if (c > 'I') --v;
    if (c > 'O') --v;
    int64_t rest;
    for (const char* p = b + 1; p < e; ++p)
      if (!is_digit(*p)) return false;
    if (!parse_int(b + 1, e, &rest)) return false;
    *out = v * 10000 + rest;
    return true;
  }
  for (const char* p = b; p < e; ++p)
    if (!is_digit(*p)) return false;
  return parse_int(b, e, out);
}

// Modulo-10 checksum of columns 1-68: digits count their value, '-' counts 1.
int tle_checksum(const char* line) {
  int s = 0;
  for (int k = 0; k < 68; ++k) {
    const char c = line[k];
    if (is_digit(c)) s += c - '0';
    else if (c == '-') s += 1;
  }
  return s % 10;
}

// Columns a..b (1-based, inclusive) of a line.
struct Line {
  const char* p;
  const char* col(int a) const { return p + a - 1; }
  const char* end(int b) const { return p + b; }
};

void parse_tle(const char* l1, const char* l2, Fields* f) {
  const Line a{l1}, b{l2};
  int32_t st = 0;
  int64_t n1 = -1, n2 = -1;
  const bool num1 = parse_satnum(a.col(3), a.end(7), &n1);
  const bool num2 = parse_satnum(b.col(3), b.end(7), &n2);
  if (!num1 || !num2) st |= SGP4_REC_FIELD;
  else if (n1 != n2) st |= SGP4_REC_MISMATCH;
  f->satnum = n1;
  if (!is_digit(l1[68]) || !is_digit(l2[68]) || tle_checksum(l1) != l1[68] - '0' || tle_checksum(l2) != l2[68] - '0')
    st |= SGP4_REC_CHECKSUM;

  // Epoch: two-digit year (57-99 -> 19xx, 00-56 -> 20xx), day of year with fraction.
  int64_t yy = 0;
  bool ok = parse_int(a.col(19), a.end(20), &yy) && yy >= 0 && yy <= 99;
  const int64_t year = yy < 57 ? 2000 + yy : 1900 + yy;
  const char* db = a.col(21);
  const char* de = a.end(32);
  trim(db, de);
  const char* dot = static_cast<const char*>(memchr(db, '.', size_t(de - db)));
  int64_t day = 0;
  double frac = 0.0;
  if (ok) ok = dot && parse_int(db, dot, &day) && digits_fraction(dot + 1, de, &frac);
  if (ok) ok = day >= 1 && day <= (leap(year) ? 366 : 365);
  f->jd_whole = ok ? jd_at_0h(year, 1, 1) + double(day - 1) : kNaN;
  f->jd_frac = ok ? frac : kNaN;

  double bstar, incl, node, ecc, argp, mo, mm;
  ok = ok && parse_assumed(a.col(54), a.end(61), &bstar);
  ok = ok && parse_double(b.col(9), b.end(16), &incl);
  ok = ok && parse_double(b.col(18), b.end(25), &node);
  // eccentricity: seven digits after an assumed leading decimal point
  {
    const char* eb = b.col(27);
    const char* ee = b.end(33);
    trim(eb, ee);
    ok = ok && eb < ee && digits_fraction(eb, ee, &ecc);
  }
  ok = ok && parse_double(b.col(35), b.end(42), &argp);
  ok = ok && parse_double(b.col(44), b.end(51), &mo);
  ok = ok && parse_double(b.col(53), b.end(63), &mm);
  if (!ok) {
    st |= SGP4_REC_FIELD;
    f->no_kozai = f->ecco = f->inclo = f->nodeo = f->argpo = f->mo = f->bstar = kNaN;
    f->jd_whole = f->jd_frac = kNaN;
  } else {
    f->no_kozai = mm / kMinPerRad;
    f->ecco = ecc;
    f->inclo = incl * kDeg2Rad;
    f->nodeo = node * kDeg2Rad;
    f->argpo = argp * kDeg2Rad;
    f->mo = mo * kDeg2Rad;
    f->bstar = bstar;
  }
  f->status = st;
}

// Lines of the text: [start, end) without the line break.
struct Span {
  const char* b;
  const char* e;
};

const char* next_line(const char* p, const char* end, Span* s) {
  const char* nl = static_cast<const char*>(memchr(p, '\n', size_t(end - p)));
  const char* le = nl ? nl : end;
  s->b = p;
  s->e = (le > p && le[-1] == '\r') ? le - 1 : le;
  return nl ? nl + 1 : end;
}

bool tle_line(const Span& s, char tag) { return s.e - s.b >= 69 && s.b[0] == tag && s.b[1] == ' '; }

// Record starts (pointer to line 1) of the TLE records whose line 1 begins in
// [from, to); scanning continues past `to` only to read the record's line 2.
void tle_scan(const char* from, const char* to, const char* end, std::vector<const char*>* out) {
  const char* p = from;
  while (p < to) {
    Span s;
    const char* q = next_line(p, end, &s);
    if (tle_line(s, '1') && q < end) {
      Span s2;
      const char* r = next_line(q, end, &s2);
      if (tle_line(s2, '2')) {
        out->push_back(s.b);
        p = r;
        continue;
      }
    }
    p = q;
  }
}

// fn(k) for k in [0, parts) on worker threads; a part whose thread cannot be
// started runs on the calling thread, every started thread is joined, and a
// failure inside a worker is rethrown on the calling thread as bad_alloc.
template <class F>
void run_parts(int parts, F fn) {
  std::atomic<bool> failed{false};
  auto body = [&](int k) {
    try {
      fn(k);
    } catch (...) {
      failed = true;
    }
  };
  std::vector<std::thread> pool;
  try {
    pool.reserve(size_t(parts));
  } catch (...) {
  }
  for (int k = 0; k < parts; ++k) {
    try {
      pool.emplace_back(body, k);
    } catch (...) {
      body(k);
    }
  }
  for (auto& th : pool) th.join();
  if (failed) throw std::bad_alloc();
}

// Line-aligned chunk boundaries of the text for `parts` workers.
std::vector<const char*> chunks(const char* text, size_t len, int parts) {
  std::vector<const char*> cut{text};
  const char* end = text + len;
  for (int k = 1; k < parts; ++k) {
    const char* p = text + len * size_t(k) / size_t(parts);
    if (p <= cut.back()) continue;
    const char* nl = static_cast<const char*>(memchr(p, '\n', size_t(end - p)));
    p = nl ? nl + 1 : end;
    if (p > cut.back() && p < end) cut.push_back(p);
  }
  cut.push_back(end);
  return cut;
}

int worker_count(int threads, size_t len) {
  int t = threads > 0 ? threads : int(std::thread::hardware_concurrency());
  if (t < 1) t = 1;
  if (t > 64) t = 64;
  const size_t per = 1 << 20;  // no worker for less than ~1 MB of text
  const size_t cap = len / per + 1;
  return int(size_t(t) < cap ? size_t(t) : cap);
}

// All TLE record starts, in text order.
std::vector<const char*> tle_records(const char* text, size_t len, int threads) {
  const std::vector<const char*> cut = chunks(text, len, worker_count(threads, len));
  const int parts = int(cut.size()) - 1;
  std::vector<std::vector<const char*>> found(size_t(parts > 0 ? parts : 0));
  const char* end = text + len;
  if (parts <= 1) {
    std::vector<const char*> all;
    if (parts == 1) tle_scan(cut[0], cut[1], end, &all);
    return all;
  }
  run_parts(parts, [&](int k) { tle_scan(cut[k], cut[k + 1], end, &found[size_t(k)]); });
  std::vector<const char*> all;
  for (auto& v : found) all.insert(all.end(), v.begin(), v.end());
  return all;
}

// ------------------------------------------------------------------- OMM --
// One OMM record as key/value pairs (views into the text).
struct KV {
  const char* kb;
  const char* ke;
  const char* vb;
  const char* ve;
};
using Record = std::vector<KV>;

bool key_is(const KV& kv, const char* name) {
  const size_t n = strlen(name);
  if (size_t(kv.ke - kv.kb) != n) return false;
  for (size_t k = 0; k < n; ++k) {
    char c = kv.kb[k];
    if (c >= 'a' && c <= 'z') c = char(c - 'a' + 'A');
    if (c != name[k]) return false;
  }
  return true;
}

const KV* find(const Record& r, const char* name) {
  for (const KV& kv : r)
    if (key_is(kv, name)) return &kv;
  return nullptr;
}

// ISO 8601 UTC epoch "YYYY-MM-DDThh:mm:ss[.f...]" or "YYYY-DDDThh:mm:ss[.f...]"
// (day of year), optional trailing 'Z'.  Day fraction = nanoseconds of the
// day / 86,400e9 (exact integer, one rounding).
bool parse_iso(const char* b, const char* e, double* whole, double* frac) {
  trim(b, e);
  if (e > b && (e[-1] == 'Z' || e[-1] == 'z')) --e;
  const char* t = static_cast<const char*>(memchr(b, 'T', size_t(e - b)));
  if (!t) return false;
  int64_t y, m = 0, d = 0, doy = 0;
  const char* h1 = static_cast<const char*>(memchr(b, '-', size_t(t - b)));
  if (!h1 || h1 - b != 4 || !fixed_digits(b, h1, &y)) return false;
  const char* h2 = static_cast<const char*>(memchr(h1 + 1, '-', size_t(t - h1 - 1)));
  if (h2) {
    if (h2 - h1 - 1 > 2 || t - h2 - 1 > 2) return false;
    if (!fixed_digits(h1 + 1, h2, &m) || !fixed_digits(h2 + 1, t, &d)) return false;
    static const int kDays[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    if (m < 1 || m > 12 || d < 1 || d > kDays[m - 1] + (m == 2 && leap(y) ? 1 : 0)) return false;
    *whole = jd_at_0h(y, m, d);
  } else {
    if (t - h1 - 1 > 3 || !fixed_digits(h1 + 1, t, &doy) || doy < 1 || doy > (leap(y) ? 366 : 365)) return false;
    *whole = jd_at_0h(y, 1, 1) + double(doy - 1);
  }
  // time of day
  const char* p = t + 1;
  if (e - p < 8 || p[2] != ':' || p[5] != ':') return false;
  int64_t hh, mi, ss;
  if (!fixed_digits(p, p + 2, &hh) || !fixed_digits(p + 3, p + 5, &mi) || !fixed_digits(p + 6, p + 8, &ss))
    return false;
  if (hh < 0 || hh > 23 || mi < 0 || mi > 59 || ss < 0 || ss > 60) return false;
  int64_t ns = 0;
  p += 8;
  if (p < e) {
    if (*p != '.') return false;
    ++p;
    int digits = 0;
    for (; p < e; ++p) {
      if (!is_digit(*p)) return false;
      if (digits < 9) { ns = ns * 10 + (*p - '0'); ++digits; }
    }
    for (; digits < 9; ++digits) ns *= 10;
  }
  const int64_t day_ns = ((hh * 60 + mi) * 60 + ss) * 1000000000LL + ns;
  *frac = double(day_ns) / 86400e9;
  return true;
}

void unquote(const char*& b, const char*& e) {
  trim(b, e);
  if (e - b >= 2 && ((*b == '"' && e[-1] == '"') || (*b == '\'' && e[-1] == '\''))) { ++b; --e; }
}

void omm_fields(const Record& r, Fields* f) {
  int32_t st = 0;
  double mm = kNaN, ecc = kNaN, incl = kNaN, node = kNaN, argp = kNaN, mo = kNaN, bstar = kNaN;
  double whole = kNaN, frac = kNaN;
  auto num = [&](const char* name, double* out) {
    const KV* kv = find(r, name);
    if (!kv) return false;
    const char* b = kv->vb;
    const char* e = kv->ve;
    unquote(b, e);
    return parse_double(b, e, out);
  };
  bool ok = num("MEAN_MOTION", &mm) && num("ECCENTRICITY", &ecc) && num("INCLINATION", &incl) &&
            num("RA_OF_ASC_NODE", &node) && num("ARG_OF_PERICENTER", &argp) && num("MEAN_ANOMALY", &mo) &&
            num("BSTAR", &bstar);
  const KV* ep = find(r, "EPOCH");
  if (ep) {
    const char* b = ep->vb;
    const char* e = ep->ve;
    unquote(b, e);
    ok = ok && parse_iso(b, e, &whole, &frac);
  } else {
    ok = false;
  }
  f->satnum = -1;
  if (const KV* id = find(r, "NORAD_CAT_ID")) {
    const char* b = id->vb;
    const char* e = id->ve;
    unquote(b, e);
    int64_t v;
    if (parse_int(b, e, &v)) f->satnum = v;
  }
  if (!ok) {
    st |= SGP4_REC_FIELD;
    f->no_kozai = f->ecco = f->inclo = f->nodeo = f->argpo = f->mo = f->bstar = kNaN;
    f->jd_whole = f->jd_frac = kNaN;
  } else {
    f->no_kozai = mm / kMinPerRad;
    f->ecco = ecc;
    f->inclo = incl * kDeg2Rad;
    f->nodeo = node * kDeg2Rad;
    f->argpo = argp * kDeg2Rad;
    f->mo = mo * kDeg2Rad;
    f->bstar = bstar;
    f->jd_whole = whole;
    f->jd_frac = frac;
  }
  f->status = st;
}

// KVN: "KEY = value" lines; a record ends where the next begins (a line
// CCSDS_OMM_VERS, or a repeated key) or at the end of the text.  COMMENT
// lines and blank lines are skipped.
std::vector<Record> omm_kvn(const char* text, size_t len) {
  std::vector<Record> recs;
  Record cur;
  const char* end = text + len;
  const char* p = text;
  while (p < end) {
    Span s;
    p = next_line(p, end, &s);
    const char* b = s.b;
    const char* e = s.e;
    trim(b, e);
    if (b == e) continue;
    if (e - b >= 7 && memcmp(b, "COMMENT", 7) == 0) continue;
    const char* eq = static_cast<const char*>(memchr(b, '=', size_t(e - b)));
    if (!eq) continue;
    KV kv{b, eq, eq + 1, e};
    trim(kv.kb, kv.ke);
    // KVN values may carry a unit in brackets: "MEAN_MOTION = 15.1 [rev/day]"
    const char* br = static_cast<const char*>(memchr(kv.vb, '[', size_t(kv.ve - kv.vb)));
    if (br) kv.ve = br;
    trim(kv.vb, kv.ve);
    const bool starts = key_is(kv, "CCSDS_OMM_VERS");
    bool repeat = false;
    for (const KV& o : cur)
      if (size_t(o.ke - o.kb) == size_t(kv.ke - kv.kb) && memcmp(o.kb, kv.kb, size_t(kv.ke - kv.kb)) == 0) {
        repeat = true;
        break;
      }
    if ((starts || repeat) && !cur.empty()) {
      recs.push_back(std::move(cur));
      cur.clear();
    }
    cur.push_back(kv);
  }
  if (!cur.empty()) recs.push_back(std::move(cur));
  return recs;
}

// CSV: a header line of field names, then one record per line (fields split
// at commas; quoted fields may hold commas).
void csv_split(const char* b, const char* e, std::vector<Span>* out) {
  out->clear();
  const char* p = b;
  while (true) {
    const char* q = p;
    bool quoted = false;
    while (q < e && (quoted || *q != ',')) {
      if (*q == '"') quoted = !quoted;
      ++q;
    }
    out->push_back(Span{p, q});
    if (q >= e) break;
    p = q + 1;
  }
}

std::vector<Record> omm_csv(const char* text, size_t len) {
  std::vector<Record> recs;
  const char* end = text + len;
  const char* p = text;
  std::vector<Span> head, cells;
  bool have_head = false;
  while (p < end) {
    Span s;
    p = next_line(p, end, &s);
    const char* b = s.b;
    const char* e = s.e;
    trim(b, e);
    if (b == e) continue;
    if (!have_head) {
      csv_split(b, e, &head);
      for (Span& h : head) unquote(h.b, h.e);
      have_head = true;
      continue;
    }
    csv_split(b, e, &cells);
    Record r;
    for (size_t k = 0; k < head.size() && k < cells.size(); ++k) r.push_back(KV{head[k].b, head[k].e, cells[k].b, cells[k].e});
    recs.push_back(std::move(r));
  }
  return recs;
}

// JSON: an array of flat objects {"KEY": value, ...} with string or number
// values (nested values are skipped as text up to the matching bracket).
const char* json_ws(const char* p, const char* e) {
  while (p < e && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
  return p;
}

const char* json_string(const char* p, const char* e, const char** sb, const char** se) {
  // p at the opening quote; escapes are kept verbatim (keys and values here need none)
  ++p;
  *sb = p;
  while (p < e && *p != '"') p += (*p == '\\' && p + 1 < e) ? 2 : 1;
  *se = p;
  return p < e ? p + 1 : e;
}

bool omm_json(const char* text, size_t len, std::vector<Record>* recs) {
  const char* e = text + len;
  const char* p = json_ws(text, e);
  bool array = p < e && *p == '[';
  if (array) p = json_ws(p + 1, e);
  while (p < e && *p == '{') {
    Record r;
    p = json_ws(p + 1, e);
    while (p < e && *p != '}') {
      if (*p != '"') return false;
      KV kv;
      p = json_ws(json_string(p, e, &kv.kb, &kv.ke), e);
      if (p >= e || *p != ':') return false;
      p = json_ws(p + 1, e);
      if (p < e && *p == '"') {
        p = json_string(p, e, &kv.vb, &kv.ve);
      } else if (p < e && (*p == '{' || *p == '[')) {
        int depth = 0;
        kv.vb = p;
        for (; p < e; ++p) {
          if (*p == '{' || *p == '[') ++depth;
          else if (*p == '}' || *p == ']') { if (--depth == 0) { ++p; break; } }
        }
        kv.ve = p;
      } else {
        kv.vb = p;
        while (p < e && *p != ',' && *p != '}') ++p;
        kv.ve = p;
      }
      r.push_back(kv);
      p = json_ws(p, e);
      if (p < e && *p == ',') p = json_ws(p + 1, e);
    }
    if (p >= e) return false;
    recs->push_back(std::move(r));
    p = json_ws(p + 1, e);
    if (p < e && *p == ',') p = json_ws(p + 1, e);
  }
  p = array && p < e && *p == ']' ? json_ws(p + 1, e) : p;
  return p == e;
}

bool omm_records(const char* text, size_t len, int format, std::vector<Record>* recs) {
  switch (format) {
    case SGP4_TEXT_OMM_KVN: *recs = omm_kvn(text, len); return true;
    case SGP4_TEXT_OMM_CSV: *recs = omm_csv(text, len); return true;
    case SGP4_TEXT_OMM_JSON: return omm_json(text, len, recs);
  }
  return false;
}

void store(const Fields& f, int64_t i, int64_t n, const double ref[2], double* elem, int64_t* satnum,
           int32_t* status) {
  elem[0 * n + i] = f.no_kozai;
  elem[1 * n + i] = f.ecco;
  elem[2 * n + i] = f.inclo;
  elem[3 * n + i] = f.nodeo;
  elem[4 * n + i] = f.argpo;
  elem[5 * n + i] = f.mo;
  elem[6 * n + i] = f.bstar;
  elem[7 * n + i] = (f.jd_whole - ref[0]) + (f.jd_frac - ref[1]);
  if (satnum) satnum[i] = f.satnum;
  if (status) status[i] = f.status;
}

constexpr double kJ2000[2] = {2451545.0, 0.0};

int text_count(const char* text, size_t len, int format, int64_t* n_out) {
  *n_out = 0;
  if (!text && len) return SGP4_E_ARG;
  if (format == SGP4_TEXT_TLE) {
    *n_out = int64_t(tle_records(text, len, 0).size());
    return SGP4_OK;
  }
  std::vector<Record> recs;
  if (format < SGP4_TEXT_OMM_KVN || format > SGP4_TEXT_OMM_JSON) return SGP4_E_ARG;
  if (!omm_records(text, len, format, &recs)) return SGP4_E_ARG;
  *n_out = int64_t(recs.size());
  return SGP4_OK;
}

int text_parse(const char* text, size_t len, int format, int64_t n, const double* ref_jd, double* elem,
               int64_t* satnum, int32_t* status, int threads) {
  if ((!text && len) || (n > 0 && !elem)) return SGP4_E_ARG;
  const double* ref = ref_jd ? ref_jd : kJ2000;
  if (!std::isfinite(ref[0]) || !std::isfinite(ref[1])) return SGP4_E_ARG;
  if (format == SGP4_TEXT_TLE) {
    const std::vector<const char*> recs = tle_records(text, len, threads);
    if (int64_t(recs.size()) != n) return SGP4_E_SIZE;
    const char* end = text + len;
    auto work = [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        Span s1, s2;
        const char* q = next_line(recs[size_t(i)], end, &s1);
        next_line(q, end, &s2);
        Fields f;
        parse_tle(s1.b, s2.b, &f);
        store(f, i, n, ref, elem, satnum, status);
      }
    };
    const int parts = worker_count(threads, len);
    if (parts <= 1 || n < 4096) {
      work(0, n);
    } else {
      run_parts(parts, [&](int k) { work(n * k / parts, n * (k + 1) / parts); });
    }
    return SGP4_OK;
  }
  if (format < SGP4_TEXT_OMM_KVN || format > SGP4_TEXT_OMM_JSON) return SGP4_E_ARG;
  std::vector<Record> recs;
  if (!omm_records(text, len, format, &recs)) return SGP4_E_ARG;
  if (int64_t(recs.size()) != n) return SGP4_E_SIZE;
  for (int64_t i = 0; i < n; ++i) {
    Fields f;
    omm_fields(recs[size_t(i)], &f);
    store(f, i, n, ref, elem, satnum, status);
  }
  return SGP4_OK;
}

}  // namespace

extern "C" {

// Host allocations and worker threads may fail; no exception crosses the C ABI.
int sgp4_text_count(const char* text, size_t len, int format, int64_t* n_out) {
  if (!n_out) return SGP4_E_ARG;
  try {
    return text_count(text, len, format, n_out);
  } catch (...) {
    *n_out = 0;
    return SGP4_E_HOST;
  }
}

int sgp4_text_parse(const char* text, size_t len, int format, int64_t n, const double* ref_jd, double* elem,
                    int64_t* satnum, int32_t* status, int threads) {
  if (n < 0) return SGP4_E_SIZE;
  try {
    return text_parse(text, len, format, n, ref_jd, elem, satnum, status, threads);
  } catch (...) {
    return SGP4_E_HOST;
  }
}

}  // extern "C"
