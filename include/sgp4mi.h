/* sgp4mi: SGP4 near-Earth propagation of N satellites x T times on MI355X.
 *
 * The operation is the batched map f(s, t) -> (r, v) of the paper's section
 * 2.2 ("Vectorisation"): for every satellite s (a set of mean elements) and
 * every time t, the SGP4 general-perturbation model (section 2.1: Hoots &
 * Roehrich 1980 as revised by Hoots et al. 2004 and Vallado et al. 2006, with
 * WGS72 constants) gives the TEME position in km and velocity in km/s.
 * Validity problems do not abort the batch: each point carries an error code
 * (section 2.2, "Control Flow").  Element sets with periods of 225 minutes or
 * more take the deep-space model's lunar and solar terms (section 6 names deep
 * space as the variant the paper leaves out), and those of its 12 h and 24 h
 * resonant classes the tesseral resonance, integrated in mean motion and
 * resonant longitude in 720-minute steps from epoch (up to 10 years from
 * epoch; beyond, code 2).
 *
 * Conventions for every call
 *   - Pointers are DEVICE pointers owned by the caller unless marked "host".
 *   - Calls validate their arguments on the host, enqueue work on `stream`
 *     (a hipStream_t; NULL is the default stream) and return without
 *     synchronising, except sgp4_plan_create, which may synchronise.
 *   - A negative return value is an SGP4_E_* error: nothing was enqueued and
 *     nothing was written.  SGP4_E_HIP reports a failed HIP call or launch.
 *   - The library allocates device memory only inside sgp4_plan objects.
 *   - Element array elem is float64 [8][n] row-major (row k at elem + k*n):
 *       0 no_kozai  mean motion (Kozai), rad/min      1 ecco   eccentricity
 *       2 inclo     inclination, rad                  3 nodeo  RAAN, rad
 *       4 argpo     argument of perigee, rad          5 mo     mean anomaly, rad
 *       6 bstar     drag term, 1/earth radii
 *       7 epoch     days after the caller's reference instant (float64; the
 *                   time since epoch is t - 1440*epoch minutes, formed in
 *                   float64, which avoids the float32 epoch error of section 6)
 *   - Times t are float64 minutes after the same reference instant.
 *   - Outputs are component-major SoA: r[c*P + p], v[c*P + p] for c = x, y, z,
 *     err[p], with P points; p = i*T + j on a dense grid, the CSR position on a
 *     ragged one.  r and v are double for SGP4_FP64 and float otherwise.
 *   - Point codes: 0 ok; 1 mean eccentricity outside [-0.001, 1) (or outside
 *     [0, 1) at epoch); 2 recovered mean motion not positive; 3 deep space:
 *     the lunar-solar terms move the eccentricity outside [0, 1]; 4
 *     semi-latus rectum negative; 6 decayed (radius below one earth radius;
 *     the state is still written); 7 not propagated by this call (a
 *     deep-space satellite met by a ragged plan made for a record without
 *     one, see sgp4_plan_create); 8 ragged point that the
 *     offsets place in no satellite's list (malformed offsets given to
 *     sgp4_propagate_ragged without a plan).  Codes 1, 2, 3, 4, 7 and 8 write
 *     NaN to r and v.
 */
#ifndef SGP4MI_H
#define SGP4MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the per-point path.  Section 4 of the paper compares 32- and
 * 64-bit propagation; FP32_MIXED keeps the time since epoch, the secular
 * (n*t and drag) accumulation and the angle reductions in float64 and runs
 * the periodic terms, Kepler solve and state assembly in float32. */
typedef enum { SGP4_FP64 = 0, SGP4_FP32 = 1, SGP4_FP32_MIXED = 2 } sgp4_precision;

enum {
  SGP4_OK = 0,
  SGP4_E_ARG = -1,       /* null pointer or inconsistent argument */
  SGP4_E_SIZE = -2,      /* negative or too large n, T, nnz */
  SGP4_E_OFFSETS = -3,   /* CSR offsets not 0 = o[0] <= ... <= o[n] = nnz */
  SGP4_E_PRECISION = -4, /* unknown precision */
  SGP4_E_HIP = -5,       /* HIP runtime or launch failure */
  SGP4_E_GRAVITY = -6,   /* gravity model rejected */
  SGP4_E_PLAN = -7,      /* plan does not match the call's buffers */
  SGP4_E_WORKSPACE = -8, /* workspace missing or too small */
  SGP4_E_HOST = -9       /* host memory or threads could not be obtained */
};

/* Library version (integer, increases with ABI changes). */
int sgp4_version(void);

/* Human-readable text for a return code (static storage). */
const char* sgp4_strerror(int code);

/* Bytes of the opaque per-satellite constant record for n satellites.  The
 * record layout is internal; allocate at least this much, 256-byte aligned. */
size_t sgp4_consts_bytes(int64_t n);

/* Initialisation (section 3.1: the constants computed from the elements before
 * propagation).  grav (host, nullable) is {mu km^3/s^2, R km, J2, J3, J4};
 * NULL selects WGS72 (section 2.1).  J3 != 0 with J2 == 0 is rejected.
 * elem: device float64 [8][n].  consts: device, sgp4_consts_bytes(n) bytes,
 * written.  sat_flags: device uint8 [n] or NULL; written with bit0 deep space
 * (period of 225 min or more), bit1 simplified drag (perigee below 220 km,
 * and every deep-space set), bit2 invalid elements, bit3 resonant deep space
 * (the 24 h class, or the 12 h class with e >= 0.5).  0 <= n < 2^31.  The deep-space terms need the
 * absolute epoch: sgp4_init takes the epoch row as days after J2000.0
 * (JD 2451545.0, the default reference of sgp4_text_parse). */
int sgp4_init(const double* grav, int64_t n, const double* elem, void* consts, uint8_t* sat_flags, void* stream);
/* As sgp4_init with the reference instant of the epoch row and of the times
 * given: ref_jd (host) {whole, frac} Julian date, NULL = J2000.0 (not finite:
 * SGP4_E_ARG).  Only the deep-space terms (their lunar and solar arguments)
 * depend on it. */
int sgp4_init_ex(const double* grav, const double* ref_jd, int64_t n, const double* elem, void* consts,
                 uint8_t* sat_flags, void* stream);

/* Dense N x T propagation (section 2.2: f applied over satellites x times).
 * t: device float64 [T].  r, v: device [3][n*T] of double (FP64) or float;
 * err: device uint8 [n*T].  consts must come from sgp4_init with the same n.
 * Uses the default launch configuration (see sgp4_propagate_ex). */
int sgp4_propagate(const void* consts, int64_t n, const double* t, int64_t T, int precision, void* r, void* v,
                   uint8_t* err, void* stream);

/* As sgp4_propagate with an explicit launch configuration.  config is the
 * workgroup size (64, 128, 256 or 512), OR'd with any of:
 *   SGP4_CFG_SCALAR_CONSTS  each satellite's constants in scalar registers
 *                           (otherwise vector registers);
 *   SGP4_CFG_PERSISTENT     a fixed grid of compute-units x k workgroups whose
 *                           wavefronts loop over 64-time tiles, with k given
 *                           by SGP4_CFG_PER_CU(k), 1 <= k <= 255;
 *   SGP4_CFG_TILES          one wavefront per 64-time tile of one satellite
 *                           (workgroups of independent wavefronts); needs
 *                           SGP4_CFG_SCALAR_CONSTS and no SGP4_CFG_PERSISTENT
 *                           (else SGP4_E_ARG), and n * ceil(T / 64) < 2^32
 *                           tiles in a grid of fewer than 2^32 lanes (else
 *                           SGP4_E_SIZE);
 *   SGP4_CFG_FLAT           one lane per point in point order, whatever T, so
 *                           short time lists leave no lane idle; each lane
 *                           reads its satellite's constants (vector loads);
 *                           excludes the three flags above (else SGP4_E_ARG)
 *                           and needs ceil(n * T / block) < 2^31 workgroups
 *                           and fewer than 2^32 lanes (else SGP4_E_SIZE).
 * Without TILES, PERSISTENT or FLAT the grid is satellites x time blocks and
 * needs n * block < 2^32 (else SGP4_E_SIZE): a dispatch spans at most 2^32 - 1
 * lanes per grid dimension.
 * The default is FLAT with 256-wide workgroups for T < 64, else TILES with
 * scalar constants (256-wide for FP64, 512 for the float paths) while they
 * fit, else PERSISTENT with 512-wide workgroups, four per compute unit.  Codes are identical for every configuration and
 * states agree to rounding (the Kepler loop ends when all lanes of a
 * wavefront have converged). */
enum { SGP4_CFG_SCALAR_CONSTS = 0x10000, SGP4_CFG_PERSISTENT = 0x20000, SGP4_CFG_TILES = 0x40000,
       SGP4_CFG_FLAT = 0x80000 };
#define SGP4_CFG_PER_CU(k) ((int)(k) << 20)
int sgp4_propagate_ex(const void* consts, int64_t n, const double* t, int64_t T, int precision, void* r, void* v,
                      uint8_t* err, int config, void* stream);

/* Elements straight to states: initialisation and dense n x T propagation in
 * one call, the pipeline jaxsgp4 traces as one function (sections 2.2 and
 * 3.1).  Arguments as sgp4_init (grav, elem, sat_flags) and sgp4_propagate
 * (t, precision, r, v, err).  For T <= 32, or when ws is NULL, one fused
 * launch initialises each workgroup's 64 satellites into on-chip memory and
 * propagates them (no record in device memory; ws untouched); for T > 32 with
 * ws (device, at least sgp4_consts_bytes(n) bytes, else SGP4_E_WORKSPACE) it
 * runs sgp4_init into ws and sgp4_propagate, and ws then holds the records.
 * A fused launch covers T <= 1,048,560 and n * min(T, 16) < 2^32 (else
 * SGP4_E_WORKSPACE when ws is NULL and T is too large, SGP4_E_SIZE when n is).
 * Results equal the two-stage path's: codes identical, states to rounding.
 * n = 0 or T = 0 writes nothing. */
int sgp4_propagate_elements(const double* grav, int64_t n, const double* elem, const double* t, int64_t T,
                            int precision, void* r, void* v, uint8_t* err, uint8_t* sat_flags, void* ws,
                            size_t ws_bytes, void* stream);
/* As sgp4_propagate_elements with the reference instant ref_jd of
 * sgp4_init_ex. */
int sgp4_propagate_elements_ex(const double* grav, const double* ref_jd, int64_t n, const double* elem,
                               const double* t, int64_t T, int precision, void* r, void* v, uint8_t* err,
                               uint8_t* sat_flags, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- screening --
 * Conjunction screening of a dense propagation output (the catalogue-wide use
 * the paper motivates batching with, sections 1 and 6; the paper defines no
 * screening algorithm, so this is the definition): at every sample time k,
 * every pair of satellites i < j whose points are both valid and whose
 * distance is below dist_km is an event (i, j, k, d), where
 *   d^2 = (dx*dx + dy*dy) + dz*dz,  dx = x_j - x_i, ... formed in double from
 * the stored positions (no fused multiply-add), d = sqrt(d^2), and the test is
 * d^2 < dist_km * dist_km (in double).  A point is valid when its three
 * position components are finite and, when err is given, its code is 0 or 6.
 *   r: device [3][n*T], double for SGP4_FP64 else float, laid out as
 *      sgp4_propagate writes it (r[c * n*T + i*T + k]);
 *   err: device uint8 [n*T] or NULL;
 *   pairs: device int32 [capacity][3] (i, j, k), dist: device double
 *      [capacity] (km); events land in unspecified order;
 *   count: device int64, set to the number of events found (which may exceed
 *      capacity: only the first `capacity` found are written).
 *   ws: device scratch of at least sgp4_screen_workspace_bytes(n, T) bytes
 *      (about 12 n T + 4 T n / 4: sorted float x, y and satellite index per
 *      point and bucket offsets per time), else SGP4_E_WORKSPACE (not needed
 *      when n < 2 or T = 0); its contents are not kept.
 * Each time's valid points are bucket-sorted by x (buckets at least D wide)
 * and every point is tested against the rest of its bucket and the next one.
 * For n <= 12288 this happens in on-chip memory, one workgroup per time (a
 * packing pass, then one launch); larger batches keep the buckets in ws (a
 * range reduction, a histogram, a scan per time, a placement and a sweep).
 * dist_km finite and > 0 (else SGP4_E_ARG); n * T within 2^31 * 256 (else
 * SGP4_E_SIZE). */
size_t sgp4_screen_workspace_bytes(int64_t n, int64_t T);
int sgp4_screen(const void* r, int precision, const uint8_t* err, int64_t n, int64_t T, double dist_km,
                int64_t capacity, int32_t* pairs, double* dist, int64_t* count, void* ws, size_t ws_bytes,
                void* stream);
/* As sgp4_screen with the path chosen: mode 0 as sgp4_screen, 1 the on-chip
 * path (n <= 12288, else SGP4_E_SIZE), 2 the device-memory path; both give
 * the same events. */
int sgp4_screen_ex(const void* r, int precision, const uint8_t* err, int64_t n, int64_t T, double dist_km,
                   int64_t capacity, int32_t* pairs, double* dist, int64_t* count, void* ws, size_t ws_bytes,
                   int mode, void* stream);

/* As sgp4_screen (automatic path), for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * allocation): no ws argument, and no device or host allocation in the call.
 * The workspace is a fixed array of SGP4_SCREEN_NOALLOC_BYTES (64 MiB) in the
 * library's code object, one per GPU, held from the library's first use on
 * that GPU until the process ends; its device address is looked up on the
 * first call on each device.  n and T must satisfy
 * sgp4_screen_workspace_bytes(n, T) <= SGP4_SCREEN_NOALLOC_BYTES (about
 * 5.2 million points, e.g. 9,341 satellites x 500 times), else SGP4_E_SIZE.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other host threads) race and give wrong events;
 * calls ordered on one stream are safe (each initialises what it reads).
 * Other arguments and the events found are as for sgp4_screen. */
#define SGP4_SCREEN_NOALLOC_BYTES (64u << 20)
int sgp4_screen_noalloc(const void* r, int precision, const uint8_t* err, int64_t n, int64_t T, double dist_km,
                        int64_t capacity, int32_t* pairs, double* dist, int64_t* count, void* stream);

/* ---------------------------------------------------------------- ingestion --
 * Element-set text to the elements sgp4_init takes, on the host.  Formats:
 *   SGP4_TEXT_TLE       two-line element sets, optionally with a name line
 *                       before each pair (3LE); a record is a line "1 ..."
 *                       of at least 69 columns followed by a line "2 ...";
 *   SGP4_TEXT_OMM_KVN   CCSDS Orbit Mean-elements Messages, "KEY = value"
 *                       lines; a record starts at CCSDS_OMM_VERS or where a
 *                       key repeats;
 *   SGP4_TEXT_OMM_CSV   a header line of OMM keywords, one record per line;
 *   SGP4_TEXT_OMM_JSON  an array of flat objects keyed by OMM keywords.
 * OMM records need EPOCH, MEAN_MOTION, ECCENTRICITY, INCLINATION,
 * RA_OF_ASC_NODE, ARG_OF_PERICENTER, MEAN_ANOMALY and BSTAR (NORAD_CAT_ID
 * optional).  Units in: rev/day, degrees, 1/earth radii; out: rad/min, rad
 * (mean motion divided by 1440 / 2 pi, angles times pi / 180).
 * The epoch row (row 7) is days after the reference ref_jd = {whole, frac}
 * (host, a two-part Julian date; NULL = J2000.0, {2451545.0, 0.0}), computed
 * as (JD0 - ref[0]) + (f - ref[1]) with JD0 the Julian date at 0h of the
 * epoch's day and f its day fraction from the text's digits, so the epoch
 * keeps the text's resolution (1e-8 day for TLE, 1 ns for OMM); section 4 of
 * the paper traces precision loss to a 32-bit Julian-date epoch. */
enum { SGP4_TEXT_TLE = 1, SGP4_TEXT_OMM_KVN = 2, SGP4_TEXT_OMM_CSV = 3, SGP4_TEXT_OMM_JSON = 4 };
/* Per-record status bits: checksum of a TLE line wrong or missing; the two
 * TLE lines carry different catalogue numbers; a field missing or not a
 * number (that record's elements are written as NaN: do not initialise it). */
enum { SGP4_REC_CHECKSUM = 1, SGP4_REC_MISMATCH = 2, SGP4_REC_FIELD = 4 };

/* Number of records in text[0, len) (host memory).  SGP4_E_ARG for an unknown
 * format, a null n_out, or JSON that is not an array of flat objects. */
int sgp4_text_count(const char* text, size_t len, int format, int64_t* n_out);

/* Parse the n records of the text (n must equal sgp4_text_count's result,
 * else SGP4_E_SIZE).  elem: host float64 [8][n], rows as for sgp4_init.
 * satnum: host int64 [n] or NULL (catalogue number, alpha-5 TLE numbers
 * decoded; -1 when absent).  status: host int32 [n] or NULL (SGP4_REC_*
 * bits).  threads: worker threads for TLE text (0 = one per hardware thread,
 * at most 64; texts under ~1 MB use one).  Record order is text order.  Never
 * touches the GPU. */
int sgp4_text_parse(const char* text, size_t len, int format, int64_t n, const double* ref_jd, double* elem,
                    int64_t* satnum, int32_t* status, int threads);

/* Opaque ragged-propagation plan (host object owning device tile tables and
 * a captured HIP graph). */
typedef struct sgp4_plan sgp4_plan;

enum { SGP4_PLAN_AUTOTUNE = 1, SGP4_PLAN_GRAPH = 2 };

/* Ragged propagation: satellite i has times t[offsets[i] .. offsets[i+1]).
 * offsets: device int64 [n+1] with offsets[0] = 0, non-decreasing,
 * offsets[n] = nnz.  t: device float64 [nnz].  r, v: [3][nnz]; err: [nnz].
 * plan: NULL (one launch, a wavefront per 64 consecutive points, whose lanes
 * locate their satellites by a search of the offsets) or a plan created for
 * exactly these buffers (launches its tuned kernel directly, without the
 * graph; the offsets must be those the plan checked).
 * Without a plan the offsets are not read on the host, so malformed offsets
 * are not reported as SGP4_E_OFFSETS.  They never cause a read outside
 * offsets[0..n], t[0..nnz) or the record, nor a write outside the outputs:
 * every point p is propagated with a satellite i whose list holds it
 * (offsets[i] <= p < offsets[i+1]; the only one for well-formed offsets), or,
 * where the search finds none (offsets[0] > p, offsets[n] <= p, or a
 * decreasing step the search lands on), gets code 8 and NaN.  A plan checks
 * the offsets once and returns SGP4_E_OFFSETS for malformed ones. */
int sgp4_propagate_ragged(const void* consts, int64_t n, const int64_t* offsets, const double* t, int64_t nnz,
                          int precision, void* r, void* v, uint8_t* err, const sgp4_plan* plan, void* stream);

/* Build a plan for one ragged batch: copies and checks the offsets (returns
 * SGP4_E_OFFSETS when malformed), builds the tile tables, optionally times
 * the candidate mappings (tiles of <= 64 points of one satellite or flat runs
 * of 64 points; workgroup size; one wavefront per tile or a persistent grid
 * of a given size) and keeps the fastest (SGP4_PLAN_AUTOTUNE), and optionally
 * captures the launch in a HIP graph (SGP4_PLAN_GRAPH).  Without autotuning
 * the plan launches one wavefront per tile in 256-wide workgroups.  The plan
 * also reads the record's satellite flags once: when no satellite is a
 * deep-space one, its tile kernels are those compiled without the deep-space
 * terms (sgp4_plan_describe reports "near_earth": true); should the record
 * later be re-initialised with deep-space satellites under the same plan,
 * their points get code 7 and NaN states (make a new plan).
 * Synchronises `stream`.  Autotuning writes r, v, err. */
int sgp4_plan_create(sgp4_plan** out, const void* consts, int64_t n, const int64_t* offsets, const double* t,
                     int64_t nnz, int precision, void* r, void* v, uint8_t* err, unsigned flags, void* stream);

/* As sgp4_plan_create with a fixed configuration instead of autotuning:
 * mode 0 = tiles of <= 64 points of one satellite per wavefront, 1 = flat
 * runs of 64 points; block = workgroup size (64, 128, 256, 512);
 * waves_per_cu > 0 scales the persistent grid (workgroups = min(needed,
 * compute units * waves_per_cu)), 0 launches one wavefront per tile or chunk
 * (no loop; grids are capped at 2^31 - 1 workgroups, beyond which the
 * wavefronts loop).
 * SGP4_PLAN_AUTOTUNE in flags is ignored; SGP4_PLAN_GRAPH is honoured. */
int sgp4_plan_create_config(sgp4_plan** out, const void* consts, int64_t n, const int64_t* offsets, const double* t,
                            int64_t nnz, int precision, void* r, void* v, uint8_t* err, int mode, int block,
                            int waves_per_cu, unsigned flags, void* stream);

/* Enqueue the plan's launch on `stream` (graph launch when captured). */
int sgp4_plan_launch(const sgp4_plan* plan, void* stream);

/* Describe the plan's chosen configuration into buf (host, NUL-terminated). */
int sgp4_plan_describe(const sgp4_plan* plan, char* buf, size_t len);

/* Free a plan and its device tables.  NULL is accepted. */
void sgp4_plan_destroy(sgp4_plan* plan);

/* Vector-Jacobian product (section 5: gradients of the state with respect to
 * the elements): for a dense n x T batch, gelem[m][i] = sum over j and
 * components c of gr[c][i*T+j] * d r_c/d theta_m + gv[c][i*T+j] * d v_c/d theta_m,
 * theta = (no_kozai, ecco, inclo, nodeo, argpo, mo, bstar) of satellite i.
 * The forward pass is recomputed, not stored.  elem: the device float64
 * [8][n] elements consts was initialised from (the gravity model is read from
 * consts); gr and gv device [3][n*T] of double
 * (FP64) or float (FP32_MIXED), gv nullable (zero).  Points with codes 1, 2,
 * 3, 4, 7 contribute nothing.  Deep-space satellites are not differentiated:
 * their gelem columns are NaN.  gelem: device float64 [7][n].  FP32 is rejected
 * (SGP4_E_PRECISION).  One 256-lane workgroup per satellite: n < 2^24 (else
 * SGP4_E_SIZE). */
int sgp4_vjp(int64_t n, const double* elem, const void* consts, const double* t, int64_t T, int precision,
             const void* gr, const void* gv, double* gelem, void* stream);

/* Vector-Jacobian product over per-satellite time lists (section 5, as
 * sgp4_vjp; the lists are those of sgp4_propagate_ragged: satellite i's
 * points are offsets[i] .. offsets[i+1]-1 at times t[p], an orbit
 * determination's irregular observation times): gelem[m][i] = sum over
 * satellite i's points p and components c of gr[c][p] * d r_c/d theta_m +
 * gv[c][p] * d v_c/d theta_m.  offsets: device int64 [n + 1], non-decreasing
 * from 0 to nnz; each satellite's two offsets are clamped to [0, nnz] (and its
 * end to at least its start), so malformed offsets read nothing outside t, gr
 * and gv (the gradient then covers the clamped lists).  t: device float64
 * [nnz]; gr, gv device [3][nnz] of double (FP64) or float (FP32_MIXED), gv
 * nullable.  Codes, deep space, precisions and limits as for sgp4_vjp; an
 * empty list gives a zero column.  A dense grid given as lists (offsets[i] =
 * i T, t repeated) gives sgp4_vjp's result bit for bit. */
int sgp4_vjp_ragged(int64_t n, const double* elem, const void* consts, const int64_t* offsets, const double* t,
                    int64_t nnz, int precision, const void* gr, const void* gv, double* gelem, void* stream);

/* Jacobian of the dense propagation (section 5: the state's sensitivity to the
 * elements, as for state-transition matrices and covariance propagation):
 * jac[(c * 7 + m) * n*T + i*T + j] = d s_c / d theta_m at satellite i, time j,
 * with s = (r_x, r_y, r_z, v_x, v_y, v_z) (km, km/s) and theta as for sgp4_vjp.
 * jac: device float64 [6][7][n*T], written in full; NaN where the point's
 * code is 1, 2, 3, 4 or 7 and at every point of a deep-space satellite (not
 * differentiated).  elem, consts, t as for sgp4_vjp.  Computed in forward
 * mode: the seven element tangents carried through one pass of the
 * propagation (in two groups of four and three directions), each point's
 * columns stored as they come.  FP32 is rejected (SGP4_E_PRECISION).
 * n < 2^24 as for sgp4_vjp. */
int sgp4_jacobian(int64_t n, const double* elem, const void* consts, const double* t, int64_t T, int precision,
                  double* jac, void* stream);

/* Jacobian over per-satellite time lists (section 5, as sgp4_jacobian; the
 * lists as for sgp4_vjp_ragged): jac[(c * 7 + m) * nnz + p] = d s_c /
 * d theta_m at CSR point p of satellite i (offsets[i] <= p < offsets[i+1]),
 * time t[p].  jac: device float64 [6][7][nnz], NaN as for sgp4_jacobian;
 * every point is written when the offsets are valid (non-decreasing from 0 to
 * nnz); each satellite's offsets are clamped as for sgp4_vjp_ragged, so
 * malformed ones never write outside jac (positions no clamped list covers
 * are then left as they were).  Precisions and limits as for sgp4_jacobian. */
int sgp4_jacobian_ragged(int64_t n, const double* elem, const void* consts, const int64_t* offsets, const double* t,
                         int64_t nnz, int precision, double* jac, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SGP4MI_H */
