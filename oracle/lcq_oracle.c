/*
 * lcq_oracle.c -- plain single-threaded CPU oracle of the guaranteed-error-
 * bound quantizers of Fallin & Burtscher (CoDaC'24).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no
 * code with the HIP library.
 *
 * The method is an encoding with free choices (which bin, when to fall back),
 * so this file walks the algorithm's steps in the paper's order, one value at
 * a time, with every free choice fixed the same way the library fixes it:
 *
 *   1. derive the field's parameters from the user's bound          (sec. 2.1)
 *   2. per value: special values are stored losslessly         (sec. 2.2, 3.1)
 *   3.            bin: ABS/NOA round x/(2e); REL rounds an approximate
 *                 log2 of |x| (sec. 2.2; the log2 of sec. 3.2)
 *   4.            bin range check done without abs() on INT_MIN     (sec. 3.3)
 *   5.            reconstruct exactly as the decoder will       (sec. 3.1, 3.2)
 *   6.            verify the bound on that reconstruction; on failure store
 *                 the value losslessly ("double-checking", sec. 3.1)
 *   7. outliers go to a separate list in input order, a sentinel code marks
 *      their place (the separate-list layout the paper contrasts with its
 *      in-line one, sec. 3.1)
 *
 * The two ablations of sec. 6 are extra quantizer codes: ABS_UNCHECKED
 * skips step 6 (the double-check), REL_LIBM uses the C library's log2 and
 * exp2 for step 3 / step 5 and for the log-space bin width.
 *
 * Parity unpinned: the REL_LIBM codes.  The host C library and the GPU's
 * math library round log2 / exp2 apart (that disagreement is the paper's
 * point in sec. 3.2), so no test expects GPU codes equal to these; they are
 * pinned only at exact powers of two (bin rint(k * inv)) and through the
 * bound, which the double-check still enforces.
 *
 * Compiled with -ffp-contract=off and no fast-math (sec. 3.2: no FMA, only
 * IEEE-754 operations), SSE arithmetic, round-to-nearest-even.
 *
 * Stream layout (little-endian):
 *   [0,64)          header: u32 magic "LCQ1", u8 version=1, u8 dtype,
 *                   u8 quantizer, u8 log2(CHUNK)=10, u64 n, u64 n_outliers,
 *                   f64 eb as passed, then step, bound, aux0, aux1 as raw
 *                   bits of the field type zero-extended to 64 bits
 *   [64, 64+4n)     int32 code per value (SENT = INT32_MIN marks an outlier)
 *   ct  = align16(64+4n):    u64 per CHUNK of values: outliers before it
 *   out = align16(ct + 8*C): raw bits of each outlier, in input order
 *   total size = out + n_outliers * sizeof(T); every padding byte is zero
 */
#include "lcq_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <xmmintrin.h>

#define CHUNK 1024u
#define LOG2_CHUNK 10u
#define SENT ((int32_t)INT32_MIN)
#define MAXBIN 1073741824.0 /* 2^30: valid bins are -(2^30-1) .. 2^30-1 */
#define MAGIC 0x3151434Cu   /* bytes 'L','C','Q','1' */

/* ---------------------------------------------------------------- bits --- */
static uint32_t bits32(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
static float from32(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }
static uint64_t bits64(double x) { uint64_t u; memcpy(&u, &x, 8); return u; }
static double from64(uint64_t u) { double x; memcpy(&x, &u, 8); return x; }

static void put_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

static uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }

/* The arithmetic below must be IEEE-754 binary32/binary64 with round-to-
 * nearest-even and subnormals kept (sec. 3.2).  MXCSR: RC bits 13-14 = 0,
 * FTZ bit 15 = 0, DAZ bit 6 = 0. */
static int fpenv_ok(void) {
  unsigned csr = _mm_getcsr();
  return (csr & ((3u << 13) | (1u << 15) | (1u << 6))) == 0;
}

/* ------------------------------------------------------------ layout ----- */
static uint64_t n_chunks(uint64_t n) { return (n + CHUNK - 1) / CHUNK; }
static uint64_t ct_offset(uint64_t n) { return align16(64 + 4 * n); }
static uint64_t out_offset(uint64_t n) { return align16(ct_offset(n) + 8 * n_chunks(n)); }

uint64_t orc_max_stream_bytes(int dtype, uint64_t n) {
  uint64_t s = dtype == ORC_F64 ? 8 : 4;
  return out_offset(n) + s * n;
}

/* ------------------------------------------- section 3.2 approximations -- */
/* Approximate log2 of a non-negative float (Mitchell's piecewise-linear
 * log2).  With E the biased exponent field and F the fraction field, the
 * value 1.F is rebuilt as a float in [1,2) and the de-biased exponent minus
 * one is added, in float arithmetic: 1.F + (E - 128).  The sign bit is
 * ignored. */
static float log2approx_f32(float a) {
  uint32_t u = bits32(a);
  uint32_t E = (u >> 23) & 0xFFu;
  uint32_t F = u & 0x007FFFFFu;
  float one_dot_f = from32((127u << 23) | F);
  float e_minus = (float)((int32_t)E - 128);
  return one_dot_f + e_minus;
}

static double log2approx_f64(double a) {
  uint64_t u = bits64(a);
  uint64_t E = (u >> 52) & 0x7FFu;
  uint64_t F = u & 0x000FFFFFFFFFFFFFull;
  double one_dot_f = from64((1023ull << 52) | F);
  double e_minus = (double)((int64_t)E - 1024);
  return one_dot_f + e_minus;
}

/* Approximate 2^y, the inverse of the above: t = y + 127 re-biases; its
 * integer part k is the exponent field; t - (k - 1) lies in [1,2) and its
 * fraction bits become the fraction field.  t is first clamped to
 * [0, 255] (NaN -> 0) so the conversion to int is always defined; every
 * code the encoder emits already lies inside that range. */
static float pow2approx_f32(float y) {
  float t = y + 127.0f;
  if (!(t >= 0.0f)) t = 0.0f;
  if (t > 255.0f) t = 255.0f;
  int32_t k = (int32_t)t;
  float g = t - (float)(k - 1);
  return from32(((uint32_t)k << 23) | (bits32(g) & 0x007FFFFFu));
}

static double pow2approx_f64(double y) {
  double t = y + 1023.0;
  if (!(t >= 0.0)) t = 0.0;
  if (t > 2047.0) t = 2047.0;
  int64_t k = (int64_t)t;
  double g = t - (double)(k - 1);
  return from64(((uint64_t)k << 52) | (bits64(g) & 0x000FFFFFFFFFFFFFull));
}

void orc_log2approx_f32(const float *in, float *out, uint64_t n) {
  for (uint64_t i = 0; i < n; i++) out[i] = log2approx_f32(in[i]);
}
void orc_pow2approx_f32(const float *in, float *out, uint64_t n) {
  for (uint64_t i = 0; i < n; i++) out[i] = pow2approx_f32(in[i]);
}
void orc_log2approx_f64(const double *in, double *out, uint64_t n) {
  for (uint64_t i = 0; i < n; i++) out[i] = log2approx_f64(in[i]);
}
void orc_pow2approx_f64(const double *in, double *out, uint64_t n) {
  for (uint64_t i = 0; i < n; i++) out[i] = pow2approx_f64(in[i]);
}

/* ------------------------------------------------ parameter derivation --- */
/* Largest float not above the positive double v (the user's bound is a
 * decimal double; rounding it down keeps the guarantee for that value). */
static float round_down_f32(double v) {
  float t = (float)v;
  if ((double)t > v) t = nextafterf(t, -INFINITY);
  return t;
}

/* Exact test of c*(1+eps) <= eps for 0 < eps < 1 and c > 0.  For c in
 * [eps/2, eps] the difference eps - c is exact (Sterbenz) and c*eps is exact
 * in binary128 (106 significant bits), so the comparison is exact. */
static int quot_le(double c, double eps) {
  if (c > eps) return 0;
  if (c < 0.5 * eps) return 1;
  double d = eps - c;
  return (__float128)c * (__float128)eps <= (__float128)d;
}

/* Largest double not above eps/(1+eps). */
static double rel_low_double(double eps) {
  double c = eps / (1.0 + eps);
  while (!quot_le(c, eps)) c = nextafter(c, 0.0);
  while (quot_le(nextafter(c, INFINITY), eps)) c = nextafter(c, INFINITY);
  return c;
}

typedef struct {
  int q;
  int degenerate;
  double step, inv, bound, aux0, aux1, lambda; /* f64 fields */
  float stepf, invf, boundf, aux0f, aux1f, lambdaf;
} params_t;

/* NOA range (sec. 2.1.3): smallest and largest finite value; -0 counts as
 * +0 so the result does not depend on visiting order. */
static void noa_range_f32(const float *x, uint64_t n, float *lo, float *hi) {
  float l = INFINITY, h = -INFINITY;
  for (uint64_t i = 0; i < n; i++) {
    float v = x[i];
    if (!isfinite(v)) continue;
    if (v == 0.0f) v = 0.0f;
    if (v < l) l = v;
    if (v > h) h = v;
  }
  *lo = l; *hi = h;
}

static void noa_range_f64(const double *x, uint64_t n, double *lo, double *hi) {
  double l = INFINITY, h = -INFINITY;
  for (uint64_t i = 0; i < n; i++) {
    double v = x[i];
    if (!isfinite(v)) continue;
    if (v == 0.0) v = 0.0;
    if (v < l) l = v;
    if (v > h) h = v;
  }
  *lo = l; *hi = h;
}

/* Parameters of a float32 field; NOA takes its range (lo, hi) from the
 * caller. */
static int derive_f32_range(int q, double eb, float lo, float hi, params_t *p) {
  memset(p, 0, sizeof *p);
  p->q = q;
  if (q == ORC_ABS || q == ORC_ABS_UNCHECKED) {
    /* sec. 2.2: bins of width 2e, value -> nearest bin centre */
    float e = round_down_f32(eb);
    p->boundf = e;
    p->stepf = e + e;
    p->invf = 1.0f / p->stepf;
  } else if (q == ORC_REL || q == ORC_REL_LIBM) {
    /* Upper side |x'| <= |x|(1+eb) is checked against eh = RD(eb), the
     * lower side |x'| >= |x|/(1+eb) against el = RD(eb/(1+eb)) (sec. 2.1.2,
     * the second, stricter form).  Bins of width 2*lambda in approximate-
     * log2 space with lambda = log2approx(1 + eh) (the library-log2
     * ablation: lambda = log2(1 + eh)). */
    float eh = round_down_f32(eb);
    float el = round_down_f32(rel_low_double(eb));
    float lam = q == ORC_REL_LIBM ? log2f(1.0f + eh) : log2approx_f32(1.0f + eh);
    p->boundf = eh;
    p->aux0f = el;
    p->lambdaf = lam;
    p->stepf = lam + lam;
    p->invf = 1.0f / p->stepf;
  } else {
    /* sec. 2.1.3: bound eb * R with R = max - min; each rounded step is
     * followed by one step down so that ebR <= eb * R holds exactly. */
    float r = hi - lo;
    if (r == INFINITY) r = 3.40282346638528859812e+38f;
    if (r > 0.0f) r = nextafterf(r, 0.0f);
    float b = round_down_f32(eb) * r;
    float ebr = b;
    if (b > 0.0f) ebr = nextafterf(b, 0.0f);
    p->aux0f = lo;
    p->aux1f = hi;
    if (ebr > 0.0f) {
      p->boundf = ebr;
      p->stepf = ebr + ebr;
      p->invf = 1.0f / p->stepf;
    } else {
      p->degenerate = 1;
      p->boundf = 0.0f;
      p->stepf = 0.0f;
      p->invf = 0.0f;
    }
  }
  return ORC_OK;
}

static int derive_f64_range(int q, double eb, double lo, double hi, params_t *p) {
  memset(p, 0, sizeof *p);
  p->q = q;
  if (q == ORC_ABS || q == ORC_ABS_UNCHECKED) {
    double e = eb;
    p->bound = e;
    p->step = e + e;
    p->inv = 1.0 / p->step;
  } else if (q == ORC_REL || q == ORC_REL_LIBM) {
    double eh = eb;
    double el = rel_low_double(eb);
    double lam = q == ORC_REL_LIBM ? log2(1.0 + eh) : log2approx_f64(1.0 + eh);
    p->bound = eh;
    p->aux0 = el;
    p->lambda = lam;
    p->step = lam + lam;
    p->inv = 1.0 / p->step;
  } else {
    double r = hi - lo;
    if (r == INFINITY) r = 1.79769313486231570815e+308;
    if (r > 0.0) r = nextafter(r, 0.0);
    double b = eb * r;
    double ebr = b;
    if (b > 0.0) ebr = nextafter(b, 0.0);
    p->aux0 = lo;
    p->aux1 = hi;
    if (ebr > 0.0) {
      p->bound = ebr;
      p->step = ebr + ebr;
      p->inv = 1.0 / p->step;
    } else {
      p->degenerate = 1;
      p->bound = 0.0;
      p->step = 0.0;
      p->inv = 0.0;
    }
  }
  return ORC_OK;
}

/* Parameters of a field; NOA first reduces the field's range. */
static int derive_f32(int q, double eb, const float *x, uint64_t n, params_t *p) {
  float lo = 0.0f, hi = 0.0f;
  if (q == ORC_NOA) noa_range_f32(x, n, &lo, &hi);
  return derive_f32_range(q, eb, lo, hi, p);
}

static int derive_f64(int q, double eb, const double *x, uint64_t n, params_t *p) {
  double lo = 0.0, hi = 0.0;
  if (q == ORC_NOA) noa_range_f64(x, n, &lo, &hi);
  return derive_f64_range(q, eb, lo, hi, p);
}

static int is_rel(int q) { return q == ORC_REL || q == ORC_REL_LIBM; }

static int check_args(int q, int dtype, double eb) {
  if (q < ORC_ABS || q > ORC_REL_LIBM) return ORC_ERR_ARG;
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_ERR_ARG;
  if (!(eb > 0.0) || !isfinite(eb)) return ORC_ERR_ARG;
  if (is_rel(q) && !(eb < 1.0)) return ORC_ERR_ARG;
  return ORC_OK;
}

static void export_params(int dtype, const params_t *p, orc_params *o) {
  memset(o, 0, sizeof *o);
  if (dtype == ORC_F32) {
    o->step = bits32(p->stepf);
    o->inv = bits32(p->invf);
    o->bound = bits32(p->boundf);
    o->aux0 = bits32(p->aux0f);
    o->aux1 = bits32(p->aux1f);
    o->lambda = bits32(p->lambdaf);
  } else {
    o->step = bits64(p->step);
    o->inv = bits64(p->inv);
    o->bound = bits64(p->bound);
    o->aux0 = bits64(p->aux0);
    o->aux1 = bits64(p->aux1);
    o->lambda = bits64(p->lambda);
  }
  o->degenerate = p->degenerate;
}

int orc_params_derive(int q, int dtype, double eb, const void *in, uint64_t n,
                      orc_params *out) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  int st = check_args(q, dtype, eb);
  if (st) return st;
  if (q == ORC_NOA && n > 0 && !in) return ORC_ERR_ARG;
  params_t p;
  if (dtype == ORC_F32) derive_f32(q, eb, (const float *)in, n, &p);
  else derive_f64(q, eb, (const double *)in, n, &p);
  export_params(dtype, &p, out);
  return ORC_OK;
}

/* ------------------------------------------------------ one value -------- */
/* Returns 1 if x must be stored losslessly, else 0 with its code in *code. */
static int encode_f32(const params_t *p, float x, int32_t *code) {
  uint32_t u = bits32(x);
  uint32_t E = (u >> 23) & 0xFFu;
  uint32_t F = u & 0x007FFFFFu;

  /* special values: INF/NaN, denormals; REL also zeros (sec. 2.2, 3.1) */
  if (E == 0xFFu) return 1;
  if (E == 0 && F != 0) return 1;
  if (is_rel(p->q) && E == 0) return 1;
  if (p->q == ORC_NOA && p->degenerate) return 1;

  if (is_rel(p->q)) {
    const int libm = p->q == ORC_REL_LIBM;
    float a = from32(u & 0x7FFFFFFFu);
    float lg = libm ? log2f(a) : log2approx_f32(a);
    float qf = rintf(lg * p->invf);
    /* sec. 3.3: two one-sided range tests, here on the float so that no
     * out-of-range float-to-int conversion ever happens */
    if (!(qf > -(float)MAXBIN && qf < (float)MAXBIN)) return 1;
    int32_t b = (int32_t)qf;
    float rec = libm ? exp2f((float)b * p->stepf) : pow2approx_f32((float)b * p->stepf);
    /* sec. 3.1 double-check, against the sec. 2.1.2 range */
    int ok;
    if (rec >= a) ok = (rec - a) < (p->boundf * a);
    else ok = (a - rec) < (p->aux0f * a);
    if (!ok) return 1;
    *code = (int32_t)(((uint32_t)b << 1) | (u >> 31));
    return 0;
  }

  float qf = rintf(x * p->invf);
  if (!(qf > -(float)MAXBIN && qf < (float)MAXBIN)) return 1;
  int32_t b = (int32_t)qf;
  float rec = (float)b * p->stepf;
  if (p->q != ORC_ABS_UNCHECKED && !(fabsf(x - rec) <= p->boundf)) return 1;
  *code = b;
  return 0;
}

static int encode_f64(const params_t *p, double x, int32_t *code) {
  uint64_t u = bits64(x);
  uint64_t E = (u >> 52) & 0x7FFu;
  uint64_t F = u & 0x000FFFFFFFFFFFFFull;

  if (E == 0x7FFu) return 1;
  if (E == 0 && F != 0) return 1;
  if (is_rel(p->q) && E == 0) return 1;
  if (p->q == ORC_NOA && p->degenerate) return 1;

  if (is_rel(p->q)) {
    const int libm = p->q == ORC_REL_LIBM;
    double a = from64(u & 0x7FFFFFFFFFFFFFFFull);
    double lg = libm ? log2(a) : log2approx_f64(a);
    double qd = rint(lg * p->inv);
    if (!(qd > -MAXBIN && qd < MAXBIN)) return 1;
    int32_t b = (int32_t)qd;
    double rec = libm ? exp2((double)b * p->step) : pow2approx_f64((double)b * p->step);
    int ok;
    if (rec >= a) ok = (rec - a) < (p->bound * a);
    else ok = (a - rec) < (p->aux0 * a);
    if (!ok) return 1;
    *code = (int32_t)(((uint32_t)b << 1) | (uint32_t)(u >> 63));
    return 0;
  }

  double qd = rint(x * p->inv);
  if (!(qd > -MAXBIN && qd < MAXBIN)) return 1;
  int32_t b = (int32_t)qd;
  double rec = (double)b * p->step;
  if (p->q != ORC_ABS_UNCHECKED && !(fabs(x - rec) <= p->bound)) return 1;
  *code = b;
  return 0;
}

/* Decoder side of one non-sentinel code. */
static float decode_f32(int q, float step, int32_t c) {
  if (is_rel(q)) {
    int32_t sgn = c & 1;
    int32_t b = (c - sgn) / 2; /* exact: c - sgn is even */
    float a = q == ORC_REL_LIBM ? exp2f((float)b * step) : pow2approx_f32((float)b * step);
    return from32(bits32(a) | ((uint32_t)sgn << 31));
  }
  return (float)c * step;
}

static double decode_f64(int q, double step, int32_t c) {
  if (is_rel(q)) {
    int32_t sgn = c & 1;
    int32_t b = (c - sgn) / 2;
    double a = q == ORC_REL_LIBM ? exp2((double)b * step) : pow2approx_f64((double)b * step);
    return from64(bits64(a) | ((uint64_t)sgn << 63));
  }
  return (double)c * step;
}

/* --------------------------------------------------------- quantize ------ */
int orc_quantize(int q, int dtype, double eb, const void *in, uint64_t n,
                 void *stream, uint64_t cap, uint64_t *stream_bytes) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  int st = check_args(q, dtype, eb);
  if (st) return st;
  if (!stream || !stream_bytes || (n > 0 && !in)) return ORC_ERR_ARG;
  if (n > (1ull << 38)) return ORC_ERR_ARG;
  if (cap < orc_max_stream_bytes(dtype, n)) return ORC_ERR_CAPACITY;

  const uint64_t s = dtype == ORC_F64 ? 8 : 4;
  uint8_t *S = (uint8_t *)stream;
  const uint64_t ct = ct_offset(n), out = out_offset(n);

  params_t p;
  if (dtype == ORC_F32) derive_f32(q, eb, (const float *)in, n, &p);
  else derive_f64(q, eb, (const double *)in, n, &p);

  uint64_t k = 0; /* outliers so far */
  for (uint64_t i = 0; i < n; i++) {
    if (i % CHUNK == 0) put_u64(S + ct + 8 * (i / CHUNK), k);
    int32_t code = 0;
    int outlier;
    if (dtype == ORC_F32) {
      float x;
      memcpy(&x, (const uint8_t *)in + 4 * i, 4);
      outlier = encode_f32(&p, x, &code);
    } else {
      double x;
      memcpy(&x, (const uint8_t *)in + 8 * i, 8);
      outlier = encode_f64(&p, x, &code);
    }
    if (outlier) {
      /* raw bits, never through a float register (keeps NaN payloads) */
      memcpy(S + out + s * k, (const uint8_t *)in + s * i, s);
      k++;
      code = SENT;
    }
    memcpy(S + 64 + 4 * i, &code, 4);
  }

  /* zero padding after the codes and after the chunk table */
  memset(S + 64 + 4 * n, 0, ct - (64 + 4 * n));
  memset(S + ct + 8 * n_chunks(n), 0, out - (ct + 8 * n_chunks(n)));

  orc_params o;
  export_params(dtype, &p, &o);
  memset(S, 0, 64);
  put_u32(S + 0, MAGIC);
  S[4] = 1;
  S[5] = (uint8_t)dtype;
  S[6] = (uint8_t)q;
  S[7] = (uint8_t)LOG2_CHUNK;
  put_u64(S + 8, n);
  put_u64(S + 16, k);
  memcpy(S + 24, &eb, 8);
  put_u64(S + 32, o.step);
  put_u64(S + 40, o.bound);
  put_u64(S + 48, o.aux0);
  put_u64(S + 56, o.aux1);

  *stream_bytes = out + s * k;
  return ORC_OK;
}

/* ------------------------------------------------------- dequantize ------ */
int orc_dequantize(int dtype, const void *stream, uint64_t bytes, void *out_v,
                   uint64_t n) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_ERR_ARG;
  if (!stream || (n > 0 && !out_v)) return ORC_ERR_ARG;
  if (bytes < 64) return ORC_ERR_STREAM;
  const uint8_t *S = (const uint8_t *)stream;
  const uint64_t s = dtype == ORC_F64 ? 8 : 4;

  if (get_u32(S) != MAGIC || S[4] != 1 || S[5] != dtype || S[6] > ORC_REL_LIBM ||
      S[7] != LOG2_CHUNK)
    return ORC_ERR_STREAM;
  if (get_u64(S + 8) != n) return ORC_ERR_STREAM;
  const int q = S[6];
  const uint64_t k = get_u64(S + 16);
  const uint64_t ct = ct_offset(n), out = out_offset(n);
  if (k > n || bytes < out + s * k) return ORC_ERR_STREAM;
  const uint64_t stepbits = get_u64(S + 32);

  uint64_t cursor = 0;
  for (uint64_t i = 0; i < n; i++) {
    if (i % CHUNK == 0 && get_u64(S + ct + 8 * (i / CHUNK)) != cursor)
      return ORC_ERR_STREAM;
    int32_t c;
    memcpy(&c, S + 64 + 4 * i, 4);
    uint8_t *dst = (uint8_t *)out_v + s * i;
    if (c == SENT) {
      if (cursor >= k) return ORC_ERR_STREAM;
      memcpy(dst, S + out + s * cursor, s);
      cursor++;
    } else if (dtype == ORC_F32) {
      float v = decode_f32(q, from32((uint32_t)stepbits), c);
      memcpy(dst, &v, 4);
    } else {
      double v = decode_f64(q, from64(stepbits), c);
      memcpy(dst, &v, 8);
    }
  }
  /* ASAN-CONTROL: dequantize output end */
  if (cursor != k) return ORC_ERR_STREAM;
  return ORC_OK;
}

/* ------------------------------------------------- in-line outlier format --
 * The paper's own layout (section 3.1): outliers are stored in-line with the
 * bin numbers, one word of the field type's width per value, so no scan is
 * needed.  Here a word holds either the value's code (the same int32 code as
 * above, sign-extended to the word) or, for a value stored losslessly, its
 * raw bits; a bitmap with one bit per value tells which.
 *
 *   [0,64)              header: u32 magic "LCQI", u8 version 1, u8 dtype,
 *                       u8 quantizer, u8 0, u64 n, u64 0, f64 eb as passed,
 *                       then step, bound, aux0, aux1 as in the format above
 *   [64, 64 + n*s)      one word per value
 *   fl = align16(64+n*s) ceil(n/8) bytes: bit (i % 8) of byte i/8 set when
 *                       value i is stored raw
 *   total size = fl + ceil(n/8); every padding or unused bit is zero
 */
#define MAGIC_INLINE 0x4951434Cu /* bytes 'L','C','Q','I' */

uint64_t orc_inline_stream_bytes(int dtype, uint64_t n) {
  uint64_t s = dtype == ORC_F64 ? 8 : 4;
  return align16(64 + s * n) + (n + 7) / 8;
}

int orc_quantize_inline(int q, int dtype, double eb, const void *in, uint64_t n,
                        void *stream, uint64_t cap, uint64_t *stream_bytes) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  if (q > ORC_NOA) return ORC_ERR_ARG; /* the ablations use the list layout only */
  int st = check_args(q, dtype, eb);
  if (st) return st;
  if (!stream || !stream_bytes || (n > 0 && !in)) return ORC_ERR_ARG;
  if (n > (1ull << 38)) return ORC_ERR_ARG;
  const uint64_t total = orc_inline_stream_bytes(dtype, n);
  if (cap < total) return ORC_ERR_CAPACITY;
  const uint64_t s = dtype == ORC_F64 ? 8 : 4;
  uint8_t *S = (uint8_t *)stream;
  const uint64_t fl = align16(64 + s * n);
  memset(S, 0, total);

  params_t p;
  if (dtype == ORC_F32) derive_f32(q, eb, (const float *)in, n, &p);
  else derive_f64(q, eb, (const double *)in, n, &p);

  for (uint64_t i = 0; i < n; i++) {
    int32_t code = 0;
    int raw;
    if (dtype == ORC_F32) {
      float x;
      memcpy(&x, (const uint8_t *)in + 4 * i, 4);
      raw = encode_f32(&p, x, &code);
    } else {
      double x;
      memcpy(&x, (const uint8_t *)in + 8 * i, 8);
      raw = encode_f64(&p, x, &code);
    }
    if (raw) {
      memcpy(S + 64 + s * i, (const uint8_t *)in + s * i, s);
      S[fl + i / 8] |= (uint8_t)(1u << (i % 8));
    } else if (s == 4) {
      memcpy(S + 64 + 4 * i, &code, 4);
    } else {
      int64_t w = code;
      memcpy(S + 64 + 8 * i, &w, 8);
    }
  }

  orc_params o;
  export_params(dtype, &p, &o);
  put_u32(S + 0, MAGIC_INLINE);
  S[4] = 1;
  S[5] = (uint8_t)dtype;
  S[6] = (uint8_t)q;
  S[7] = 0;
  put_u64(S + 8, n);
  put_u64(S + 16, 0);
  memcpy(S + 24, &eb, 8);
  put_u64(S + 32, o.step);
  put_u64(S + 40, o.bound);
  put_u64(S + 48, o.aux0);
  put_u64(S + 56, o.aux1);
  *stream_bytes = total;
  return ORC_OK;
}

int orc_dequantize_inline(int dtype, const void *stream, uint64_t bytes, void *out_v,
                          uint64_t n) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_ERR_ARG;
  if (!stream || (n > 0 && !out_v)) return ORC_ERR_ARG;
  if (bytes < 64) return ORC_ERR_STREAM;
  const uint8_t *S = (const uint8_t *)stream;
  const uint64_t s = dtype == ORC_F64 ? 8 : 4;
  if (get_u32(S) != MAGIC_INLINE || S[4] != 1 || S[5] != dtype || S[6] > ORC_NOA || S[7] != 0)
    return ORC_ERR_STREAM;
  if (get_u64(S + 8) != n || bytes < orc_inline_stream_bytes(dtype, n)) return ORC_ERR_STREAM;
  const int q = S[6];
  const uint64_t fl = align16(64 + s * n);
  const uint64_t stepbits = get_u64(S + 32);
  for (uint64_t i = 0; i < n; i++) {
    uint8_t *dst = (uint8_t *)out_v + s * i;
    if (S[fl + i / 8] & (1u << (i % 8))) {
      memcpy(dst, S + 64 + s * i, s);
      continue;
    }
    int32_t c;
    memcpy(&c, S + 64 + s * i, 4); /* low word (little-endian) */
    if (dtype == ORC_F32) {
      float v = decode_f32(q, from32((uint32_t)stepbits), c);
      memcpy(dst, &v, 4);
    } else {
      double v = decode_f64(q, from64(stepbits), c);
      memcpy(dst, &v, 8);
    }
  }
  return ORC_OK;
}

/* --------------------------------------------- lossless packing stage ----
 * A lossless back-end for the code stream (the paper passes the quantizer's
 * output to further lossless stages of its framework without naming them;
 * this one is defined here).  It rewrites an LCQ1 stream, chunk by chunk of
 * 1024 codes, at the smallest bit width that holds the chunk:
 *
 *   c'_j = code_j, or 0 where code_j is the outlier sentinel
 *   plain mode: z_j = zigzag(c'_j)
 *   delta mode: z_j = zigzag(c'_j - c'_{j-1}), c'_{-1} = 0 (mod 2^32)
 *   zigzag(v) = (v << 1) ^ (v >> 31) on 32-bit two's complement
 *   w = bit length of the largest z_j of the chunk (0..32); the mode with
 *   the smaller w is kept (plain on a tie)
 *
 *   [0,64)            LCQ1 header with magic "LCQP"
 *   [64, 64+8C)       the LCQ1 chunk table, verbatim
 *   ot = align16(64+8C):   u64 offset of each chunk record in the payload,
 *                     C+1 entries (the last is the payload size)
 *   pl = align16(ot + 8(C+1)): records, each starting 16-byte aligned:
 *       16-byte record header: u8 w, u8 mode (0 plain, 1 delta),
 *                     u8 has_bitmap, 13 zero bytes
 *       if has_bitmap: 128 bytes, bit i%8 of byte i/8 set when value i of
 *                     the chunk is an outlier (chunks with outliers only)
 *       ceil(len*w/8) bytes: z_j in bits [j*w, j*w+w), least significant
 *                     bit first; then zeros to the next 16-byte boundary
 *   oo = align16(pl + payload): the k raw outlier words, verbatim
 *   total = oo + k*s; every padding byte is zero
 */
#define MAGIC_PACKED 0x5051434Cu /* bytes 'L','C','Q','P' */

static uint32_t zigzag32(uint32_t v) { return (v << 1) ^ (uint32_t)((int32_t)v >> 31); }
static uint32_t unzigzag32(uint32_t z) { return (z >> 1) ^ (0u - (z & 1u)); }
static unsigned bitlen32(uint32_t v) { unsigned b = 0; while (v) { b++; v >>= 1; } return b; }

static int32_t code_at(const uint8_t *codes, uint64_t i) {
  int32_t c;
  memcpy(&c, codes + 4 * i, 4);
  return c;
}

/* Width, mode and bitmap flag of a chunk of len codes. */
static void pack_plan(const uint8_t *codes, uint64_t len, unsigned *w, unsigned *mode,
                      unsigned *has_bm) {
  uint32_t prev = 0, mp = 0, md = 0;
  *has_bm = 0;
  for (uint64_t j = 0; j < len; j++) {
    const int32_t cj = code_at(codes, j);
    uint32_t c = cj == SENT ? 0u : (uint32_t)cj;
    if (cj == SENT) *has_bm = 1;
    uint32_t zp = zigzag32(c), zd = zigzag32(c - prev);
    if (zp > mp) mp = zp;
    if (zd > md) md = zd;
    prev = c;
  }
  unsigned wp = bitlen32(mp), wd = bitlen32(md);
  *mode = wd < wp;
  *w = *mode ? wd : wp;
}

static uint64_t record_bytes(uint64_t len, unsigned w, unsigned has_bm) {
  return 16 + (has_bm ? 128 : 0) + align16((len * w + 7) / 8);
}

uint64_t orc_pack_max_bytes(int dtype, uint64_t n) {
  uint64_t s = dtype == ORC_F64 ? 8 : 4, C = n_chunks(n);
  uint64_t ot = align16(64 + 8 * C), pl = align16(ot + 8 * (C + 1));
  return align16(pl + C * record_bytes(CHUNK, 32, 1)) + s * n;
}

int orc_pack(int dtype, const void *stream, uint64_t bytes, uint64_t n, void *out_v,
             uint64_t cap, uint64_t *out_bytes) {
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_ERR_ARG;
  if (!stream || !out_v || !out_bytes) return ORC_ERR_ARG;
  const uint8_t *S = (const uint8_t *)stream;
  const uint64_t s = dtype == ORC_F64 ? 8 : 4;
  if (bytes < 64 || get_u32(S) != MAGIC || S[4] != 1 || S[5] != dtype || S[6] > ORC_NOA ||
      S[7] != LOG2_CHUNK || get_u64(S + 8) != n)
    return ORC_ERR_STREAM;
  const uint64_t k = get_u64(S + 16), C = n_chunks(n);
  if (k > n || bytes < out_offset(n) + s * k) return ORC_ERR_STREAM;
  if (cap < orc_pack_max_bytes(dtype, n)) return ORC_ERR_CAPACITY;
  uint8_t *P = (uint8_t *)out_v;
  const uint64_t ot = align16(64 + 8 * C), pl = align16(ot + 8 * (C + 1));
  const uint8_t *codes = S + 64;
  memcpy(P, S, 64);
  put_u32(P, MAGIC_PACKED);
  memcpy(P + 64, S + ct_offset(n), 8 * C);
  memset(P + 64 + 8 * C, 0, ot - (64 + 8 * C));
  memset(P + ot + 8 * (C + 1), 0, pl - (ot + 8 * (C + 1)));
  uint64_t off = 0;
  for (uint64_t c = 0; c < C; c++) {
    const uint64_t b = c * CHUNK, len = n - b < CHUNK ? n - b : CHUNK;
    unsigned w, mode, hb;
    pack_plan(codes + 4 * b, len, &w, &mode, &hb);
    const uint64_t rb = record_bytes(len, w, hb);
    put_u64(P + ot + 8 * c, off);
    uint8_t *R = P + pl + off;
    memset(R, 0, rb);
    R[0] = (uint8_t)w;
    R[1] = (uint8_t)mode;
    R[2] = (uint8_t)hb;
    uint8_t *bits = R + 16 + (hb ? 128 : 0);
    uint32_t prev = 0;
    for (uint64_t j = 0; j < len; j++) {
      const int32_t cj = code_at(codes, b + j);
      const int sent = cj == SENT;
      const uint32_t cv = sent ? 0u : (uint32_t)cj;
      if (sent) R[16 + j / 8] |= (uint8_t)(1u << (j % 8));
      const uint32_t z = zigzag32(mode ? cv - prev : cv);
      prev = cv;
      for (unsigned t = 0; t < w; t++) /* bit t of z goes to stream bit j*w+t */
        if ((z >> t) & 1u) bits[(j * w + t) / 8] |= (uint8_t)(1u << ((j * w + t) % 8));
    }
    off += rb;
  }
  put_u64(P + ot + 8 * C, off);
  const uint64_t oo = align16(pl + off);
  memset(P + pl + off, 0, oo - (pl + off));
  memcpy(P + oo, S + out_offset(n), s * k);
  *out_bytes = oo + s * k;
  return ORC_OK;
}

int orc_unpack(int dtype, const void *packed, uint64_t bytes, uint64_t n, void *out_v,
               uint64_t cap, uint64_t *out_bytes) {
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_ERR_ARG;
  if (!packed || !out_v || !out_bytes) return ORC_ERR_ARG;
  const uint8_t *P = (const uint8_t *)packed;
  const uint64_t s = dtype == ORC_F64 ? 8 : 4, C = n_chunks(n);
  if (bytes < 64 || get_u32(P) != MAGIC_PACKED || P[4] != 1 || P[5] != dtype || P[6] > ORC_NOA ||
      P[7] != LOG2_CHUNK || get_u64(P + 8) != n)
    return ORC_ERR_STREAM;
  const uint64_t k = get_u64(P + 16);
  const uint64_t ot = align16(64 + 8 * C), pl = align16(ot + 8 * (C + 1));
  if (k > n || bytes < pl) return ORC_ERR_STREAM;
  const uint64_t payload = get_u64(P + ot + 8 * C);
  if (payload > bytes - pl) return ORC_ERR_STREAM;
  const uint64_t oo = align16(pl + payload);
  if (oo > bytes || bytes - oo < s * k) return ORC_ERR_STREAM;
  if (cap < out_offset(n) + s * k) return ORC_ERR_CAPACITY;
  uint8_t *S = (uint8_t *)out_v;
  memcpy(S, P, 64);
  put_u32(S, MAGIC);
  memcpy(S + ct_offset(n), P + 64, 8 * C);
  memset(S + 64 + 4 * n, 0, ct_offset(n) - (64 + 4 * n));
  memset(S + ct_offset(n) + 8 * C, 0, out_offset(n) - (ct_offset(n) + 8 * C));
  memcpy(S + out_offset(n), P + oo, s * k);
  for (uint64_t c = 0; c < C; c++) {
    const uint64_t b = c * CHUNK, len = n - b < CHUNK ? n - b : CHUNK;
    const uint64_t off = get_u64(P + ot + 8 * c);
    if (off > payload || payload - off < 16) return ORC_ERR_STREAM;
    const uint8_t *R = P + pl + off;
    const unsigned w = R[0], mode = R[1], hb = R[2];
    if (w > 32 || mode > 1 || hb > 1) return ORC_ERR_STREAM;
    if (payload - off < record_bytes(len, w, hb)) return ORC_ERR_STREAM;
    /* records are contiguous: the next offset must follow this record */
    if (get_u64(P + ot + 8 * (c + 1)) != off + record_bytes(len, w, hb)) return ORC_ERR_STREAM;
    const uint8_t *bits = R + 16 + (hb ? 128 : 0);
    uint32_t prev = 0;
    for (uint64_t j = 0; j < len; j++) {
      uint32_t z = 0;
      for (unsigned t = 0; t < w; t++)
        z |= (uint32_t)((bits[(j * w + t) / 8] >> ((j * w + t) % 8)) & 1u) << t;
      const uint32_t v = unzigzag32(z);
      const uint32_t cv = mode ? prev + v : v;
      prev = cv;
      const int sent = hb && ((R[16 + j / 8] >> (j % 8)) & 1u);
      const int32_t code = sent ? SENT : (int32_t)cv;
      memcpy(S + 64 + 4 * (b + j), &code, 4);
    }
  }
  *out_bytes = out_offset(n) + s * k;
  return ORC_OK;
}

/* ------------------------------------------- chunk-parallel wrapper ------
 * The same quantize / dequantize, with the values split into contiguous
 * ranges of whole CHUNKs, one per thread.  Every per-value step is the one
 * above (encode_f32 / encode_f64, decode_f32 / decode_f64); only the order
 * in which independent values are visited changes, and the few quantities
 * that depend on earlier values are put together serially:
 *   quantize    pass 1 (threads): codes of the range, its outlier count;
 *               serial: exclusive prefix of the counts;
 *               pass 2 (threads): chunk-table entries and raw outlier bits
 *               of the range, from its codes, at its prefix;
 *               serial: padding and header.
 *               NOA: the range's finite min / max per thread, combined
 *               (min / max of finite values, -0 read as +0, do not depend
 *               on the order), then the parameters as for one thread.
 *   dequantize  threads: sentinels per range and each chunk-table entry
 *               against the range's running count; serial: the first entry
 *               of every range against the prefix of the counts and the
 *               total against the header's count (together exactly the
 *               checks of the single-threaded walk); threads: decode.
 * Output bytes and error statuses equal the single-threaded calls'. */
#include <pthread.h>
#include <unistd.h>

#define ORC_MAX_THREADS 256

typedef struct {
  int dtype;
  const params_t *p;
  const uint8_t *in;
  uint8_t *S;
  uint64_t n, b, e; /* values [b, e) */
  uint64_t k;       /* pass 1: outliers of the range; pass 2: first index */
  float lo32, hi32;
  double lo64, hi64;
  int fp_ok;
} qrange_t;

static void *q_range_minmax(void *arg) {
  qrange_t *r = (qrange_t *)arg;
  r->fp_ok = fpenv_ok();
  if (r->dtype == ORC_F32) noa_range_f32((const float *)r->in + r->b, r->e - r->b, &r->lo32, &r->hi32);
  else noa_range_f64((const double *)r->in + r->b, r->e - r->b, &r->lo64, &r->hi64);
  return NULL;
}

static void *q_range_pass1(void *arg) {
  qrange_t *r = (qrange_t *)arg;
  r->fp_ok = fpenv_ok();
  const uint64_t s = r->dtype == ORC_F64 ? 8 : 4;
  uint64_t k = 0;
  for (uint64_t i = r->b; i < r->e; i++) {
    int32_t code = 0;
    int outlier;
    if (r->dtype == ORC_F32) {
      float x;
      memcpy(&x, r->in + 4 * i, 4);
      outlier = encode_f32(r->p, x, &code);
    } else {
      double x;
      memcpy(&x, r->in + 8 * i, 8);
      outlier = encode_f64(r->p, x, &code);
    }
    if (outlier) {
      code = SENT;
      k++;
    }
    memcpy(r->S + 64 + 4 * i, &code, 4);
  }
  (void)s;
  r->k = k;
  return NULL;
}

static void *q_range_pass2(void *arg) {
  qrange_t *r = (qrange_t *)arg;
  const uint64_t s = r->dtype == ORC_F64 ? 8 : 4;
  const uint64_t ct = ct_offset(r->n), out = out_offset(r->n);
  uint64_t k = r->k;
  for (uint64_t i = r->b; i < r->e; i++) {
    if (i % CHUNK == 0) put_u64(r->S + ct + 8 * (i / CHUNK), k);
    int32_t code;
    memcpy(&code, r->S + 64 + 4 * i, 4);
    if (code == SENT) {
      memcpy(r->S + out + s * k, r->in + s * i, s);
      k++;
    }
  }
  return NULL;
}

static int orc_threads(int nthreads) {
  if (nthreads <= 0) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    nthreads = c > 0 ? (int)c : 1;
  }
  return nthreads > ORC_MAX_THREADS ? ORC_MAX_THREADS : nthreads;
}

/* Split [0, n) into at most `want` ranges of whole chunks; returns the
 * number of ranges and fills b[] / e[]. */
static int split_chunks(uint64_t n, int want, uint64_t *b, uint64_t *e) {
  const uint64_t C = n_chunks(n);
  uint64_t parts = (uint64_t)want < C ? (uint64_t)want : C;
  if (parts == 0) parts = 1;
  for (uint64_t t = 0; t < parts; t++) {
    const uint64_t c0 = C * t / parts, c1 = C * (t + 1) / parts;
    b[t] = c0 * CHUNK < n ? c0 * CHUNK : n;
    e[t] = c1 * CHUNK < n ? c1 * CHUNK : n;
  }
  return (int)parts;
}

/* Runs fn over ranges[0..m) on m threads (the calling thread takes the
 * last); returns 0 if every thread started. */
static int run_ranges(void *(*fn)(void *), void *ranges, size_t stride, int m) {
  pthread_t th[ORC_MAX_THREADS];
  int started = 0, ok = 1;
  for (int t = 0; t < m - 1; t++) {
    if (pthread_create(&th[t], NULL, fn, (uint8_t *)ranges + stride * (size_t)t) != 0) {
      ok = 0;
      break;
    }
    started++;
  }
  if (ok) fn((uint8_t *)ranges + stride * (size_t)(m - 1));
  for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
  return ok ? 0 : -1;
}

int orc_threads_used(int nthreads) { return orc_threads(nthreads); }

int orc_quantize_mt(int q, int dtype, double eb, const void *in, uint64_t n,
                    void *stream, uint64_t cap, uint64_t *stream_bytes, int nthreads) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  int st = check_args(q, dtype, eb);
  if (st) return st;
  if (!stream || !stream_bytes || (n > 0 && !in)) return ORC_ERR_ARG;
  if (n > (1ull << 38)) return ORC_ERR_ARG;
  if (cap < orc_max_stream_bytes(dtype, n)) return ORC_ERR_CAPACITY;

  const uint64_t s = dtype == ORC_F64 ? 8 : 4;
  uint8_t *S = (uint8_t *)stream;
  const uint64_t ct = ct_offset(n), out = out_offset(n);
  uint64_t b[ORC_MAX_THREADS], e[ORC_MAX_THREADS];
  const int m = split_chunks(n, orc_threads(nthreads), b, e);
  qrange_t R[ORC_MAX_THREADS];
  memset(R, 0, sizeof R);
  for (int t = 0; t < m; t++) {
    R[t].dtype = dtype;
    R[t].in = (const uint8_t *)in;
    R[t].S = S;
    R[t].n = n;
    R[t].b = b[t];
    R[t].e = e[t];
  }

  params_t p;
  if (q == ORC_NOA) {
    if (run_ranges(q_range_minmax, R, sizeof R[0], m)) return ORC_ERR_ARG;
    if (dtype == ORC_F32) {
      float lo = INFINITY, hi = -INFINITY;
      for (int t = 0; t < m; t++) {
        if (R[t].lo32 < lo) lo = R[t].lo32;
        if (R[t].hi32 > hi) hi = R[t].hi32;
      }
      derive_f32_range(q, eb, lo, hi, &p);
    } else {
      double lo = INFINITY, hi = -INFINITY;
      for (int t = 0; t < m; t++) {
        if (R[t].lo64 < lo) lo = R[t].lo64;
        if (R[t].hi64 > hi) hi = R[t].hi64;
      }
      derive_f64_range(q, eb, lo, hi, &p);
    }
  } else if (dtype == ORC_F32) {
    derive_f32_range(q, eb, 0.0f, 0.0f, &p);
  } else {
    derive_f64_range(q, eb, 0.0, 0.0, &p);
  }
  for (int t = 0; t < m; t++) R[t].p = &p;

  if (run_ranges(q_range_pass1, R, sizeof R[0], m)) return ORC_ERR_ARG;
  for (int t = 0; t < m; t++)
    if (!R[t].fp_ok) return ORC_ERR_FPENV;
  uint64_t k = 0;
  for (int t = 0; t < m; t++) {
    const uint64_t kt = R[t].k;
    R[t].k = k;
    k += kt;
  }
  if (run_ranges(q_range_pass2, R, sizeof R[0], m)) return ORC_ERR_ARG;

  memset(S + 64 + 4 * n, 0, ct - (64 + 4 * n));
  memset(S + ct + 8 * n_chunks(n), 0, out - (ct + 8 * n_chunks(n)));
  orc_params o;
  export_params(dtype, &p, &o);
  memset(S, 0, 64);
  put_u32(S + 0, MAGIC);
  S[4] = 1;
  S[5] = (uint8_t)dtype;
  S[6] = (uint8_t)q;
  S[7] = (uint8_t)LOG2_CHUNK;
  put_u64(S + 8, n);
  put_u64(S + 16, k);
  memcpy(S + 24, &eb, 8);
  put_u64(S + 32, o.step);
  put_u64(S + 40, o.bound);
  put_u64(S + 48, o.aux0);
  put_u64(S + 56, o.aux1);
  *stream_bytes = out + s * k;
  return ORC_OK;
}

typedef struct {
  int dtype, q;
  const uint8_t *S;
  uint8_t *out;
  uint64_t n, b, e, k, stepbits;
  uint64_t sent;   /* sentinels in [b, e) */
  int table_ok;    /* every chunk entry in the range matches its own walk */
  int fp_ok;
} drange_t;

static void *d_range_check(void *arg) {
  drange_t *r = (drange_t *)arg;
  const uint64_t ct = ct_offset(r->n);
  const uint64_t base = r->b < r->e ? get_u64(r->S + ct + 8 * (r->b / CHUNK)) : 0;
  uint64_t cnt = 0;
  int ok = 1;
  for (uint64_t i = r->b; i < r->e; i++) {
    if (i % CHUNK == 0 && get_u64(r->S + ct + 8 * (i / CHUNK)) - base != cnt) ok = 0;
    int32_t c;
    memcpy(&c, r->S + 64 + 4 * i, 4);
    cnt += c == SENT;
  }
  r->sent = cnt;
  r->table_ok = ok;
  return NULL;
}

static void *d_range_decode(void *arg) {
  drange_t *r = (drange_t *)arg;
  r->fp_ok = fpenv_ok();
  const uint64_t s = r->dtype == ORC_F64 ? 8 : 4;
  const uint64_t ct = ct_offset(r->n), out = out_offset(r->n);
  uint64_t cursor = r->b < r->e ? get_u64(r->S + ct + 8 * (r->b / CHUNK)) : 0;
  for (uint64_t i = r->b; i < r->e; i++) {
    int32_t c;
    memcpy(&c, r->S + 64 + 4 * i, 4);
    uint8_t *dst = r->out + s * i;
    if (c == SENT) {
      memcpy(dst, r->S + out + s * cursor, s);
      cursor++;
    } else if (r->dtype == ORC_F32) {
      float v = decode_f32(r->q, from32((uint32_t)r->stepbits), c);
      memcpy(dst, &v, 4);
    } else {
      double v = decode_f64(r->q, from64(r->stepbits), c);
      memcpy(dst, &v, 8);
    }
  }
  return NULL;
}

int orc_dequantize_mt(int dtype, const void *stream, uint64_t bytes, void *out_v, uint64_t n,
                      int nthreads) {
  if (!fpenv_ok()) return ORC_ERR_FPENV;
  if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_ERR_ARG;
  if (!stream || (n > 0 && !out_v)) return ORC_ERR_ARG;
  if (bytes < 64) return ORC_ERR_STREAM;
  const uint8_t *S = (const uint8_t *)stream;
  const uint64_t s = dtype == ORC_F64 ? 8 : 4;
  if (get_u32(S) != MAGIC || S[4] != 1 || S[5] != dtype || S[6] > ORC_REL_LIBM ||
      S[7] != LOG2_CHUNK)
    return ORC_ERR_STREAM;
  if (get_u64(S + 8) != n) return ORC_ERR_STREAM;
  const uint64_t k = get_u64(S + 16);
  if (k > n || bytes < out_offset(n) + s * k) return ORC_ERR_STREAM;

  uint64_t b[ORC_MAX_THREADS], e[ORC_MAX_THREADS];
  const int m = split_chunks(n, orc_threads(nthreads), b, e);
  drange_t R[ORC_MAX_THREADS];
  memset(R, 0, sizeof R);
  for (int t = 0; t < m; t++) {
    R[t].dtype = dtype;
    R[t].q = S[6];
    R[t].S = S;
    R[t].out = (uint8_t *)out_v;
    R[t].n = n;
    R[t].b = b[t];
    R[t].e = e[t];
    R[t].k = k;
    R[t].stepbits = get_u64(S + 32);
  }
  if (run_ranges(d_range_check, R, sizeof R[0], m)) return ORC_ERR_ARG;
  /* the walk's checks: every chunk entry equals the sentinels before it,
   * and all sentinels together equal the outlier count */
  const uint64_t ctab = ct_offset(n);
  uint64_t before = 0;
  for (int t = 0; t < m; t++) {
    if (!R[t].table_ok) return ORC_ERR_STREAM;
    if (R[t].b < R[t].e && get_u64(S + ctab + 8 * (R[t].b / CHUNK)) != before)
      return ORC_ERR_STREAM;
    before += R[t].sent;
  }
  if (before != k) return ORC_ERR_STREAM;
  if (run_ranges(d_range_decode, R, sizeof R[0], m)) return ORC_ERR_ARG;
  for (int t = 0; t < m; t++)
    if (!R[t].fp_ok) return ORC_ERR_FPENV;
  return ORC_OK;
}
