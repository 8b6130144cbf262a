/*
 * pmc_oracle.c -- plain, serial CPU oracle for the block codec used inside the
 * multi-component residual loop (Magri & Lindstrom, "A General Framework for
 * Progressive Data Compression and Retrieval", Sec. 4, Alg. 1 and Alg. 2).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  The product path (HIP
 * kernels behind the C-ABI) shares no code, header, table or constant with it.
 *
 * The paper treats the compressor as a black box C(e, tau) / D(y) with a
 * pointwise tolerance (Sec. 4, opening paragraphs).  It names zfp as the
 * block-transform codec with custom bit-plane coding (Sec. 5, compressor list),
 * with one exponent per block and component (Sec. 4.4), independently
 * decodable blocks of 4^d values (Sec. 6.1) and group-testing bit-plane coding
 * (Sec. 2).  The codec below is a zfp-STYLE fixed-accuracy codec written from
 * that description; every constant is a reading frozen in the format
 * specification (version 1), not a copy of any zfp source.
 *
 * Written for obviousness, not speed: bits are set one at a time, every
 * integer operation wraps to the P-bit word explicitly, and floating-point
 * rounding is the single IEEE rounding of a plain C cast.
 *
 * Parity status of each function (see the tests that pin them):
 *   negabinary            pinned: textbook base(-2) digit sum, exhaustive int16
 *   fwd/inv lift          pinned: closed forms (constant, ramp), matrix bound
 *   inverse pass order    pinned: hand-derived single-coefficient inverse
 *   permutation           pinned: sequency order property
 *   minexp                pinned: exact floor(log2 tau) (rationals), incl.
 *                          tau not a power of two and subnormal tau
 *   plane coder           pinned: hand-derived golden encodings, lossless at
 *                          p = P, closed-form bit count
 *   block acceptance      pinned: Eq. (1) bound, monotone error (invariants);
 *                          coded-before-empty and the raw payload (residual
 *                          bits) by hand-derived cases
 *   stream layout         pinned: hand-derived golden streams (one chunk, two
 *                          chunks, a partial block with edge replication)
 *   rates / bit counts    parity unpinned against the paper (the paper prints
 *                          rates only for an unnamed field)
 *
 * Compile: gcc -std=c11 -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 * gcc defines >> on negative signed integers as an arithmetic shift, which is
 * the floor(x / 2) the lifting steps need.
 */
#include <float.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>

/* The float64 dequantisation below forms q * 2^s exactly in long double and
 * rounds once to double; that needs a significand of at least 64 bits (x87
 * extended precision).  Where long double is binary64 the product would be
 * rounded twice, so refuse to build there. */
#if LDBL_MANT_DIG < 64
#error "pmc_oracle.c needs a long double with a 64-bit significand (x87 extended precision)"
#endif

enum { ORC_F32 = 1, ORC_F64 = 2 };
enum {
  ORC_OK = 0, ORC_E_ARG = -1, ORC_E_NOMEM = -3, ORC_E_CORRUPT = -4
};
enum { ORC_EMPTY = 0, ORC_CODED = 1, ORC_RAW = 2 };

#define ORC_CHUNK_BLOCKS 16
#define ORC_HEADER_BYTES 64
#define ORC_MAGIC 0x31434D50u /* "PMC1" */
#define ORC_VERSION 1

typedef struct {
  int dtype;          /* ORC_F32 or ORC_F64 */
  int d;              /* dimensionality 1..3 */
  uint64_t dims[3];   /* nx, ny, nz (x fastest); unused axes are 1 */
} orc_field;

typedef struct {
  uint64_t nempty, ncoded, nraw, nesc, nmiss;
  double linf;          /* max over blocks of the accepted block error */
  uint64_t bits;        /* total payload bits (without chunk padding) */
} orc_stats;

/* ------------------------------------------------------------------ */
/* precision parameters                                               */
/* ------------------------------------------------------------------ */
static int prec_bits(int dtype) { return dtype == ORC_F32 ? 32 : 64; }
static int exp_bits(int dtype) { return dtype == ORC_F32 ? 8 : 11; }
static int exp_bias(int dtype) { return dtype == ORC_F32 ? 127 : 1023; }
static int guard_planes(int d) { return 2 * (d + 1); }
static int block_size(int d) { return d == 1 ? 4 : d == 2 ? 16 : 64; }

/* wrap an integer to a signed P-bit word (two's complement) */
static int64_t wrapP(int64_t v, int P) {
  if (P == 32) return (int64_t)(int32_t)(uint32_t)(uint64_t)v;
  return v;
}
static int64_t addw(int64_t a, int64_t b, int P) {
  return wrapP((int64_t)((uint64_t)a + (uint64_t)b), P);
}
static int64_t subw(int64_t a, int64_t b, int P) {
  return wrapP((int64_t)((uint64_t)a - (uint64_t)b), P);
}
static int64_t dblw(int64_t a, int P) { return wrapP((int64_t)((uint64_t)a << 1), P); }
static int64_t half(int64_t a) { return a >> 1; } /* floor(a / 2) */

/* ------------------------------------------------------------------ */
/* exponent of a value: frexp convention, zero and subnormals -> 2-bias */
/* ------------------------------------------------------------------ */
static int value_expo(double v, int dtype) {
  int bias = exp_bias(dtype);
  int biased;
  if (dtype == ORC_F32) {
    float f = (float)v;
    uint32_t b;
    memcpy(&b, &f, 4);
    biased = (int)((b >> 23) & 0xffu);
  } else {
    uint64_t b;
    memcpy(&b, &v, 8);
    biased = (int)((b >> 52) & 0x7ffu);
  }
  if (biased < 1) biased = 1;
  return biased - bias + 1;
}

/* floor(log2(tau)) for a positive finite tau, exact (frexp is exact) */
int orc_minexp(double tau) {
  int e;
  (void)frexp(tau, &e);
  return e - 1;
}

/* ------------------------------------------------------------------ */
/* 4-point decorrelating lifting transform.                           */
/* It realises, up to the rounding of the halving steps, the          */
/* non-orthogonal basis of the zfp paper:                             */
/*   (1/16) [[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]].          */
/* Derivation: pair sums/differences of (a,d) and (b,c); the two sums */
/* give the DC and the second-order term, the two differences are     */
/* mixed by one halving step and two lifting steps so that            */
/* c1 = (5 t0 + t1) / 8 and c3 = (3 t1 - t0) / 4 with t0 = (a-d)/2,   */
/* t1 = (b-c)/2.                                                      */
/* ------------------------------------------------------------------ */
void orc_fwd_lift4(int64_t v[4], int P) {
  int64_t a = v[0], b = v[1], c = v[2], d = v[3];
  int64_t s0 = half(addw(a, d, P));
  int64_t t0 = subw(a, s0, P);
  int64_t s1 = half(addw(b, c, P));
  int64_t t1 = subw(b, s1, P);
  int64_t c0 = half(addw(s0, s1, P));
  int64_t c2 = subw(s1, c0, P);
  int64_t w = half(addw(t0, t1, P));
  int64_t c3 = subw(t1, half(w), P);
  int64_t c1 = subw(w, half(c3), P);
  v[0] = c0; v[1] = c1; v[2] = c2; v[3] = c3;
}

/* undo the lifting steps of orc_fwd_lift4 in reverse order; the three   */
/* halving steps are undone by doubling, so the pair is exact up to the */
/* parity bits those halvings dropped.                                  */
void orc_inv_lift4(int64_t v[4], int P) {
  int64_t c0 = v[0], c1 = v[1], c2 = v[2], c3 = v[3];
  int64_t w = addw(c1, half(c3), P);
  int64_t t1 = addw(c3, half(w), P);
  int64_t t0 = subw(dblw(w, P), t1, P);
  int64_t s1 = addw(c2, c0, P);
  int64_t s0 = subw(dblw(c0, P), s1, P);
  int64_t a = addw(t0, s0, P);
  int64_t d = subw(dblw(s0, P), a, P);
  int64_t b = addw(t1, s1, P);
  int64_t c = subw(dblw(s1, P), b, P);
  v[0] = a; v[1] = b; v[2] = c; v[3] = d;
}

/* local index l = lx + 4 ly + 16 lz */
static int local_coord(int l, int axis) { return (l >> (2 * axis)) & 3; }

/* separable transform: x lines, then y lines, then z lines */
void orc_fwd_xform(int64_t* q, int d, int P) {
  int B = block_size(d);
  for (int axis = 0; axis < d; axis++) {
    int stride = 1 << (2 * axis);
    for (int l = 0; l < B; l++) {
      if (local_coord(l, axis) != 0) continue; /* l is the start of a line */
      int64_t v[4];
      for (int t = 0; t < 4; t++) v[t] = q[l + t * stride];
      orc_fwd_lift4(v, P);
      for (int t = 0; t < 4; t++) q[l + t * stride] = v[t];
    }
  }
}

/* inverse: z lines, then y, then x (the forward passes in reverse) */
void orc_inv_xform(int64_t* q, int d, int P) {
  int B = block_size(d);
  for (int axis = d - 1; axis >= 0; axis--) {
    int stride = 1 << (2 * axis);
    for (int l = 0; l < B; l++) {
      if (local_coord(l, axis) != 0) continue;
      int64_t v[4];
      for (int t = 0; t < 4; t++) v[t] = q[l + t * stride];
      orc_inv_lift4(v, P);
      for (int t = 0; t < 4; t++) q[l + t * stride] = v[t];
    }
  }
}

/* coefficient order: ascending total sequency lx+ly+lz, ties by l.      */
/* perm[r] = local index of the r-th coded coefficient.  Built here by a */
/* plain selection sort rather than stored as a table.                   */
void orc_perm(int d, int* perm) {
  int B = block_size(d);
  int used[64] = {0};
  for (int r = 0; r < B; r++) {
    int best = -1, bestkey = 1 << 30;
    for (int l = 0; l < B; l++) {
      if (used[l]) continue;
      int key = 0;
      for (int a = 0; a < d; a++) key += local_coord(l, a);
      key = key * 64 + l;
      if (key < bestkey) { bestkey = key; best = l; }
    }
    used[best] = 1;
    perm[r] = best;
  }
}

/* negabinary: u = (q + M) xor M with M = 0xAAAA...; wrapping P-bit */
static uint64_t nb_mask(int P) { return P == 32 ? 0xAAAAAAAAull : 0xAAAAAAAAAAAAAAAAull; }
static uint64_t pmask(int P) { return P == 32 ? 0xFFFFFFFFull : ~0ull; }
uint64_t orc_to_negabinary(int64_t q, int P) {
  uint64_t M = nb_mask(P);
  return (((uint64_t)q + M) ^ M) & pmask(P);
}
int64_t orc_from_negabinary(uint64_t u, int P) {
  uint64_t M = nb_mask(P);
  return wrapP((int64_t)(((u ^ M) - M) & pmask(P)), P);
}

/* ------------------------------------------------------------------ */
/* bit I/O: one bit at a time, LSB-first within little-endian words    */
/* ------------------------------------------------------------------ */
typedef struct { uint8_t* buf; uint64_t cap_bits; uint64_t pos; int overflow; } bitw;
typedef struct { const uint8_t* buf; uint64_t end_bits; uint64_t pos; int overrun; } bitr;

static void put_bit(bitw* w, unsigned bit) {
  if (w->pos >= w->cap_bits) { w->overflow = 1; w->pos++; return; }
  if (bit & 1u) w->buf[w->pos >> 3] |= (uint8_t)(1u << (w->pos & 7));
  w->pos++;
}
static void put_bits(bitw* w, uint64_t value, int count) {
  for (int i = 0; i < count; i++) put_bit(w, (unsigned)((value >> i) & 1u));
}
static unsigned get_bit(bitr* r) {
  if (r->pos >= r->end_bits) { r->overrun = 1; r->pos++; return 0; }
  unsigned b = (r->buf[r->pos >> 3] >> (r->pos & 7)) & 1u;
  r->pos++;
  return b;
}
static uint64_t get_bits(bitr* r, int count) {
  uint64_t v = 0;
  for (int i = 0; i < count; i++) v |= (uint64_t)get_bit(r) << i;
  return v;
}

/* ------------------------------------------------------------------ */
/* embedded bit-plane coder with group testing                        */
/* Planes k = P-1 down to P-p.  n = length of the significant prefix   */
/* (persists across planes).  For each plane: the first n bits go out  */
/* verbatim; then, while n < B, one group-test bit tells whether any   */
/* bit at position >= n is set; if so the bits from n on are sent one  */
/* by one up to and including the next 1, which makes everything up to */
/* it significant.  A 1 at position B-1 reached by such a scan is      */
/* implied and not sent.                                               */
/* ------------------------------------------------------------------ */
static void encode_planes(bitw* w, const uint64_t* u, int B, int P, int p) {
  int n = 0;
  for (int k = P - 1; k >= P - p; k--) {
    for (int j = 0; j < n; j++) put_bit(w, (unsigned)((u[j] >> k) & 1u));
    while (n < B) {
      unsigned any = 0;
      for (int j = n; j < B; j++) any |= (unsigned)((u[j] >> k) & 1u);
      put_bit(w, any);
      if (!any) break;
      for (;;) {
        if (n == B - 1) { n = B; break; } /* implied one */
        unsigned bit = (unsigned)((u[n] >> k) & 1u);
        put_bit(w, bit);
        n++;
        if (bit) break;
      }
    }
  }
}

static void decode_planes(bitr* r, uint64_t* u, int B, int P, int p) {
  for (int j = 0; j < B; j++) u[j] = 0;
  int n = 0;
  for (int k = P - 1; k >= P - p; k--) {
    for (int j = 0; j < n; j++) u[j] |= (uint64_t)get_bit(r) << k;
    while (n < B) {
      if (!get_bit(r)) break;
      for (;;) {
        if (n == B - 1) { u[n] |= 1ull << k; n = B; break; }
        unsigned bit = get_bit(r);
        u[n] |= (uint64_t)bit << k;
        n++;
        if (bit) break;
      }
    }
  }
}

/* exported for tests: code p planes of B words into buf; returns bits */
uint64_t orc_encode_planes(const uint64_t* u, int B, int P, int p, uint8_t* buf, uint64_t cap_bytes) {
  bitw w = {buf, cap_bytes * 8, 0, 0};
  memset(buf, 0, (size_t)cap_bytes);
  encode_planes(&w, u, B, P, p);
  return w.overflow ? ~0ull : w.pos;
}
uint64_t orc_decode_planes(const uint8_t* buf, uint64_t nbits, int B, int P, int p, uint64_t* u) {
  bitr r = {buf, nbits, 0, 0};
  decode_planes(&r, u, B, P, p);
  return r.overrun ? ~0ull : r.pos;
}

/* ------------------------------------------------------------------ */
/* quantisation (block floating point) and dequantisation              */
/* q = trunc(e * 2^(P-2-emax)); the scaling by a power of two is exact */
/* in double for f32 data and for f64 data (|q| < 2^(P-2) < 2^63).     */
/* ------------------------------------------------------------------ */
static int64_t quantize(double e, int emax, int P) {
  return (int64_t)trunc(ldexp(e, P - 2 - emax));
}
/* v = q * 2^(emax-P+2) rounded once to the field type.  For f32 the     */
/* product is exact in double and the cast rounds once.  For f64 the     */
/* product is exact in x87 extended precision (64-bit significand) and   */
/* the cast to double rounds once (including the subnormal range).       */
static double dequantize(int64_t q, int emax, int P, int dtype) {
  if (dtype == ORC_F32) {
    double v = ldexp((double)q, emax - P + 2);
    return (double)(float)v;
  }
  long double v = (long double)q * ldexpl(1.0L, emax - P + 2);
  return (double)v;
}

/* ------------------------------------------------------------------ */
/* field access                                                       */
/* ------------------------------------------------------------------ */
static double load_val(const void* p, uint64_t i, int dtype) {
  return dtype == ORC_F32 ? (double)((const float*)p)[i] : ((const double*)p)[i];
}
static void store_val(void* p, uint64_t i, double v, int dtype) {
  if (dtype == ORC_F32) ((float*)p)[i] = (float)v;
  else ((double*)p)[i] = v;
}
/* field-precision add (RNE in the field type) */
static double add_T(double a, double b, int dtype) {
  if (dtype == ORC_F32) { float fa = (float)a, fb = (float)b; float s = fa + fb; return (double)s; }
  return a + b;
}
static int is_zero_bits(double v) { return v == 0.0; }

typedef struct {
  uint64_t nb[3];
  uint64_t nblocks;
  uint64_t nchunks;
  int B, P;
} geom;

static int make_geom(const orc_field* f, geom* g) {
  if (f->d < 1 || f->d > 3) return ORC_E_ARG;
  if (f->dtype != ORC_F32 && f->dtype != ORC_F64) return ORC_E_ARG;
  g->nblocks = 1;
  for (int a = 0; a < 3; a++) {
    if (a < f->d) {
      if (f->dims[a] < 1) return ORC_E_ARG;
      g->nb[a] = (f->dims[a] + 3) / 4;
    } else {
      if (f->dims[a] != 1) return ORC_E_ARG;
      g->nb[a] = 1;
    }
    g->nblocks *= g->nb[a];
  }
  g->nchunks = (g->nblocks + ORC_CHUNK_BLOCKS - 1) / ORC_CHUNK_BLOCKS;
  g->B = block_size(f->d);
  g->P = prec_bits(f->dtype);
  return ORC_OK;
}

/* linear field index of local sample l of block b (edge replication) */
static uint64_t sample_index(const orc_field* f, const geom* g, uint64_t b, int l) {
  uint64_t bc[3];
  bc[0] = b % g->nb[0];
  bc[1] = (b / g->nb[0]) % g->nb[1];
  bc[2] = b / (g->nb[0] * g->nb[1]);
  uint64_t c[3];
  for (int a = 0; a < 3; a++) {
    uint64_t v = a < f->d ? bc[a] * 4 + (uint64_t)local_coord(l, a) : 0;
    if (v > f->dims[a] - 1) v = f->dims[a] - 1;
    c[a] = v;
  }
  return c[0] + f->dims[0] * (c[1] + f->dims[1] * c[2]);
}
static int sample_valid(const orc_field* f, const geom* g, uint64_t b, int l) {
  uint64_t bc[3];
  bc[0] = b % g->nb[0];
  bc[1] = (b / g->nb[0]) % g->nb[1];
  bc[2] = b / (g->nb[0] * g->nb[1]);
  for (int a = 0; a < f->d; a++)
    if (bc[a] * 4 + (uint64_t)local_coord(l, a) >= f->dims[a]) return 0;
  return 1;
}

/* ------------------------------------------------------------------ */
/* block coefficients: exponent, quantise, transform, reorder, nb      */
/* returns 0 for an all-zero block                                     */
/* ------------------------------------------------------------------ */
int orc_block_coeffs(int dtype, int d, const double* e, int* emax_out, uint64_t* u) {
  int B = block_size(d), P = prec_bits(dtype);
  int allzero = 1;
  int emax = -100000;
  for (int l = 0; l < B; l++) {
    if (!is_zero_bits(e[l])) allzero = 0;
    int x = value_expo(e[l], dtype);
    if (x > emax) emax = x;
  }
  *emax_out = emax;
  if (allzero) return 0;
  int64_t q[64];
  for (int l = 0; l < B; l++) q[l] = quantize(e[l], emax, P);
  orc_fwd_xform(q, d, P);
  int perm[64];
  orc_perm(d, perm);
  for (int r = 0; r < B; r++) u[r] = orc_to_negabinary(q[perm[r]], P);
  return 1;
}

/* values of a coded block from its (possibly truncated) coefficients */
void orc_block_values(int dtype, int d, int emax, const uint64_t* u, double* out) {
  int B = block_size(d), P = prec_bits(dtype);
  int perm[64];
  orc_perm(d, perm);
  int64_t q[64];
  for (int r = 0; r < B; r++) q[perm[r]] = orc_from_negabinary(u[r], P);
  orc_inv_xform(q, d, P);
  for (int l = 0; l < B; l++) out[l] = dequantize(q[l], emax, P, dtype);
}

/* bits of a coded block with p planes and escalation delta */
static uint64_t coded_bits(const uint64_t* u, int dtype, int d, int p, int delta) {
  int B = block_size(d), P = prec_bits(dtype);
  uint8_t tmp[64 * 64 * 3 / 8 + 64];
  uint64_t pb = orc_encode_planes(u, B, P, p, tmp, sizeof(tmp));
  return 2u + (uint64_t)(delta + 1) + (uint64_t)exp_bits(dtype) + pb;
}
static uint64_t raw_bits(int dtype, int d) {
  return 2u + (uint64_t)block_size(d) * (uint64_t)prec_bits(dtype);
}

/* ------------------------------------------------------------------ */
/* encode one block: residual e (gathered), x and xt (gathered), valid */
/* mask; writes the block bits to w; returns the mode and outputs the  */
/* accepted error and the decoded component values xi.                 */
/* Acceptance rule (format v1):                                        */
/*   err_before = max |x - xt|, err_after(p) = max |x - (xt + D)| (f64) */
/*   for p = p0, p0+1, ...:                                            */
/*     feasible = 1 <= p <= P and coded_bits(p) <= raw_bits            */
/*     if feasible and err_after(p) <= tau and <= err_before: CODED(p) */
/*     else if err_before <= tau: EMPTY                                */
/*     else if not feasible: RAW                                       */
/*     else escalate p by one                                          */
/* ------------------------------------------------------------------ */
typedef struct {
  int mode, p, delta, emax;
  double err;
  int miss;
} block_result;

static double block_err(const double* x, const double* xt, const double* xi, const int* valid,
                        int B, int dtype) {
  double m = 0.0;
  for (int l = 0; l < B; l++) {
    if (!valid[l]) continue;
    double s = add_T(xt[l], xi[l], dtype);
    double a = fabs(x[l] - s);
    if (!(a <= m)) m = a; /* a NaN error propagates as NaN */
  }
  return m;
}

static block_result encode_block(bitw* w, int dtype, int d, const double* e, const double* x,
                                 const double* xt, const int* valid, double tau, int minexp,
                                 double* xi) {
  int B = block_size(d), P = prec_bits(dtype);
  block_result res = {ORC_EMPTY, 0, 0, 0, 0.0, 0};
  double zero[64] = {0};
  double err_before = block_err(x, xt, zero, valid, B, dtype);
  uint64_t u[64];
  int emax;
  int nonzero = orc_block_coeffs(dtype, d, e, &emax, u);
  res.emax = emax;
  for (int l = 0; l < B; l++) xi[l] = 0.0;
  if (!nonzero) {
    res.mode = ORC_EMPTY;
  } else {
    int p0 = emax - minexp + guard_planes(d);
    if (p0 < 0) p0 = 0;
    if (p0 > P) p0 = P;
    int p = p0, delta = 0;
    for (;;) {
      int feasible = p >= 1 && p <= P && coded_bits(u, dtype, d, p, delta) <= raw_bits(dtype, d);
      if (feasible) {
        uint64_t ut[64];
        uint64_t keep = (p == P) ? ~0ull : ~((1ull << (P - p)) - 1ull);
        for (int r = 0; r < B; r++) ut[r] = u[r] & keep;
        double dv[64];
        orc_block_values(dtype, d, emax, ut, dv);
        double ea = block_err(x, xt, dv, valid, B, dtype);
        if (ea <= tau && ea <= err_before) {
          res.mode = ORC_CODED; res.p = p; res.delta = delta;
          for (int l = 0; l < B; l++) xi[l] = dv[l];
          break;
        }
      }
      if (err_before <= tau) { res.mode = ORC_EMPTY; break; }
      if (!feasible) { res.mode = ORC_RAW; break; }
      p++; delta++;
    }
  }
  if (res.mode == ORC_RAW)
    for (int l = 0; l < B; l++) xi[l] = e[l];
  res.err = res.mode == ORC_EMPTY ? err_before : block_err(x, xt, xi, valid, B, dtype);
  /* a miss of Eq. (1) or of monotonicity; only reachable through RAW when */
  /* the residual itself was rounded, never expected for the schedules here */
  res.miss = (res.err <= tau && res.err <= err_before) ? 0 : 1;

  /* emit */
  if (res.mode == ORC_EMPTY) {
    put_bit(w, 0);
  } else if (res.mode == ORC_RAW) {
    put_bit(w, 1);
    put_bit(w, 1);
    for (int l = 0; l < B; l++) {
      if (dtype == ORC_F32) {
        float f = (float)e[l];
        uint32_t b;
        memcpy(&b, &f, 4);
        put_bits(w, b, 32);
      } else {
        uint64_t b;
        memcpy(&b, &e[l], 8);
        put_bits(w, b, 64);
      }
    }
  } else {
    put_bit(w, 1);
    put_bit(w, 0);
    for (int t = 0; t < res.delta; t++) put_bit(w, 1);
    put_bit(w, 0);
    put_bits(w, (uint64_t)(res.emax + exp_bias(dtype)), exp_bits(dtype));
    encode_planes(w, u, B, P, res.p);
  }
  return res;
}

/* decode one block at reader r into values out[B]; returns mode or <0 */
static int decode_block(bitr* r, int dtype, int d, int minexp, double* out) {
  int B = block_size(d), P = prec_bits(dtype);
  for (int l = 0; l < B; l++) out[l] = 0.0;
  if (!get_bit(r)) return ORC_EMPTY;
  if (get_bit(r)) {
    for (int l = 0; l < B; l++) {
      if (dtype == ORC_F32) {
        uint32_t b = (uint32_t)get_bits(r, 32);
        float f;
        memcpy(&f, &b, 4);
        out[l] = (double)f;
      } else {
        uint64_t b = get_bits(r, 64);
        memcpy(&out[l], &b, 8);
      }
    }
    return ORC_RAW;
  }
  int delta = 0;
  while (get_bit(r)) {
    delta++;
    if (delta > P || r->overrun) return ORC_E_CORRUPT;
  }
  int emax = (int)get_bits(r, exp_bits(dtype)) - exp_bias(dtype);
  if (emax < 2 - exp_bias(dtype)) return ORC_E_CORRUPT;
  int p0 = emax - minexp + guard_planes(d);
  if (p0 < 0) p0 = 0;
  if (p0 > P) p0 = P;
  int p = p0 + delta;
  if (p < 1 || p > P) return ORC_E_CORRUPT;
  uint64_t u[64];
  decode_planes(r, u, B, P, p);
  orc_block_values(dtype, d, emax, u, out);
  return ORC_CODED;
}

/* ================================================================== */
/* Codec 1: prediction and uniform quantisation on the same blocks.    */
/* The paper's driver works with any error-bounded lossy compressor    */
/* (Sec. 6.2) and names prediction-based ones beside the transform     */
/* codecs (Sec. 5, compressor list).  This one is written from the     */
/* general recipe of such codecs: quantise the residual to integer     */
/* multiples of a bin h, predict each integer from its neighbours,     */
/* and code the prediction errors.  Readings (format version 1,        */
/* codec 1):                                                           */
/*   h = 2 tau, halved per escalation step: h_d = h * 2^-d, 0 <= d <= 63 */
/*   q = rint(e * (1/h_d)) in double (1/h computed once, scaled by 2^d); */
/*     a block is feasible only while every |e * (1/h_d)| < 2^(P-2)      */
/*   decoded value = fl_T(fl_double(q * h_d))                           */
/*   prediction: the block-local Lorenzo predictor of q (the mixed     */
/*     first difference along each of the d axes, samples outside the  */
/*     block taken as 0), in wrapping P-bit integers; it is used only  */
/*     when it needs fewer bits than q itself (ties: q itself)         */
/*   coding: zigzag z = 2r for r >= 0, -2r - 1 for r < 0 (P-bit), a   */
/*     common width w = bit length of the largest z, then all B values */
/*     in w bits each, local index order, LSB first                   */
/*   block header: 1 nonempty, 0 coded (1 raw), d ones and a zero, one */
/*     bit "predicted", w in 6 bits, then the B values                */
/*   acceptance: as codec 0, with d in place of the plane escalation;  */
/*     raw = the residual's IEEE bits                                 */
/* ================================================================== */
#define PQ_MAX_DELTA 63

static uint64_t zigzag(int64_t r, int P) {
  uint64_t u = (uint64_t)r;
  uint64_t sign = r < 0 ? pmask(P) : 0;  /* all ones when negative */
  return ((u << 1) ^ sign) & pmask(P);
}
static int64_t unzigzag(uint64_t z, int P) {
  uint64_t mag = z >> 1;
  uint64_t v = (z & 1u) ? ~mag : mag;  /* -(m) - 1 = ~m */
  return wrapP((int64_t)(v & pmask(P)), P);
}

/* Lorenzo prediction errors of q in place: along every axis, each sample
 * minus its predecessor on the line (0 before the first), so that after all
 * d axes each entry is the mixed difference of q at that point */
void orc_lorenzo_fwd(int64_t* q, int d, int P) {
  int B = block_size(d);
  for (int axis = 0; axis < d; axis++) {
    int stride = 1 << (2 * axis);
    for (int l = B - 1; l >= 0; l--)
      if (local_coord(l, axis) > 0) q[l] = subw(q[l], q[l - stride], P);
  }
}
/* inverse: running sums along every axis (z first, then y, then x; the
 * order does not matter for wrapping integer sums) */
void orc_lorenzo_inv(int64_t* r, int d, int P) {
  int B = block_size(d);
  for (int axis = d - 1; axis >= 0; axis--) {
    int stride = 1 << (2 * axis);
    for (int l = 0; l < B; l++)
      if (local_coord(l, axis) > 0) r[l] = addw(r[l], r[l - stride], P);
  }
}

static int bit_length(uint64_t v) {
  int n = 0;
  while (v) { n++; v >>= 1; }
  return n;
}

/* the integers of a block at escalation d: 0 if some |e / h_d| is too large */
static int pq_quantize_block(const double* e, int B, int P, double inv0, int delta, int64_t* q) {
  double inv = ldexp(inv0, delta);
  double lim = ldexp(1.0, P - 2);
  for (int l = 0; l < B; l++) {
    double t = e[l] * inv;
    if (!(fabs(t) < lim)) return 0;
    q[l] = (int64_t)rint(t);
  }
  return 1;
}

/* code of a quantised block: predicted flag, width, values (zigzag) */
static void pq_code(const int64_t* q, int d, int P, int* pred, int* w, uint64_t* z) {
  int B = block_size(d);
  int64_t r[64];
  uint64_t zp[64], zq[64], mp = 0, mq = 0;
  for (int l = 0; l < B; l++) r[l] = q[l];
  orc_lorenzo_fwd(r, d, P);
  for (int l = 0; l < B; l++) {
    zp[l] = zigzag(r[l], P);
    zq[l] = zigzag(q[l], P);
    if (zp[l] > mp) mp = zp[l];
    if (zq[l] > mq) mq = zq[l];
  }
  int wp = bit_length(mp), wq = bit_length(mq);
  *pred = wp < wq;
  *w = *pred ? wp : wq;
  for (int l = 0; l < B; l++) z[l] = *pred ? zp[l] : zq[l];
}

static uint64_t pq_bits(int d, int delta, int w) {
  return 2u + (uint64_t)(delta + 1) + 1u + 6u + (uint64_t)block_size(d) * (uint64_t)w;
}

static void pq_values(const int64_t* q, int B, double h0, int delta, int dtype, double* out) {
  double h = ldexp(h0, -delta);
  for (int l = 0; l < B; l++) {
    double v = (double)q[l] * h;
    out[l] = dtype == ORC_F32 ? (double)(float)v : v;
  }
}

static block_result encode_block_pq(bitw* w, int dtype, int d, const double* e, const double* x,
                                    const double* xt, const int* valid, double tau, double* xi) {
  int B = block_size(d), P = prec_bits(dtype);
  block_result res = {ORC_EMPTY, 0, 0, 0, 0.0, 0};
  double zero[64] = {0};
  double err_before = block_err(x, xt, zero, valid, B, dtype);
  double h0 = 2.0 * tau, inv0 = 1.0 / h0;
  int allzero = 1;
  for (int l = 0; l < B; l++)
    if (!is_zero_bits(e[l])) allzero = 0;
  for (int l = 0; l < B; l++) xi[l] = 0.0;
  int64_t q[64];
  uint64_t z[64];
  int pred = 0, width = 0;
  if (!allzero) {
    int delta = 0;
    for (;;) {
      int feasible = delta <= PQ_MAX_DELTA && pq_quantize_block(e, B, P, inv0, delta, q);
      if (feasible) {
        pq_code(q, d, P, &pred, &width, z);
        feasible = pq_bits(d, delta, width) <= raw_bits(dtype, d);
      }
      if (feasible) {
        double dv[64];
        pq_values(q, B, h0, delta, dtype, dv);
        double ea = block_err(x, xt, dv, valid, B, dtype);
        if (ea <= tau && ea <= err_before) {
          res.mode = ORC_CODED; res.delta = delta;
          for (int l = 0; l < B; l++) xi[l] = dv[l];
          break;
        }
      }
      if (err_before <= tau) { res.mode = ORC_EMPTY; break; }
      if (!feasible) { res.mode = ORC_RAW; break; }
      delta++;
    }
  }
  if (res.mode == ORC_RAW)
    for (int l = 0; l < B; l++) xi[l] = e[l];
  res.err = res.mode == ORC_EMPTY ? err_before : block_err(x, xt, xi, valid, B, dtype);
  res.miss = (res.err <= tau && res.err <= err_before) ? 0 : 1;

  if (res.mode == ORC_EMPTY) {
    put_bit(w, 0);
  } else if (res.mode == ORC_RAW) {
    put_bit(w, 1);
    put_bit(w, 1);
    for (int l = 0; l < B; l++) {
      if (dtype == ORC_F32) {
        float f = (float)e[l];
        uint32_t b;
        memcpy(&b, &f, 4);
        put_bits(w, b, 32);
      } else {
        uint64_t b;
        memcpy(&b, &e[l], 8);
        put_bits(w, b, 64);
      }
    }
  } else {
    put_bit(w, 1);
    put_bit(w, 0);
    for (int t = 0; t < res.delta; t++) put_bit(w, 1);
    put_bit(w, 0);
    put_bit(w, (unsigned)pred);
    put_bits(w, (uint64_t)width, 6);
    for (int l = 0; l < B; l++) put_bits(w, z[l], width);
  }
  return res;
}

static int decode_block_pq(bitr* r, int dtype, int d, double tau, double* out) {
  int B = block_size(d), P = prec_bits(dtype);
  for (int l = 0; l < B; l++) out[l] = 0.0;
  if (!get_bit(r)) return ORC_EMPTY;
  if (get_bit(r)) {
    for (int l = 0; l < B; l++) {
      if (dtype == ORC_F32) {
        uint32_t b = (uint32_t)get_bits(r, 32);
        float f;
        memcpy(&f, &b, 4);
        out[l] = (double)f;
      } else {
        uint64_t b = get_bits(r, 64);
        memcpy(&out[l], &b, 8);
      }
    }
    return ORC_RAW;
  }
  int delta = 0;
  while (get_bit(r)) {
    delta++;
    if (delta > PQ_MAX_DELTA || r->overrun) return ORC_E_CORRUPT;
  }
  int pred = (int)get_bit(r);
  int width = (int)get_bits(r, 6);
  if (width > P || r->overrun) return ORC_E_CORRUPT;
  int64_t q[64];
  for (int l = 0; l < B; l++) q[l] = unzigzag(get_bits(r, width), P);
  if (pred) orc_lorenzo_inv(q, d, P);
  pq_values(q, B, 2.0 * tau, delta, dtype, out);
  return ORC_CODED;
}

/* exported for tests */
uint64_t orc_zigzag(int64_t r, int P) { return zigzag(r, P); }
int64_t orc_unzigzag(uint64_t z, int P) { return unzigzag(z, P); }

/* ------------------------------------------------------------------ */
/* stream header (64 bytes, little-endian)                             */
/*  0 u32 magic   4 u8 version   5 u8 codec  6 u8 dtype  7 u8 d       */
/*  8 u64 nx     16 u64 ny      24 u64 nz                              */
/* 32 f64 tau    40 i32 minexp  44 u32 chunk blocks                    */
/* 48 u64 nchunks                56 u64 payload words (32-bit)          */
/* then nchunks u32 chunk start offsets (in words, from payload start), */
/* then the payload; every chunk starts on a 32-bit word boundary.     */
/* ------------------------------------------------------------------ */
static void wr_u32(uint8_t* p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void wr_u64(uint8_t* p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t rd_u32(const uint8_t* p) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i); return v; }
static uint64_t rd_u64(const uint8_t* p) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i); return v; }

/* worst-case stream bytes for a field */
uint64_t orc_stream_cap(const orc_field* f) {
  geom g;
  if (make_geom(f, &g) != ORC_OK) return 0;
  uint64_t chunk_bits = (uint64_t)ORC_CHUNK_BLOCKS * raw_bits(f->dtype, f->d);
  uint64_t chunk_words = (chunk_bits + 31) / 32;
  return ORC_HEADER_BYTES + 4 * g.nchunks + 4 * g.nchunks * chunk_words;
}

/*
 * Encode one component: y = C(e, tau) with the acceptance rule that needs
 * x and xt = x~_{i-1} (Alg. 1, Sec. 4.1; Eq. (1), Sec. 4.3).  e must be
 * x - xt computed in the field type by the caller (the residual step of Alg. 1).
 */
int orc_encode_codec(const orc_field* f, int codec, const void* e, const void* x, const void* xt, double tau,
                     uint8_t* out, uint64_t cap, uint64_t* nbytes, orc_stats* st) {
  geom g;
  int rc = make_geom(f, &g);
  if (rc != ORC_OK) return rc;
  if (!(tau > 0.0) || !isfinite(tau)) return ORC_E_ARG;
  if (codec != 0 && codec != 1) return ORC_E_ARG;
  /* codec 1 keeps every bin h_d normal and 1 / (2 tau) finite */
  if (codec == 1 && !(tau >= ldexp(1.0, -960) && tau <= ldexp(1.0, 1000))) return ORC_E_ARG;
  memset(st, 0, sizeof(*st));
  int B = g.B;
  int minexp = orc_minexp(tau);
  uint64_t index_bytes = 4 * g.nchunks;
  if (cap < ORC_HEADER_BYTES + index_bytes) return ORC_E_NOMEM;
  memset(out, 0, (size_t)cap);
  uint8_t* index = out + ORC_HEADER_BYTES;
  uint8_t* payload = index + index_bytes;
  uint64_t payload_cap_bits = (cap - ORC_HEADER_BYTES - index_bytes) * 8;
  bitw w = {payload, payload_cap_bits, 0, 0};

  for (uint64_t c = 0; c < g.nchunks; c++) {
    /* chunk starts on a 32-bit word boundary */
    w.pos = (w.pos + 31) / 32 * 32;
    if (w.pos / 32 > 0xFFFFFFFFull) return ORC_E_NOMEM;
    wr_u32(index + 4 * c, (uint32_t)(w.pos / 32));
    for (uint64_t b = c * ORC_CHUNK_BLOCKS; b < (c + 1) * ORC_CHUNK_BLOCKS && b < g.nblocks; b++) {
      double eb[64], xb[64], tb[64], xi[64];
      int valid[64];
      for (int l = 0; l < B; l++) {
        uint64_t idx = sample_index(f, &g, b, l);
        eb[l] = load_val(e, idx, f->dtype);
        xb[l] = load_val(x, idx, f->dtype);
        tb[l] = load_val(xt, idx, f->dtype);
        valid[l] = sample_valid(f, &g, b, l);
      }
      block_result res = codec == 0 ? encode_block(&w, f->dtype, f->d, eb, xb, tb, valid, tau, minexp, xi)
                                    : encode_block_pq(&w, f->dtype, f->d, eb, xb, tb, valid, tau, xi);
      if (res.mode == ORC_EMPTY) st->nempty++;
      else if (res.mode == ORC_RAW) st->nraw++;
      else st->ncoded++;
      if (res.mode == ORC_CODED && res.delta > 0) st->nesc++;
      st->nmiss += (uint64_t)res.miss;
      if (!(res.err <= st->linf)) st->linf = res.err;
    }
  }
  if (w.overflow) return ORC_E_NOMEM;
  st->bits = w.pos;
  uint64_t words = (w.pos + 31) / 32;
  uint8_t* h = out;
  wr_u32(h + 0, ORC_MAGIC);
  h[4] = (uint8_t)ORC_VERSION;
  h[5] = (uint8_t)codec;
  h[6] = (uint8_t)f->dtype;
  h[7] = (uint8_t)f->d;
  wr_u64(h + 8, f->dims[0]);
  wr_u64(h + 16, f->dims[1]);
  wr_u64(h + 24, f->dims[2]);
  uint64_t tb;
  memcpy(&tb, &tau, 8);
  wr_u64(h + 32, tb);
  wr_u32(h + 40, (uint32_t)minexp);
  wr_u32(h + 44, ORC_CHUNK_BLOCKS);
  wr_u64(h + 48, g.nchunks);
  wr_u64(h + 56, words);
  *nbytes = ORC_HEADER_BYTES + index_bytes + 4 * words;
  return ORC_OK;
}

/* codec 0, the block-transform codec */
int orc_encode(const orc_field* f, const void* e, const void* x, const void* xt, double tau,
               uint8_t* out, uint64_t cap, uint64_t* nbytes, orc_stats* st) {
  return orc_encode_codec(f, 0, e, x, xt, tau, out, cap, nbytes, st);
}

/* parse and validate a stream header; fills f and the payload extents */
int orc_stream_info(const uint8_t* s, uint64_t nbytes, orc_field* f, double* tau,
                    uint64_t* nchunks, uint64_t* words) {
  if (nbytes < ORC_HEADER_BYTES) return ORC_E_CORRUPT;
  if (rd_u32(s) != ORC_MAGIC || s[4] != ORC_VERSION || s[5] > 1) return ORC_E_CORRUPT;
  f->dtype = s[6];
  f->d = s[7];
  f->dims[0] = rd_u64(s + 8);
  f->dims[1] = rd_u64(s + 16);
  f->dims[2] = rd_u64(s + 24);
  uint64_t tb = rd_u64(s + 32);
  memcpy(tau, &tb, 8);
  geom g;
  if (make_geom(f, &g) != ORC_OK) return ORC_E_CORRUPT;
  if (!(*tau > 0.0) || !isfinite(*tau)) return ORC_E_CORRUPT;
  if ((int32_t)rd_u32(s + 40) != orc_minexp(*tau)) return ORC_E_CORRUPT;
  if (rd_u32(s + 44) != ORC_CHUNK_BLOCKS) return ORC_E_CORRUPT;
  *nchunks = rd_u64(s + 48);
  *words = rd_u64(s + 56);
  if (*nchunks != g.nchunks) return ORC_E_CORRUPT;
  if (nbytes != ORC_HEADER_BYTES + 4 * *nchunks + 4 * *words) return ORC_E_CORRUPT;
  return ORC_OK;
}

/* x_i = D(y_i): decode a whole component into a dense field (the decode step of Alg. 2) */
int orc_decode(const uint8_t* s, uint64_t nbytes, const orc_field* expect, void* out) {
  orc_field f;
  double tau;
  uint64_t nchunks, words;
  int rc = orc_stream_info(s, nbytes, &f, &tau, &nchunks, &words);
  if (rc != ORC_OK) return rc;
  if (expect && (f.dtype != expect->dtype || f.d != expect->d || f.dims[0] != expect->dims[0] ||
                 f.dims[1] != expect->dims[1] || f.dims[2] != expect->dims[2]))
    return ORC_E_ARG;
  geom g;
  make_geom(&f, &g);
  int minexp = orc_minexp(tau);
  int codec = s[5];
  const uint8_t* index = s + ORC_HEADER_BYTES;
  const uint8_t* payload = index + 4 * nchunks;
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t start = rd_u32(index + 4 * c);
    uint64_t end = c + 1 < nchunks ? rd_u32(index + 4 * (c + 1)) : words;
    if (start > end || end > words) return ORC_E_CORRUPT;
    bitr r = {payload, end * 32, start * 32, 0};
    for (uint64_t b = c * ORC_CHUNK_BLOCKS; b < (c + 1) * ORC_CHUNK_BLOCKS && b < g.nblocks; b++) {
      double v[64];
      int m = codec == 0 ? decode_block(&r, f.dtype, f.d, minexp, v) : decode_block_pq(&r, f.dtype, f.d, tau, v);
      if (m < 0 || r.overrun) return ORC_E_CORRUPT;
      for (int l = 0; l < g.B; l++)
        if (sample_valid(&f, &g, b, l)) store_val(out, sample_index(&f, &g, b, l), v[l], f.dtype);
    }
  }
  return ORC_OK;
}

/* encode a single block on its own (tests): e, x, xt of B values each */
int orc_encode_one_block(int dtype, int d, const double* e, const double* x, const double* xt,
                         double tau, uint8_t* buf, uint64_t cap_bytes, uint64_t* nbits,
                         int* mode, int* p, double* err, double* xi) {
  bitw w = {buf, cap_bytes * 8, 0, 0};
  memset(buf, 0, (size_t)cap_bytes);
  int valid[64];
  for (int l = 0; l < 64; l++) valid[l] = 1;
  block_result res = encode_block(&w, dtype, d, e, x, xt, valid, tau, orc_minexp(tau), xi);
  if (w.overflow) return ORC_E_NOMEM;
  *nbits = w.pos;
  *mode = res.mode;
  *p = res.p;
  *err = res.err;
  return res.miss ? 1 : 0;
}

/* the same for codec 1 (tests): delta receives the escalation count */
int orc_encode_one_block_pq(int dtype, int d, const double* e, const double* x, const double* xt,
                            double tau, uint8_t* buf, uint64_t cap_bytes, uint64_t* nbits,
                            int* mode, int* delta, double* err, double* xi) {
  bitw w = {buf, cap_bytes * 8, 0, 0};
  memset(buf, 0, (size_t)cap_bytes);
  int valid[64];
  for (int l = 0; l < 64; l++) valid[l] = 1;
  block_result res = encode_block_pq(&w, dtype, d, e, x, xt, valid, tau, xi);
  if (w.overflow) return ORC_E_NOMEM;
  *nbits = w.pos;
  *mode = res.mode;
  *delta = res.delta;
  *err = res.err;
  return res.miss ? 1 : 0;
}
int orc_decode_one_block_pq(int dtype, int d, double tau, const uint8_t* buf, uint64_t nbits,
                            double* out, uint64_t* used) {
  bitr r = {buf, nbits, 0, 0};
  int m = decode_block_pq(&r, dtype, d, tau, out);
  *used = r.pos;
  if (r.overrun) return ORC_E_CORRUPT;
  return m;
}

/* decode a single block (tests) */
int orc_decode_one_block(int dtype, int d, double tau, const uint8_t* buf, uint64_t nbits,
                         double* out, uint64_t* used) {
  bitr r = {buf, nbits, 0, 0};
  int m = decode_block(&r, dtype, d, orc_minexp(tau), out);
  *used = r.pos;
  if (r.overrun) return ORC_E_CORRUPT;
  return m;
}

/* exported for tests: the two roundings of the quantiser */
int64_t orc_quantize(double e, int emax, int dtype) { return quantize(e, emax, prec_bits(dtype)); }
double orc_dequantize(int64_t q, int emax, int dtype) {
  return dequantize(q, emax, prec_bits(dtype), dtype);
}
int orc_value_expo(double v, int dtype) { return value_expo(v, dtype); }
