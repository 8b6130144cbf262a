/*
 * Sanitizer driver for the oracle (test infrastructure, CPU only).  Built
 * together with oracle/pmc_oracle.c under -fsanitize=address,undefined by
 * tests/test_sanitizers.py, it runs the multi-component loop of Alg. 1 with
 * both codecs over small ragged fields (partial blocks, several chunks,
 * escalated and raw blocks, an exact last component), checks Eq. (1) on
 * every component, and then feeds each stream, with flipped bits and
 * truncated, to the decoder.  Every buffer is allocated at its exact size,
 * so a read or write past any of them is reported.  Exit status 0 means no
 * check failed and no sanitizer fired.
 *
 * usage: oracle_fuzz SEED MUTATIONS_PER_STREAM
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int dtype;
  int d;
  uint64_t dims[3];
} orc_field;
typedef struct {
  uint64_t nempty, ncoded, nraw, nesc, nmiss;
  double linf;
  uint64_t bits;
} orc_stats;
uint64_t orc_stream_cap(const orc_field* f);
int orc_encode_codec(const orc_field* f, int codec, const void* e, const void* x, const void* xt, double tau,
                     uint8_t* out, uint64_t cap, uint64_t* nbytes, orc_stats* st);
int orc_decode(const uint8_t* s, uint64_t nbytes, const orc_field* expect, void* out);

static uint64_t rs;
static uint64_t rnd(void) { /* xorshift64* (Vigna) */
  rs ^= rs >> 12;
  rs ^= rs << 25;
  rs ^= rs >> 27;
  return rs * 0x2545F4914F6CDD1Dull;
}
static double unif(void) { return (double)(rnd() >> 11) * 0x1p-53; }

static int failures = 0;
#define CHECK(c, ...)                  \
  do {                                 \
    if (!(c)) {                        \
      fprintf(stderr, __VA_ARGS__);    \
      fprintf(stderr, "\n");           \
      failures++;                      \
    }                                  \
  } while (0)

static double get(const void* p, uint64_t i, int dt) {
  return dt == 1 ? (double)((const float*)p)[i] : ((const double*)p)[i];
}
static void put(void* p, uint64_t i, double v, int dt) {
  if (dt == 1) ((float*)p)[i] = (float)v;
  else ((double*)p)[i] = v;
}

/* one field: smooth waves plus noise, optionally with values spread over many
 * binades (wide = 1) */
static void make_field(void* x, uint64_t n, const uint64_t* dims, int dt, int wide) {
  for (uint64_t i = 0; i < n; i++) {
    uint64_t ix = i % dims[0], iy = i / dims[0] % dims[1], iz = i / (dims[0] * dims[1]);
    double v = sin(0.37 * ix + 0.11 * iy) * cos(0.23 * iz) + 0.05 * (unif() - 0.5);
    if (wide) v *= pow(10.0, (double)(rnd() % 9) - 6.0);
    put(x, i, v, dt);
  }
}

static void mutate_and_decode(const uint8_t* s, uint64_t nbytes, const orc_field* f, int mutations) {
  uint64_t n = f->dims[0] * f->dims[1] * f->dims[2];
  size_t es = f->dtype == 1 ? 4 : 8;
  void* out = malloc(n * es);
  for (int m = 0; m < mutations; m++) {
    uint64_t len = nbytes;
    if (rnd() % 4 == 0) len = rnd() % (nbytes + 1); /* truncated */
    uint8_t* c = (uint8_t*)malloc(len ? len : 1);
    memcpy(c, s, len);
    int flips = len ? 1 + (int)(rnd() % 3) : 0;
    for (int k = 0; k < flips; k++) {
      /* half of the flips land in the header and chunk index */
      uint64_t lim = rnd() % 2 ? (len < 256 ? len : 256) : len;
      uint64_t b = rnd() % lim;
      c[b] ^= (uint8_t)(1u << (rnd() % 8));
    }
    int rc = orc_decode(c, len, f, out);
    CHECK(rc == 0 || rc == -1 || rc == -4, "decode of a mutated stream returned %d", rc);
    if (len < nbytes && flips == 0) CHECK(rc != 0, "a truncated stream decoded");
    free(c);
  }
  free(out);
}

static void run_case(const uint64_t* dims, int dt, int codec, const double* tau, int ntau, int wide, int mutations) {
  orc_field f = {dt, 3, {dims[0], dims[1], dims[2]}};
  uint64_t n = dims[0] * dims[1] * dims[2];
  size_t es = dt == 1 ? 4 : 8;
  void *x = malloc(n * es), *xt = malloc(n * es), *e = malloc(n * es), *d = malloc(n * es);
  make_field(x, n, dims, dt, wide);
  memset(xt, 0, n * es);
  uint64_t cap = orc_stream_cap(&f);
  CHECK(cap > 0, "no stream capacity");
  for (int i = 0; i < ntau; i++) {
    for (uint64_t j = 0; j < n; j++) put(e, j, get(x, j, dt) - get(xt, j, dt), dt); /* residual in the field type */
    uint8_t* s = (uint8_t*)malloc(cap);
    uint64_t nbytes = 0;
    orc_stats st;
    int rc = orc_encode_codec(&f, codec, e, x, xt, tau[i], s, cap, &nbytes, &st);
    CHECK(rc == 0, "encode failed (%d) dims %llu %llu %llu codec %d tau %g", rc, (unsigned long long)dims[0],
          (unsigned long long)dims[1], (unsigned long long)dims[2], codec, tau[i]);
    if (rc != 0) {
      free(s);
      break;
    }
    /* the stream at its exact length */
    uint8_t* t = (uint8_t*)malloc(nbytes);
    memcpy(t, s, nbytes);
    free(s);
    rc = orc_decode(t, nbytes, &f, d);
    CHECK(rc == 0, "decode failed (%d)", rc);
    double linf = 0.0;
    for (uint64_t j = 0; j < n; j++) {
      put(xt, j, get(xt, j, dt) + get(d, j, dt), dt); /* x~_i = x~_{i-1} + x_i in the field type */
      double err = fabs(get(x, j, dt) - get(xt, j, dt));
      if (!(err <= linf)) linf = err;
    }
    CHECK(st.nmiss > 0 || linf <= tau[i], "Eq. (1) missed: %g > %g", linf, tau[i]);
    CHECK(linf == st.linf, "measured error %g differs from the encoder's %g", linf, st.linf);
    mutate_and_decode(t, nbytes, &f, mutations);
    free(t);
  }
  free(x);
  free(xt);
  free(e);
  free(d);
}

int main(int argc, char** argv) {
  rs = argc > 1 ? strtoull(argv[1], NULL, 10) * 0x9E3779B97F4A7C15ull + 1 : 1;
  int mutations = argc > 2 ? atoi(argv[2]) : 50;
  static const uint64_t shapes[][3] = {{1, 1, 1}, {3, 5, 2}, {4, 4, 4}, {13, 7, 5}, {17, 9, 11}, {33, 4, 6}};
  const double lossy[] = {0.5, 0.05, 5e-3, 5e-4, 5e-5};
  const double f32_deep[] = {1e-2, 0x1p-24, 0x1p-150}; /* escalated, raw, exact */
  const double f64_deep[] = {1e-2, 0x1p-52, 0x1p-1074};
  const double f64_deep_pq[] = {1e-2, 0x1p-52, 0x1p-960}; /* the prediction codec's smallest tolerance */
  const double wide_taus[] = {10.0, 1e-3, 1e-6, 1e-9};
  for (int s = 0; s < (int)(sizeof(shapes) / sizeof(shapes[0])); s++)
    for (int dt = 1; dt <= 2; dt++)
      for (int codec = 0; codec <= 1; codec++) {
        run_case(shapes[s], dt, codec, lossy, 5, 0, mutations);
        run_case(shapes[s], dt, codec, dt == 1 ? f32_deep : codec ? f64_deep_pq : f64_deep, 3, 0, mutations);
        run_case(shapes[s], dt, codec, wide_taus, 4, 1, mutations);
      }
  printf("oracle_fuzz: %d failures\n", failures);
  return failures ? 1 : 0;
}
