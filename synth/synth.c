/*
 * Seeded synthetic-input generators shared by the tests, the benchmark and the
 * oracle-side checks.  This file holds no arithmetic of the tensor method
 * itself: it draws coordinates and values, removes duplicate coordinates and
 * nothing else.
 *
 * Random stream: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Element i of the stream
 * with key k is mix(k + (i + 1) * 0x9e3779b97f4a7c15), so any element can be
 * computed on its own; every routine below takes a start counter so a caller
 * can extend a sequence without changing the prefix it already drew.
 *
 * Build: gcc -O2 -fPIC -shared -pthread synth.c -o libsynth.so -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define SM_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static inline uint64_t sm_at(uint64_t key, uint64_t i) {
  return sm_mix(key + (i + 1) * SM_GAMMA);
}

/* Key of an independent stream: (seed, stream id) -> 64-bit key. */
uint64_t synth_stream_key(uint64_t seed, uint64_t stream) {
  return sm_mix(sm_mix(seed + SM_GAMMA) ^ sm_mix(stream * 0xd1b54a32d192ed03ULL + 1));
}

/* ------------------------------------------------------------------ threads */

static int synth_threads(void) {
  const char* e = getenv("SYNTH_THREADS");
  long n = e ? atol(e) : sysconf(_SC_NPROCESSORS_ONLN);
  if (n < 1) n = 1;
  if (n > 16) n = 16;
  return (int)n;
}

typedef void (*range_fn)(void* ctx, int64_t lo, int64_t hi, int tid);
typedef struct {
  range_fn fn;
  void* ctx;
  int64_t lo, hi;
  int tid;
} range_job;

static void* range_tramp(void* p) {
  range_job* j = (range_job*)p;
  j->fn(j->ctx, j->lo, j->hi, j->tid);
  return NULL;
}

/* Split [0, n) into nt contiguous chunks and run fn on each in its own thread. */
static void parallel_ranges(int64_t n, int nt, range_fn fn, void* ctx) {
  if (nt < 1) nt = 1;
  if (n < 65536) nt = 1;
  pthread_t th[16];
  range_job jobs[16];
  for (int t = 0; t < nt; ++t) {
    jobs[t].fn = fn;
    jobs[t].ctx = ctx;
    jobs[t].lo = n * t / nt;
    jobs[t].hi = n * (t + 1) / nt;
    jobs[t].tid = t;
  }
  for (int t = 1; t < nt; ++t) pthread_create(&th[t], NULL, range_tramp, &jobs[t]);
  range_tramp(&jobs[0]);
  for (int t = 1; t < nt; ++t) pthread_join(th[t], NULL);
}

/* -------------------------------------------------------- scalar draws */

static inline double u01_53(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
  uint64_t key, start, I;
  const double* cdf;
  uint32_t* out_u32;
  float* out_f32;
  double* out_f64;
  double mu, sigma;
} draw_ctx;

static void uniform_u32_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  draw_ctx* c = (draw_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    uint64_t r = sm_at(c->key, c->start + (uint64_t)i);
    c->out_u32[i] = (uint32_t)(((unsigned __int128)r * c->I) >> 64);
  }
}

/* out[i] uniform in [0, I), I <= 2^32 (Lemire's multiply-shift). */
void synth_uniform_u32(uint64_t key, uint64_t start, int64_t n, uint64_t I, uint32_t* out) {
  draw_ctx c = {key, start, I, NULL, out, NULL, NULL, 0, 0};
  parallel_ranges(n, synth_threads(), uniform_u32_fn, &c);
}

/* cdf[k-1] = sum_{j<=k} j^-alpha / sum_{j<=I} j^-alpha, k = 1..I (sequential sum). */
void synth_zipf_cdf(uint64_t I, double alpha, double* cdf) {
  double s = 0.0;
  for (uint64_t k = 1; k <= I; ++k) {
    s += pow((double)k, -alpha);
    cdf[k - 1] = s;
  }
  for (uint64_t k = 0; k < I; ++k) cdf[k] /= s;
  cdf[I - 1] = 1.0;
}

#define ZIPF_GUIDE 65536

typedef struct {
  draw_ctx* c;
  const uint32_t* guide; /* guide[g] = first k with cdf[k] > g / ZIPF_GUIDE */
} zipf_ctx;

static uint64_t first_above(const double* cdf, uint64_t a, uint64_t b, double u) {
  /* first k in [a, b] with cdf[k] > u (cdf[b] > u holds) */
  while (a < b) {
    uint64_t m = (a + b) >> 1;
    if (cdf[m] > u) b = m; else a = m + 1;
  }
  return a;
}

static void zipf_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  zipf_ctx* z = (zipf_ctx*)p;
  draw_ctx* c = z->c;
  for (int64_t i = lo; i < hi; ++i) {
    double u = u01_53(sm_at(c->key, c->start + (uint64_t)i));
    uint64_t g = (uint64_t)(u * ZIPF_GUIDE);
    uint64_t a = z->guide[g];
    uint64_t b = (g + 1 < ZIPF_GUIDE) ? z->guide[g + 1] : c->I - 1;
    c->out_u32[i] = (uint32_t)first_above(c->cdf, a, b, u); /* rank a+1 -> index a */
  }
}

/* out[i] = (Zipf rank) - 1 drawn by inverse CDF from the table of synth_zipf_cdf. */
void synth_zipf_u32(uint64_t key, uint64_t start, int64_t n, const double* cdf, uint64_t I,
                    uint32_t* out) {
  draw_ctx c = {key, start, I, cdf, out, NULL, NULL, 0, 0};
  uint32_t* guide = (uint32_t*)malloc(sizeof(uint32_t) * ZIPF_GUIDE);
  for (uint64_t g = 0; g < ZIPF_GUIDE; ++g)
    guide[g] = (uint32_t)first_above(cdf, 0, I - 1, (double)g / ZIPF_GUIDE);
  zipf_ctx z = {&c, guide};
  parallel_ranges(n, synth_threads(), zipf_fn, &z);
  free(guide);
}

static void u01_f32_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  draw_ctx* c = (draw_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    uint64_t r = sm_at(c->key, c->start + (uint64_t)i);
    c->out_f32[i] = (float)(r >> 40) * (1.0f / 16777216.0f); /* exact in fp32, [0,1) */
  }
}

void synth_u01_f32(uint64_t key, uint64_t start, int64_t n, float* out) {
  draw_ctx c = {key, start, 0, NULL, NULL, out, NULL, 0, 0};
  parallel_ranges(n, synth_threads(), u01_f32_fn, &c);
}

static void u01_f64_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  draw_ctx* c = (draw_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) c->out_f64[i] = u01_53(sm_at(c->key, c->start + (uint64_t)i));
}

void synth_u01_f64(uint64_t key, uint64_t start, int64_t n, double* out) {
  draw_ctx c = {key, start, 0, NULL, NULL, NULL, out, 0, 0};
  parallel_ranges(n, synth_threads(), u01_f64_fn, &c);
}

/* Box-Muller on elements 2i and 2i+1 of the stream. */
static inline double normal_at(uint64_t key, uint64_t i) {
  double u1 = 1.0 - u01_53(sm_at(key, 2 * i)); /* (0, 1] */
  double u2 = u01_53(sm_at(key, 2 * i + 1));
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static void normal_f64_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  draw_ctx* c = (draw_ctx*)p;
  for (int64_t i = lo; i < hi; ++i)
    c->out_f64[i] = c->mu + c->sigma * normal_at(c->key, c->start + (uint64_t)i);
}

/* out[i] = mu + sigma * N(0,1), in fp64. */
void synth_normal_f64(uint64_t key, uint64_t start, int64_t n, double mu, double sigma, double* out) {
  draw_ctx c = {key, start, 0, NULL, NULL, NULL, out, mu, sigma};
  parallel_ranges(n, synth_threads(), normal_f64_fn, &c);
}

static void normal_f32_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  draw_ctx* c = (draw_ctx*)p;
  for (int64_t i = lo; i < hi; ++i)
    c->out_f32[i] = (float)(c->mu + c->sigma * normal_at(c->key, c->start + (uint64_t)i));
}

/* out[i] = fp32(mu + sigma * N(0,1)) (fp64 draw, round to nearest even). */
void synth_normal_f32(uint64_t key, uint64_t start, int64_t n, double mu, double sigma, float* out) {
  draw_ctx c = {key, start, 0, NULL, NULL, out, NULL, mu, sigma};
  parallel_ranges(n, synth_threads(), normal_f32_fn, &c);
}

static void lognormal_f32_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  draw_ctx* c = (draw_ctx*)p;
  for (int64_t i = lo; i < hi; ++i)
    c->out_f32[i] = (float)exp(c->mu + c->sigma * normal_at(c->key, c->start + (uint64_t)i));
}

/* out[i] = fp32(exp(mu + sigma * N(0,1))). */
void synth_lognormal_f32(uint64_t key, uint64_t start, int64_t n, double mu, double sigma, float* out) {
  draw_ctx c = {key, start, 0, NULL, NULL, out, NULL, mu, sigma};
  parallel_ranges(n, synth_threads(), lognormal_f32_fn, &c);
}

/* ------------------------------------------------------------- dedupe */

typedef struct {
  int nmodes;
  const uint64_t* dims;
  const uint32_t* const* coords;
  uint64_t* keys;
  int exact;
} key_ctx;

static void coord_key_fn(void* p, int64_t lo, int64_t hi, int tid) {
  (void)tid;
  key_ctx* c = (key_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    uint64_t k = 0;
    if (c->exact) {
      for (int m = c->nmodes - 1; m >= 0; --m) k = k * c->dims[m] + c->coords[m][i];
    } else {
      k = 0x243f6a8885a308d3ULL;
      for (int m = 0; m < c->nmodes; ++m) k = sm_mix(k ^ ((uint64_t)c->coords[m][i] + (uint64_t)(m + 1) * SM_GAMMA));
    }
    c->keys[i] = k;
  }
}

typedef struct {
  uint64_t *ka, *kb;
  uint32_t *ia, *ib;
  int64_t n;
  int shift;
  int nt;
  int64_t* hist; /* nt * 2048 */
} rs_ctx;

static void rs_count(void* p, int64_t lo, int64_t hi, int tid) {
  rs_ctx* c = (rs_ctx*)p;
  int64_t* h = c->hist + (int64_t)tid * 2048;
  memset(h, 0, 2048 * sizeof(int64_t));
  for (int64_t i = lo; i < hi; ++i) h[(c->ka[i] >> c->shift) & 2047]++;
}

static void rs_scatter(void* p, int64_t lo, int64_t hi, int tid) {
  rs_ctx* c = (rs_ctx*)p;
  int64_t* h = c->hist + (int64_t)tid * 2048;
  for (int64_t i = lo; i < hi; ++i) {
    int d = (int)((c->ka[i] >> c->shift) & 2047);
    int64_t o = h[d]++;
    c->kb[o] = c->ka[i];
    c->ib[o] = c->ia[i];
  }
}

/* Stable LSD radix sort of (key, idx) by key, 11-bit digits, skipping digits that never vary. */
static void radix_sort_u64_u32(uint64_t* k, uint32_t* idx, int64_t n, uint64_t* kt, uint32_t* it) {
  int nt = synth_threads();
  if (n < 65536) nt = 1;
  uint64_t all_or = 0, all_and = ~0ULL;
  for (int64_t i = 0; i < n; ++i) { all_or |= k[i]; all_and &= k[i]; }
  uint64_t varying = all_or ^ all_and;
  int64_t* hist = (int64_t*)malloc(sizeof(int64_t) * 2048 * (size_t)nt);
  rs_ctx c = {k, kt, idx, it, n, 0, nt, hist};
  for (int shift = 0; shift < 64; shift += 11) {
    if (((varying >> shift) & 2047) == 0) continue;
    c.shift = shift;
    parallel_ranges(n, nt, rs_count, &c);
    int64_t run = 0;
    for (int d = 0; d < 2048; ++d)
      for (int t = 0; t < nt; ++t) {
        int64_t v = hist[(int64_t)t * 2048 + d];
        hist[(int64_t)t * 2048 + d] = run;
        run += v;
      }
    parallel_ranges(n, nt, rs_scatter, &c);
    uint64_t* tk = c.ka; c.ka = c.kb; c.kb = tk;
    uint32_t* ti = c.ia; c.ia = c.ib; c.ib = ti;
  }
  if (c.ka != k) {
    memcpy(k, c.ka, sizeof(uint64_t) * (size_t)n);
    memcpy(idx, c.ia, sizeof(uint32_t) * (size_t)n);
  }
  free(hist);
}

/*
 * Distinct coordinates, first occurrence in draw order.
 * coords: nmodes arrays of m draws (m < 2^32).  Writes the draw indices of the
 * first occurrence of each distinct coordinate, ascending, into keep (capacity
 * m) and returns how many there are.  Coordinates are compared through an
 * exact mixed-radix key when the product of dims fits 64 bits, else through a
 * 64-bit hash (a colliding distinct pair loses one member, which keeps the
 * output distinct).
 */
int64_t synth_dedupe(int nmodes, const uint64_t* dims, int64_t m, const uint32_t* const* coords,
                     uint32_t* keep) {
  unsigned __int128 prod = 1;
  int exact = 1;
  for (int d = 0; d < nmodes; ++d) {
    prod *= dims[d];
    if (prod > (unsigned __int128)UINT64_MAX) { exact = 0; break; }
  }
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m);
  uint64_t* kt = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m);
  uint32_t* it = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m);
  uint32_t* idx = keep;
  key_ctx kc = {nmodes, dims, coords, keys, exact};
  parallel_ranges(m, synth_threads(), coord_key_fn, &kc);
  for (int64_t i = 0; i < m; ++i) idx[i] = (uint32_t)i;
  radix_sort_u64_u32(keys, idx, m, kt, it);
  /* mark first of each run (stable sort: smallest draw index first) */
  uint8_t* mark = (uint8_t*)calloc((size_t)m, 1);
  for (int64_t i = 0; i < m; ++i)
    if (i == 0 || keys[i] != keys[i - 1]) mark[idx[i]] = 1;
  int64_t cnt = 0;
  for (int64_t i = 0; i < m; ++i)
    if (mark[i]) keep[cnt++] = (uint32_t)i;
  free(mark);
  free(keys);
  free(kt);
  free(it);
  return cnt;
}

/* out[i] = src[idx[i]] for u32 and f32 payloads (compaction helpers). */
void synth_gather_u32(const uint32_t* src, const uint32_t* idx, int64_t n, uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = src[idx[i]];
}
