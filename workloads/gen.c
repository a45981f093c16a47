/*
 * Seeded synthetic join inputs (host C, OpenMP).
 *
 * This module only draws inputs; it computes nothing the join computes (no
 * checksums, no sort-merge).  Both the CPU oracle and the GPU path read what
 * it writes.  Tuples are two uint64 words {key, payload}, 16 bytes, as in the
 * paper's relation schema (Section 5.1).
 *
 * Randomness: every value comes from a SplitMix64 counter stream
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): x_i = mix(seed + (i+1)*0x9E3779B97F4A7C15).  Each field of a
 * workload uses its own stream seed (seed of the workload + a field tag), so
 * any element can be recomputed from (seed, tag, i) alone.  Bounded integers
 * use the multiply-high reduction (Lemire 2019), normals use Box-Muller in
 * double precision, permutations use Fisher-Yates, Zipf ranks use an inverse
 * CDF table.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define WL_GAMMA 0x9E3779B97F4A7C15ULL

/* field tags, one stream per field */
enum {
  TAG_RPERM = 1, TAG_RPAY = 2, TAG_SPARTNER = 3, TAG_SPAY = 4, TAG_KEYMIX = 5,
  TAG_BLOB = 6, TAG_CAND = 7, TAG_ZIPF = 8, TAG_ZPERM = 9, TAG_LOGN = 10,
  TAG_BINOM = 11, TAG_ADJ = 12, TAG_SSHUF = 13, TAG_BATCH = 14
};

static inline uint64_t wl_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t wl_stream(uint64_t seed, uint64_t tag) { return wl_mix(seed ^ (tag * 0xD1B54A32D192ED03ULL)); }
static inline uint64_t wl_rand(uint64_t s, uint64_t i) { return wl_mix(s + (i + 1) * WL_GAMMA); }
static inline uint64_t wl_below(uint64_t x, uint64_t n) { return (uint64_t)(((unsigned __int128)x * n) >> 64); }
static inline double wl_unit(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }          /* [0,1) */
static inline double wl_unit_open(uint64_t x) { return ((double)(x >> 11) + 1.0) * 0x1.0p-53; } /* (0,1] */

/* i-th standard normal of stream s (Box-Muller, cosine branch). */
static inline double wl_normal(uint64_t s, uint64_t i) {
  double u1 = wl_unit_open(wl_rand(s, 2 * i)), u2 = wl_unit(wl_rand(s, 2 * i + 1));
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

uint64_t wl_splitmix_at(uint64_t seed, uint64_t i) { return wl_rand(seed, i); }

/* Fisher-Yates permutation of [0,n) drawn from stream s. */
static void wl_permutation(uint32_t* p, uint64_t n, uint64_t s) {
  for (uint64_t i = 0; i < n; i++) p[i] = (uint32_t)i;
  for (uint64_t i = n; i > 1; i--) {
    uint64_t j = wl_below(wl_rand(s, i), i);
    uint32_t t = p[i - 1]; p[i - 1] = p[j]; p[j] = t;
  }
}

/* Unique R keys + random payloads.  spread=0: keys are a permutation of
 * [0,nR).  spread=1: that permutation pushed through a keyed bijection of
 * uint64 (mix(pi(i) + k)), so keys are distinct and cover 64 bits. */
static int wl_unique_r(uint64_t* R, uint64_t nR, uint64_t seed, int spread) {
  uint32_t* perm = (uint32_t*)malloc(nR * sizeof(uint32_t));
  if (!perm) return -1;
  wl_permutation(perm, nR, wl_stream(seed, TAG_RPERM));
  uint64_t kmix = wl_stream(seed, TAG_KEYMIX), spay = wl_stream(seed, TAG_RPAY);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)nR; i++) {
    uint64_t k = perm[i];
    R[2 * i] = spread ? wl_mix(k + kmix) : k;
    R[2 * i + 1] = wl_rand(spay, (uint64_t)i);
  }
  free(perm);
  return 0;
}

/* S as foreign keys: S[j].key = R[partner[j]].key. */
static void wl_fill_s_from_partner(const uint64_t* R, uint64_t* S, const uint32_t* partner, uint64_t nS, uint64_t seed) {
  uint64_t spay = wl_stream(seed, TAG_SPAY);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)nS; j++) {
    S[2 * j] = R[2 * (uint64_t)partner[j]];
    S[2 * j + 1] = wl_rand(spay, (uint64_t)j);
  }
}

/* Uniform foreign-key join: every S tuple picks its R partner uniformly. */
int wl_gen_fk_uniform(uint64_t nR, uint64_t nS, uint64_t seed, int spread,
                      uint64_t* R, uint64_t* S, uint32_t* partner) {
  if (nR == 0 && nS > 0) return -2;
  if (wl_unique_r(R, nR, seed, spread)) return -1;
  uint64_t sp = wl_stream(seed, TAG_SPARTNER);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)nS; j++) partner[j] = (uint32_t)wl_below(wl_rand(sp, (uint64_t)j), nR);
  wl_fill_s_from_partner(R, S, partner, nS, seed);
  return 0;
}

/* Zipf(theta) foreign keys over the nR R tuples: rank r (1-based) has weight
 * r^-theta; ranks map to R tuples through a seeded permutation, so hot keys
 * are scattered over the key space. */
int wl_gen_zipf_partner(uint64_t nR, uint64_t nS, double theta, uint64_t seed, uint32_t* partner) {
  if (nR == 0) return nS ? -2 : 0;
  double* cdf = (double*)malloc(nR * sizeof(double));
  uint32_t* perm = (uint32_t*)malloc(nR * sizeof(uint32_t));
  if (!cdf || !perm) { free(cdf); free(perm); return -1; }
  double acc = 0.0;
  for (uint64_t r = 0; r < nR; r++) { acc += pow((double)(r + 1), -theta); cdf[r] = acc; }
  wl_permutation(perm, nR, wl_stream(seed, TAG_ZPERM));
  uint64_t sz = wl_stream(seed, TAG_ZIPF);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)nS; j++) {
    double u = wl_unit(wl_rand(sz, (uint64_t)j)) * acc;
    uint64_t lo = 0, hi = nR - 1;               /* first r with cdf[r] > u */
    while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (cdf[mid] > u) hi = mid; else lo = mid + 1; }
    partner[j] = perm[lo];
  }
  free(cdf); free(perm);
  return 0;
}

/* Open-addressing set of uint64 keys (key 0 handled by a flag). */
typedef struct { uint64_t* slot; uint64_t mask; int has_zero; } wl_set;
static int wl_set_init(wl_set* s, uint64_t n) {
  uint64_t cap = 1; while (cap < 2 * n + 16) cap <<= 1;
  s->slot = (uint64_t*)calloc(cap, sizeof(uint64_t)); s->mask = cap - 1; s->has_zero = 0;
  return s->slot ? 0 : -1;
}
static int wl_set_insert(wl_set* s, uint64_t k) { /* 1 if new */
  if (k == 0) { if (s->has_zero) return 0; s->has_zero = 1; return 1; }
  uint64_t h = wl_mix(k) & s->mask;
  for (;;) {
    if (s->slot[h] == 0) { s->slot[h] = k; return 1; }
    if (s->slot[h] == k) return 0;
    h = (h + 1) & s->mask;
  }
}

/* Clustered R: nR distinct keys from a mixture of nblob Gaussian blobs with
 * uniform uint64 centres and sigma = 2^(32 + 12u), u ~ U[0,1).  Candidates
 * are drawn in stream order; the first occurrence of a key is kept until nR
 * distinct keys exist. */
int wl_gen_clustered_r(uint64_t nR, uint64_t seed, int nblob, uint64_t* R) {
  uint64_t sb = wl_stream(seed, TAG_BLOB), sc = wl_stream(seed, TAG_CAND), spay = wl_stream(seed, TAG_RPAY);
  uint64_t* center = (uint64_t*)malloc(sizeof(uint64_t) * nblob);
  double* sigma = (double*)malloc(sizeof(double) * nblob);
  wl_set set;
  if (!center || !sigma || wl_set_init(&set, nR)) { free(center); free(sigma); return -1; }
  for (int b = 0; b < nblob; b++) {
    center[b] = wl_rand(sb, 2 * (uint64_t)b);
    sigma[b] = ldexp(1.0, 32) * pow(2.0, 12.0 * wl_unit(wl_rand(sb, 2 * (uint64_t)b + 1)));
  }
  const uint64_t batch = 1u << 20;
  uint64_t* cand = (uint64_t*)malloc(batch * sizeof(uint64_t));
  uint64_t have = 0, next = 0;
  while (have < nR) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)batch; t++) {
      uint64_t i = next + (uint64_t)t;
      int b = (int)wl_below(wl_rand(sc, 3 * i), (uint64_t)nblob);
      double z = wl_normal(sc ^ 0x5bd1e995ULL, i);
      double d = sigma[b] * z;
      uint64_t c = center[b], k;
      if (d >= 0) { double m = (double)(UINT64_MAX - c); k = (d >= m) ? UINT64_MAX : c + (uint64_t)llround(d); }
      else { double m = (double)c; k = (-d >= m) ? 0 : c - (uint64_t)llround(-d); }
      cand[t] = k;
    }
    for (uint64_t t = 0; t < batch && have < nR; t++)
      if (wl_set_insert(&set, cand[t])) R[2 * have++] = cand[t];
    next += batch;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)nR; i++) R[2 * i + 1] = wl_rand(spay, (uint64_t)i);
  free(cand); free(set.slot); free(center); free(sigma);
  return 0;
}

/* Foreign-key S from an arbitrary partner index list (used by C3, C5). */
int wl_gen_s_from_partner(const uint64_t* R, uint64_t nS, uint64_t seed, const uint32_t* partner, uint64_t* S) {
  wl_fill_s_from_partner(R, S, partner, nS, seed);
  return 0;
}

/* LSD radix sort of uint64 keys (generator helper, 16-bit digits). */
static int wl_sort_u64(uint64_t* a, uint64_t n) {
  uint64_t* b = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!b) return -1;
  uint64_t* cnt = (uint64_t*)malloc(65536 * sizeof(uint64_t));
  for (int pass = 0; pass < 4; pass++) {
    int sh = 16 * pass;
    memset(cnt, 0, 65536 * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) cnt[(a[i] >> sh) & 0xFFFF]++;
    uint64_t s = 0;
    for (int d = 0; d < 65536; d++) { uint64_t c = cnt[d]; cnt[d] = s; s += c; }
    for (uint64_t i = 0; i < n; i++) b[cnt[(a[i] >> sh) & 0xFFFF]++] = a[i];
    uint64_t* t = a; a = b; b = t;
  }
  /* four passes: result is back in the caller's array */
  free(b); free(cnt);
  return 0;
}

/* Log-normal keys with duplicates (the large-join workload):
 *   R key = floor(exp(2Z) * 2^28), Z ~ N(0,1), duplicates kept.
 *   For each distinct R key k, cnt_S(k) = 1 + Binomial(15, p) with
 *   p = (nS/D - 1)/15 (D distinct keys), then +-1 adjustments at seeded keys
 *   (within [1,16]) until the counts sum to nS; S lists each key cnt_S(k)
 *   times in Fisher-Yates shuffled order.
 * Outputs: R, S and the exact join size sum_k cnt_R(k) * cnt_S(k) (it is
 * known here because the generator chose both counts). */
int wl_gen_lognormal(uint64_t nR, uint64_t nS, uint64_t seed, double sigma, uint64_t* R, uint64_t* S,
                     uint64_t* out_distinct, uint64_t* out_pairs) {
  uint64_t sl = wl_stream(seed, TAG_LOGN), spay = wl_stream(seed, TAG_RPAY);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)nR; i++) {
    double x = exp(sigma * wl_normal(sl, (uint64_t)i)) * 268435456.0;
    R[2 * i] = (x >= 18446744073709551615.0) ? UINT64_MAX : (uint64_t)x;
    R[2 * i + 1] = wl_rand(spay, (uint64_t)i);
  }
  uint64_t* keys = (uint64_t*)malloc(nR * sizeof(uint64_t));
  if (!keys) return -1;
  for (uint64_t i = 0; i < nR; i++) keys[i] = R[2 * i];
  if (wl_sort_u64(keys, nR)) { free(keys); return -1; }
  /* distinct keys and their R multiplicities */
  uint64_t D = 0;
  uint32_t* rc = (uint32_t*)malloc(nR * sizeof(uint32_t));
  for (uint64_t i = 0; i < nR;) {
    uint64_t j = i; while (j < nR && keys[j] == keys[i]) j++;
    keys[D] = keys[i]; rc[D] = (uint32_t)(j - i); D++; i = j;
  }
  if (nS < D || nS > 16 * D) { free(keys); free(rc); return -3; }
  uint8_t* sc = (uint8_t*)malloc(D);
  double p = ((double)nS / (double)D - 1.0) / 15.0;
  if (p < 0) p = 0; if (p > 1) p = 1;
  uint64_t sbn = wl_stream(seed, TAG_BINOM);
  uint64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (int64_t d = 0; d < (int64_t)D; d++) {
    int c = 1;
    for (int t = 0; t < 15; t++) c += wl_unit(wl_rand(sbn, 15 * (uint64_t)d + t)) < p;
    sc[d] = (uint8_t)c; total += c;
  }
  uint64_t sa = wl_stream(seed, TAG_ADJ), it = 0;
  while (total != nS) {
    uint64_t d = wl_below(wl_rand(sa, it++), D);
    if (total < nS && sc[d] < 16) { sc[d]++; total++; }
    else if (total > nS && sc[d] > 1) { sc[d]--; total--; }
  }
  uint64_t pairs = 0, pos = 0;
  for (uint64_t d = 0; d < D; d++) {
    pairs += (uint64_t)rc[d] * sc[d];
    for (int c = 0; c < sc[d]; c++) S[2 * pos++] = keys[d];
  }
  uint64_t ss = wl_stream(seed, TAG_SSHUF);
  for (uint64_t i = nS; i > 1; i--) {
    uint64_t j = wl_below(wl_rand(ss, i), i);
    uint64_t t = S[2 * (i - 1)]; S[2 * (i - 1)] = S[2 * j]; S[2 * j] = t;
  }
  uint64_t spy = wl_stream(seed, TAG_SPAY);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)nS; j++) S[2 * j + 1] = wl_rand(spy, (uint64_t)j);
  *out_distinct = D; *out_pairs = pairs;
  free(keys); free(rc); free(sc);
  return 0;
}

/* Batched workload: n_join joins; |R_b| = floor(2^(lo + (hi-lo)u)),
 * |S_b| = k_b |R_b| with k_b uniform in {1..8}; R keys unique and spread over
 * 64 bits; a seeded half of the joins draw S partners uniformly, the other
 * half Zipf(theta_b), theta_b ~ U[zlo, zhi].  Sizes first (wl_batch_sizes),
 * then the data into caller buffers laid out join after join. */
int wl_batch_sizes(int n_join, uint64_t seed, int lo_log2, int hi_log2, uint64_t* nR, uint64_t* nS,
                   int* zipf, double* theta, double zlo, double zhi) {
  uint64_t s = wl_stream(seed, TAG_BATCH);
  int* order = (int*)malloc(sizeof(int) * n_join);
  for (int b = 0; b < n_join; b++) order[b] = b;
  for (int i = n_join; i > 1; i--) {
    int j = (int)wl_below(wl_rand(s, 1000000 + (uint64_t)i), (uint64_t)i);
    int t = order[i - 1]; order[i - 1] = order[j]; order[j] = t;
  }
  for (int b = 0; b < n_join; b++) zipf[order[b]] = (b >= n_join / 2);
  for (int b = 0; b < n_join; b++) {
    double u = wl_unit(wl_rand(s, 4 * (uint64_t)b));
    nR[b] = (uint64_t)floor(pow(2.0, lo_log2 + (hi_log2 - lo_log2) * u));
    uint64_t k = 1 + wl_below(wl_rand(s, 4 * (uint64_t)b + 1), 8);
    nS[b] = k * nR[b];
    theta[b] = zlo + (zhi - zlo) * wl_unit(wl_rand(s, 4 * (uint64_t)b + 2));
  }
  free(order);
  return 0;
}

int wl_batch_fill(int b, uint64_t seed, uint64_t nR, uint64_t nS, int zipf, double theta,
                  uint64_t* R, uint64_t* S, uint32_t* partner) {
  uint64_t sb = wl_mix(seed + 0x100000000ULL * (uint64_t)(b + 1));
  if (wl_unique_r(R, nR, sb, 1)) return -1;
  if (zipf) {
    if (wl_gen_zipf_partner(nR, nS, theta, sb, partner)) return -1;
  } else {
    uint64_t sp = wl_stream(sb, TAG_SPARTNER);
    for (uint64_t j = 0; j < nS; j++) partner[j] = (uint32_t)wl_below(wl_rand(sp, j), nR);
  }
  wl_fill_s_from_partner(R, S, partner, nS, sb);
  return 0;
}

/* Generic helpers for edge-case tests: uniform keys in [0, domain) (domain 0
 * means the full 64-bit range), random payloads. */
int wl_gen_uniform_keys(uint64_t n, uint64_t domain, uint64_t seed, uint64_t tag, uint64_t* T) {
  uint64_t s = wl_stream(seed, 100 + tag), p = wl_stream(seed, 200 + tag);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; i++) {
    uint64_t x = wl_rand(s, (uint64_t)i);
    T[2 * i] = domain ? wl_below(x, domain) : x;
    T[2 * i + 1] = wl_rand(p, (uint64_t)i);
  }
  return 0;
}
