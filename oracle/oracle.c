/*
 * CPU oracle for the range-partitioned massively parallel sort-merge join
 * (P-MPSM) of Albutiu, Kemper and Neumann, "Massively Parallel Sort-Merge
 * Joins in Main Memory Multi-Core Database Systems" (PVLDB 5(10), 2012).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the GPU path.
 *
 * Everything here is plain, slow and sequential on purpose.  All join
 * arithmetic is on unsigned 64-bit integers (the paper's keys and payloads
 * are 64-bit integers, Section 5.1).  Floating point appears only in the two
 * estimates of Section 4 (the S distribution and the partition cost), which
 * choose splitters and never decide a join result.
 *
 * Tuples are arrays of 2*n uint64: T[2i] = key, T[2i+1] = payload.
 *
 * Contents, in the paper's order:
 *   - the result's definition: equi-join of R and S on the key (Section 5.1
 *     query), reported as count, checksum (a reading, see orc_pair_hash),
 *     the paper's aggregate max(R.payload + S.payload), and the pair list;
 *   - independent checks of that definition: nested loops, hash join,
 *     foreign-key closed form;
 *   - the method's steps: phase 1 run sort (Section 2.3/3.2), phase 2
 *     histogram / prefix sum / scatter (Section 3.2.1, eq. for ps_i,
 *     Figs. 6 and 10), equi-depth sampled splitters and their bucket
 *     function, phase 4 start search by lower bound and by interpolation
 *     (Section 3.2.2, Fig. 7), the global S distribution from merged
 *     equi-height bounds (Section 4.1, Fig. 8), the split-relevant cost and
 *     its min-max split (Section 4.3), the basic B-MPSM join (Section 2.1,
 *     Fig. 3), the full P-MPSM join (Fig. 5), and the knots of a
 *     piecewise-linear CDF over a seeded sample (Section 4.1's shape).
 *
 * Pins: see tests/test_oracle_pins.py.  The learned CDF's residual network
 * and its quality are not computed here (parity unpinned: the paper has no
 * learned model; its knots and the exactness of the join result are
 * pinned).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_GAMMA 0x9E3779B97F4A7C15ULL

/* ---------------------------------------------------------------- hashing */

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27; z *= 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return z;
}

/* i-th output (0-based) of the SplitMix64 generator seeded with `seed`. */
uint64_t orc_splitmix_at(uint64_t seed, uint64_t i) { return orc_mix64(seed + (i + 1) * ORC_GAMMA); }

/* Per-pair checksum term.  The paper reports no checksum; its query feeds
 * both payloads through the join (Section 5.1).  Reading: a pair (key, r
 * payload, s payload) hashes to mix(mix(mix(key + gamma) + rp) + sp), and
 * the join checksum is the wrapping (mod 2^64) sum over all pairs, so it is
 * order independent and counts duplicate pairs. */
uint64_t orc_pair_hash(uint64_t key, uint64_t rp, uint64_t sp) {
  uint64_t h = orc_mix64(key + ORC_GAMMA);
  h = orc_mix64(h + rp);
  return orc_mix64(h + sp);
}

/* ------------------------------------------------------------ stable sort */

/* Bottom-up merge sort of tuples by key; equal keys keep input order. */
int orc_sort_by_key(uint64_t* T, uint64_t n) {
  if (n < 2) return 0;
  uint64_t* B = (uint64_t*)malloc(2 * n * sizeof(uint64_t));
  if (!B) return -1;
  uint64_t *src = T, *dst = B;
  for (uint64_t w = 1; w < n; w *= 2) {
    for (uint64_t lo = 0; lo < n; lo += 2 * w) {
      uint64_t mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
      uint64_t i = lo, j = mid, k = lo;
      while (i < mid && j < hi) {
        if (src[2 * j] < src[2 * i]) { dst[2 * k] = src[2 * j]; dst[2 * k + 1] = src[2 * j + 1]; j++; }
        else { dst[2 * k] = src[2 * i]; dst[2 * k + 1] = src[2 * i + 1]; i++; }
        k++;
      }
      while (i < mid) { dst[2 * k] = src[2 * i]; dst[2 * k + 1] = src[2 * i + 1]; i++; k++; }
      while (j < hi) { dst[2 * k] = src[2 * j]; dst[2 * k + 1] = src[2 * j + 1]; j++; k++; }
    }
    uint64_t* t = src; src = dst; dst = t;
  }
  if (src != T) memcpy(T, src, 2 * n * sizeof(uint64_t));
  free(B);
  return 0;
}

static int cmp_triple(const void* a, const void* b) {
  const uint64_t *x = (const uint64_t*)a, *y = (const uint64_t*)b;
  for (int i = 0; i < 3; i++) { if (x[i] < y[i]) return -1; if (x[i] > y[i]) return 1; }
  return 0;
}

/* Sort pairs (key, r payload, s payload) lexicographically. */
void orc_sort_pairs(uint64_t* P, uint64_t n) { qsort(P, n, 3 * sizeof(uint64_t), cmp_triple); }

/* ------------------------------------------------- the result, by definition */

typedef struct { uint64_t count, checksum, maxsum; int nonempty; } orc_acc;

static void acc_pair(orc_acc* a, uint64_t k, uint64_t rp, uint64_t sp, uint64_t* pairs, uint64_t cap) {
  if (pairs && a->count < cap) {
    pairs[3 * a->count] = k; pairs[3 * a->count + 1] = rp; pairs[3 * a->count + 2] = sp;
  }
  a->count++;
  a->checksum += orc_pair_hash(k, rp, sp);
  uint64_t s = rp + sp;                         /* wrapping, as uint64 arithmetic */
  if (!a->nonempty || s > a->maxsum) a->maxsum = s;
  a->nonempty = 1;
}

static void acc_out(const orc_acc* a, uint64_t* out4) {
  out4[0] = a->count; out4[1] = a->checksum; out4[2] = a->maxsum; out4[3] = (uint64_t)a->nonempty;
}

/* Textbook sort-merge join (both inputs sorted, equal-key groups joined by
 * their cross product): the B-MPSM idea with one worker (Section 2.1).
 * out4 = {count, checksum, max(rp+sp), nonempty}.  If pairs != NULL the
 * first min(count, cap) pairs are stored and then sorted lexicographically. */
int orc_join(const uint64_t* R, uint64_t nR, const uint64_t* S, uint64_t nS, uint64_t* out4,
             uint64_t* pairs, uint64_t cap) {
  uint64_t* r = (uint64_t*)malloc((2 * nR + 2) * sizeof(uint64_t));
  uint64_t* s = (uint64_t*)malloc((2 * nS + 2) * sizeof(uint64_t));
  if (!r || !s) { free(r); free(s); return -1; }
  memcpy(r, R, 2 * nR * sizeof(uint64_t)); memcpy(s, S, 2 * nS * sizeof(uint64_t));
  if (orc_sort_by_key(r, nR) || orc_sort_by_key(s, nS)) { free(r); free(s); return -1; }
  orc_acc a = {0, 0, 0, 0};
  uint64_t i = 0, j = 0;
  while (i < nR && j < nS) {
    if (r[2 * i] < s[2 * j]) i++;
    else if (r[2 * i] > s[2 * j]) j++;
    else {
      uint64_t k = r[2 * i], i2 = i, j2 = j;
      while (i2 < nR && r[2 * i2] == k) i2++;
      while (j2 < nS && s[2 * j2] == k) j2++;
      for (uint64_t a1 = i; a1 < i2; a1++)
        for (uint64_t b1 = j; b1 < j2; b1++) acc_pair(&a, k, r[2 * a1 + 1], s[2 * b1 + 1], pairs, cap);
      i = i2; j = j2;
    }
  }
  acc_out(&a, out4);
  if (pairs) orc_sort_pairs(pairs, a.count < cap ? a.count : cap);
  free(r); free(s);
  return 0;
}

/* The join restricted to the keys in [lo, hi) (to_top != 0: [lo, 2^64-1]).
 * Pairs have equal keys, so the joins of the slices of any partition of the
 * key space add up to the whole join (counts and checksums as wrapping sums,
 * max as the largest slice max): large joins are checked slice by slice
 * with bounded memory and one slice per thread.  out4 as in orc_join. */
int orc_join_key_range(const uint64_t* R, uint64_t nR, const uint64_t* S, uint64_t nS, uint64_t lo, uint64_t hi,
                       int to_top, uint64_t* out4) {
  uint64_t mR = 0, mS = 0;
  for (uint64_t i = 0; i < nR; i++) mR += R[2 * i] >= lo && (to_top || R[2 * i] < hi);
  for (uint64_t j = 0; j < nS; j++) mS += S[2 * j] >= lo && (to_top || S[2 * j] < hi);
  uint64_t* r = (uint64_t*)malloc((2 * mR + 2) * sizeof(uint64_t));
  uint64_t* s = (uint64_t*)malloc((2 * mS + 2) * sizeof(uint64_t));
  if (!r || !s) { free(r); free(s); return -1; }
  uint64_t a = 0, b = 0;
  for (uint64_t i = 0; i < nR; i++)
    if (R[2 * i] >= lo && (to_top || R[2 * i] < hi)) { r[2 * a] = R[2 * i]; r[2 * a + 1] = R[2 * i + 1]; a++; }
  for (uint64_t j = 0; j < nS; j++)
    if (S[2 * j] >= lo && (to_top || S[2 * j] < hi)) { s[2 * b] = S[2 * j]; s[2 * b + 1] = S[2 * j + 1]; b++; }
  int rc = orc_join(r, mR, s, mS, out4, NULL, 0);
  free(r); free(s);
  return rc;
}

/* Pin: nested-loop join (every R tuple against every S tuple). */
int orc_join_nested(const uint64_t* R, uint64_t nR, const uint64_t* S, uint64_t nS, uint64_t* out4,
                    uint64_t* pairs, uint64_t cap) {
  orc_acc a = {0, 0, 0, 0};
  for (uint64_t i = 0; i < nR; i++)
    for (uint64_t j = 0; j < nS; j++)
      if (R[2 * i] == S[2 * j]) acc_pair(&a, R[2 * i], R[2 * i + 1], S[2 * j + 1], pairs, cap);
  acc_out(&a, out4);
  if (pairs) orc_sort_pairs(pairs, a.count < cap ? a.count : cap);
  return 0;
}

/* Pin: hash join (chained table on R, probed by S), plus the key-count
 * invariant count = sum_k cnt_R(k) * cnt_S(k) computed from the table. */
int orc_join_hash(const uint64_t* R, uint64_t nR, const uint64_t* S, uint64_t nS, uint64_t* out4,
                  uint64_t* invariant_count) {
  uint64_t cap = 16; while (cap < 2 * nR + 16) cap <<= 1;
  int64_t* head = (int64_t*)malloc(cap * sizeof(int64_t));
  uint64_t* hkey = (uint64_t*)malloc(cap * sizeof(uint64_t));
  uint64_t* scnt = (uint64_t*)calloc(cap, sizeof(uint64_t));
  uint64_t* rcnt = (uint64_t*)calloc(cap, sizeof(uint64_t));
  int64_t* next = (int64_t*)malloc((nR + 1) * sizeof(int64_t));
  if (!head || !hkey || !scnt || !rcnt || !next) { free(head); free(hkey); free(scnt); free(rcnt); free(next); return -1; }
  for (uint64_t h = 0; h < cap; h++) head[h] = -1;
  for (uint64_t i = 0; i < nR; i++) {
    uint64_t k = R[2 * i], h = orc_mix64(k) & (cap - 1);
    while (head[h] != -1 && hkey[h] != k) h = (h + 1) & (cap - 1);
    if (head[h] == -1) hkey[h] = k;
    next[i] = head[h]; head[h] = (int64_t)i; rcnt[h]++;
  }
  orc_acc a = {0, 0, 0, 0};
  for (uint64_t j = 0; j < nS; j++) {
    uint64_t k = S[2 * j], h = orc_mix64(k) & (cap - 1);
    while (head[h] != -1 && hkey[h] != k) h = (h + 1) & (cap - 1);
    if (head[h] == -1) continue;
    scnt[h]++;
    for (int64_t i = head[h]; i != -1; i = next[i]) acc_pair(&a, k, R[2 * i + 1], S[2 * j + 1], NULL, 0);
  }
  uint64_t inv = 0;
  for (uint64_t h = 0; h < cap; h++) inv += rcnt[h] * scnt[h];
  acc_out(&a, out4);
  *invariant_count = inv;
  free(head); free(hkey); free(scnt); free(rcnt); free(next);
  return 0;
}

/* Pin: foreign-key closed form.  When R keys are unique and every S tuple j
 * names its partner R tuple partner[j], the join is exactly the |S| pairs
 * (R[partner[j]], S[j]).  Returns -1 if some S key differs from its partner's
 * key.  out4 as above. */
int orc_fk_closed_form(const uint64_t* R, const uint64_t* S, const uint32_t* partner, uint64_t nS, uint64_t* out4) {
  orc_acc a = {0, 0, 0, 0};
  for (uint64_t j = 0; j < nS; j++) {
    uint64_t i = partner[j];
    if (R[2 * i] != S[2 * j]) return -1;
    acc_pair(&a, S[2 * j], R[2 * i + 1], S[2 * j + 1], NULL, 0);
  }
  acc_out(&a, out4);
  return 0;
}

/* ------------------------------------------------------ phase 1: S runs */

/* Phase 1 (Section 3.2, Fig. 5): S is cut into chunks of run_len tuples
 * (the last one may be shorter) and every chunk is sorted by key on its own.
 * Runs are never merged (Section 2.1).  Sorting is stable. */
int orc_sort_runs(const uint64_t* S, uint64_t nS, uint64_t run_len, uint64_t* out) {
  memcpy(out, S, 2 * nS * sizeof(uint64_t));
  for (uint64_t a = 0; a < nS; a += run_len) {
    uint64_t n = nS - a < run_len ? nS - a : run_len;
    if (orc_sort_by_key(out + 2 * a, n)) return -1;
  }
  return 0;
}

/* --------------------------------------- phase 2: histogram, ps, scatter */

/* Radix clustering on the highest B bits after a left shift that removes
 * leading bits common to the key domain (Section 3.2.1: keys are
 * preprocessed with bitwise shifts so the B leading bits discriminate):
 *   digit(k) = ((k << shift) >> (64 - B)).
 * sp maps each of the 2^B digits to a partition (Section 4.3, the splitter
 * vector).  Each of the nchunk chunks of chunk_len tuples (worker W_i's C_i)
 * builds its histogram h_i over partitions; the prefix sums are
 *   ps_i[j] = sum_{k < i} h_k[j]                     (the eq. in Section 3.2.1)
 * and partition j of the output starts at base[j] = sum_{j' < j} |R_j'|.
 * Each chunk then scatters its tuples in input order to base[j] + ps_i[j]++.
 * Outputs: hist[nchunk*P], ps[nchunk*P] (the values before scattering),
 * base[P+1], out (n tuples). */
int orc_radix_partition(const uint64_t* C, uint64_t n, uint64_t chunk_len, int B, int shift, const uint32_t* sp,
                        uint32_t P, uint64_t* hist, uint64_t* ps, uint64_t* base, uint64_t* out) {
  if (B < 1 || B > 24 || shift < 0 || shift > 63 || chunk_len == 0) return -2;
  uint64_t nchunk = (n + chunk_len - 1) / chunk_len;
  memset(hist, 0, nchunk * P * sizeof(uint64_t));
  for (uint64_t c = 0; c < nchunk; c++)
    for (uint64_t t = c * chunk_len; t < n && t < (c + 1) * chunk_len; t++) {
      uint64_t d = (C[2 * t] << shift) >> (64 - B);
      uint32_t p = sp[d];
      if (p >= P) return -3;
      hist[c * P + p]++;
    }
  for (uint32_t j = 0; j < P; j++) {
    uint64_t s = 0;
    for (uint64_t c = 0; c < nchunk; c++) { ps[c * P + j] = s; s += hist[c * P + j]; }
    base[j + 1] = s;
  }
  base[0] = 0;
  for (uint32_t j = 0; j < P; j++) base[j + 1] += base[j];
  uint64_t* cur = (uint64_t*)malloc(P * sizeof(uint64_t));
  if (!cur) return -1;
  for (uint64_t c = 0; c < nchunk; c++) {
    for (uint32_t j = 0; j < P; j++) cur[j] = base[j] + ps[c * P + j];
    for (uint64_t t = c * chunk_len; t < n && t < (c + 1) * chunk_len; t++) {
      uint32_t p = sp[(C[2 * t] << shift) >> (64 - B)];
      uint64_t o = cur[p]++;
      out[2 * o] = C[2 * t]; out[2 * o + 1] = C[2 * t + 1];
    }
  }
  free(cur);
  return 0;
}

/* ----------------------------------------- sampled splitters and buckets */

/* Equi-depth sampled splitters (the range partitioning's bounds, Sections
 * 3.2.1 and 4.3, drawn from a sample instead of a radix histogram; the paper
 * fixes no sample, so this is a reading).  m = oversample * nbucket sample
 * positions are drawn uniformly, with replacement, from the segment [0, len)
 * by the SplitMix64 stream `seed`: pos_t = floor(x_t * len / 2^64).  The
 * sampled keys are sorted and splitter j (j = 0 .. nbucket-2) is the sample
 * key of rank (j+1) * oversample.  Writes nbucket-1 non-decreasing
 * splitters to spl. */
int orc_sample_splitters(const uint64_t* T, uint64_t len, uint32_t nbucket, uint32_t oversample, uint64_t seed,
                         uint64_t* spl) {
  if (nbucket < 2) return 0;
  uint64_t m = (uint64_t)nbucket * oversample;
  uint64_t* smp = (uint64_t*)malloc(2 * m * sizeof(uint64_t));
  if (!smp) return -1;
  for (uint64_t t = 0; t < m; t++) {
    uint64_t pos = (uint64_t)(((unsigned __int128)orc_splitmix_at(seed, t) * len) >> 64);
    smp[2 * t] = T[2 * pos]; smp[2 * t + 1] = 0;
  }
  orc_sort_by_key(smp, m);
  for (uint32_t j = 0; j + 1 < nbucket; j++) spl[j] = smp[2 * ((uint64_t)(j + 1) * oversample)];
  free(smp);
  return 0;
}

/* Knots of a piecewise-linear CDF of T's keys, the shape of Section 4.1's S
 * distribution (sample quantiles taken as equally high steps, linear between
 * them) that the learned CDF's first part has (the learned model itself is an
 * addition to the paper, so the sample is a reading): m keys drawn as in
 * orc_sample_splitters (positions floor(x_t * len / 2^64), x_t the SplitMix64
 * stream `seed`, t = 0 .. m-1), sorted; knot i (i = 0 .. k-1, k >= 2) is the
 * sample key of rank floor(i (m-1) / (k-1)), so the first knot is the
 * sample's smallest key and the last its largest.  Writes k knots. */
int orc_cdf_knots(const uint64_t* T, uint64_t len, uint32_t m, uint32_t k, uint64_t seed, uint64_t* knots) {
  if (len == 0 || m == 0 || k < 2) return -1;
  uint64_t* smp = (uint64_t*)malloc(2 * (uint64_t)m * sizeof(uint64_t));
  if (!smp) return -1;
  for (uint64_t t = 0; t < m; t++) {
    uint64_t pos = (uint64_t)(((unsigned __int128)orc_splitmix_at(seed, t) * len) >> 64);
    smp[2 * t] = T[2 * pos]; smp[2 * t + 1] = 0;
  }
  orc_sort_by_key(smp, m);
  for (uint32_t i = 0; i < k; i++) knots[i] = smp[2 * ((uint64_t)i * (m - 1) / (k - 1))];
  free(smp);
  return 0;
}

/* Bucket of a key under nbucket-1 sorted splitters: the number of splitters
 * <= key, so bucket b holds the keys in [spl[b-1], spl[b]) (the partition
 * [low, high) of Section 4.3).  Non-decreasing in the key, which is all the
 * range partitioning needs (Section 3.2.1). */
uint32_t orc_bucket_of(const uint64_t* spl, uint32_t nbucket, uint64_t key) {
  uint32_t b = 0;
  while (b + 1 < nbucket && spl[b] <= key) b++;
  return b;
}

/* Stable partition of T[0,n) into nbucket buckets by orc_bucket_of; writes
 * out and bstart[nbucket+1]. */
int orc_bucket_partition(const uint64_t* T, uint64_t n, const uint64_t* spl, uint32_t nbucket, uint64_t* out,
                         uint64_t* bstart) {
  uint32_t* b = (uint32_t*)malloc((n + 1) * sizeof(uint32_t));
  if (!b) return -1;
  memset(bstart, 0, (nbucket + 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) { b[i] = orc_bucket_of(spl, nbucket, T[2 * i]); bstart[b[i] + 1]++; }
  for (uint32_t k = 0; k < nbucket; k++) bstart[k + 1] += bstart[k];
  uint64_t* cur = (uint64_t*)malloc(nbucket * sizeof(uint64_t));
  memcpy(cur, bstart, nbucket * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) {
    uint64_t o = cur[b[i]]++;
    out[2 * o] = T[2 * i]; out[2 * o + 1] = T[2 * i + 1];
  }
  free(cur); free(b);
  return 0;
}

/* ------------------------------------------------- phase 4: start search */

/* First index in the sorted run (stride 2) whose key is >= key. */
uint64_t orc_lower_bound(const uint64_t* run, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (run[2 * mid] < key) lo = mid + 1; else hi = mid; }
  return lo;
}

/* Interpolation search for the start of a merge (Section 3.2.2, Fig. 7): the
 * next probe comes from the rule of proportion over the current search
 * space [lo, hi]: lo + (hi - lo) (key - s_lo) / (s_hi - s_lo).  The paper
 * gives only the narrowing step; reading: keep S[lo] < key <= S[hi] (the
 * answer is the first position whose key is >= key), clamp the probe into
 * (lo, hi), compute the proportion exactly in 128-bit integers, and finish
 * by bisection once a probe fails to halve the space twice or hi - lo <= 16.
 * Returns the same index as orc_lower_bound; *probes counts key reads. */
uint64_t orc_interp_search(const uint64_t* run, uint64_t n, uint64_t key, uint32_t* probes) {
  uint32_t p = 0;
  if (n == 0) { if (probes) *probes = 0; return 0; }
  p++; if (run[0] >= key) { if (probes) *probes = p; return 0; }
  p++; if (run[2 * (n - 1)] < key) { if (probes) *probes = p; return n; }
  uint64_t lo = 0, hi = n - 1;            /* run[lo] < key <= run[hi] */
  int slow = 0;
  while (hi - lo > 1) {
    uint64_t m;
    if (hi - lo <= 16 || slow >= 2) m = lo + (hi - lo) / 2;
    else {
      uint64_t klo = run[2 * lo], khi = run[2 * hi];
      unsigned __int128 num = (unsigned __int128)(hi - lo) * (key - klo);
      m = lo + (uint64_t)(num / (khi - klo));
      if (m <= lo) m = lo + 1;
      if (m >= hi) m = hi - 1;
    }
    uint64_t before = hi - lo;
    p++;
    if (run[2 * m] < key) lo = m; else hi = m;
    if (2 * (hi - lo) > before) slow++;
  }
  if (probes) *probes = p;
  return hi;
}

/* ------------------------------------------- Section 4: S CDF and costs */

/* Equi-height histogram of one sorted run (Section 4.1): buckets of
 * `stride` consecutive tuples (the last one may be shorter); the bound of
 * bucket t is its first key, at position t * stride.  Writes
 * ceil(n / stride) bounds; returns their number. */
uint64_t orc_equi_height(const uint64_t* run, uint64_t n, uint64_t stride, uint64_t* out) {
  uint64_t m = 0;
  for (uint64_t p = 0; p < n; p += stride) out[m++] = run[2 * p];
  return m;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* Global S distribution from the runs' local equi-height histograms
 * (Section 4.1, Fig. 8).  The Q sorted runs are concatenated in S (run j
 * holds positions [run_start[j], run_start[j+1])).  Steps:
 *   1. every run contributes its equi-height bounds (orc_equi_height with
 *      `stride`);
 *   2. the bounds of all runs are merged into one sorted list v_1 <= ... <=
 *      v_N;
 *   3. every bound is taken as one step of the same height h = |S| / N
 *      (the paper approximates the steps as equally high);
 *   4. between steps the distribution is interpolated linearly (the
 *      diagonal connections of Fig. 8): for v_k < x <= v_{k+1}
 *          C(x) = h (k - 1) + h (x - v_k) / (v_{k+1} - v_k),
 *      with C(x) = 0 for x <= v_1 and, past the last bound, the last step
 *      running up to one past the largest key of S, where C = |S|.
 * out[i] = C(x[i]), the estimated number of S tuples with key < x[i].
 * Floating point (long double) only shapes the estimate; the join never
 * depends on it. */
int orc_s_cdf(const uint64_t* S, const uint64_t* run_start, uint32_t Q, uint64_t stride, const uint64_t* x,
              uint64_t nx, double* out) {
  uint64_t nS = run_start[Q], cap = 0;
  for (uint32_t j = 0; j < Q; j++) cap += (run_start[j + 1] - run_start[j] + stride - 1) / stride;
  uint64_t* v = (uint64_t*)malloc((cap + 1) * sizeof(uint64_t));
  if (!v) return -1;
  uint64_t N = 0, kmax = 0;
  for (uint32_t j = 0; j < Q; j++) {
    uint64_t a = run_start[j], n = run_start[j + 1] - a;
    N += orc_equi_height(S + 2 * a, n, stride, v + N);
    if (n && S[2 * (a + n - 1)] > kmax) kmax = S[2 * (a + n - 1)];
  }
  qsort(v, N, sizeof(uint64_t), cmp_u64);
  const long double h = N ? (long double)nS / (long double)N : 0.0L;
  for (uint64_t i = 0; i < nx; i++) {
    const uint64_t q = x[i];
    if (N == 0 || q <= v[0]) { out[i] = 0.0; continue; }
    uint64_t lo = 0, hi = N;                /* k = number of bounds < q (k >= 1 here) */
    while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (v[mid] < q) lo = mid + 1; else hi = mid; }
    const uint64_t k = lo;
    const long double vk = (long double)v[k - 1];
    const long double vn = k < N ? (long double)v[k] : (long double)kmax + 1.0L;
    long double frac = vn > vk ? ((long double)q - vk) / (vn - vk) : 1.0L;
    if (frac > 1.0L) frac = 1.0L;
    out[i] = (double)(h * (long double)(k - 1) + h * frac);
  }
  free(v);
  return 0;
}

/* split-relevant cost of one R partition (Section 4.3):
 *   |R_i| log2|R_i| + T |R_i| + (CDF_S(high) - CDF_S(low)),
 * with the S term in tuples (reading: the CDF difference times |S|). */
double orc_split_cost(uint64_t r_size, uint32_t T, uint64_t s_tuples) {
  double r = (double)r_size;
  double sort = r_size > 1 ? r * log2(r) : 0.0;
  return sort + (double)T * r + (double)s_tuples;
}

/* Cost-balanced splitters at radix granularity (Section 4.3): given the fine
 * R histogram h[0..nb) and the S tuples per fine bucket s[0..nb), choose
 * P contiguous groups of buckets minimising the largest group cost.  The
 * paper names the objective but no algorithm; reading: exhaustive dynamic
 * programming over group ends (exact, for small nb).  Writes the first bucket
 * of each group to first[0..P) (first[0] = 0) and returns the optimum. */
double orc_cost_splitters_dp(const uint64_t* h, const uint64_t* s, uint32_t nb, uint32_t P, uint32_t T,
                             uint32_t* first) {
  double* best = (double*)malloc(sizeof(double) * (nb + 1) * (P + 1));
  uint32_t* arg = (uint32_t*)malloc(sizeof(uint32_t) * (nb + 1) * (P + 1));
#define BEST(i, p) best[(uint64_t)(i) * (P + 1) + (p)]
#define ARG(i, p) arg[(uint64_t)(i) * (P + 1) + (p)]
  for (uint32_t i = 0; i <= nb; i++) for (uint32_t p = 0; p <= P; p++) BEST(i, p) = 1e300;
  BEST(0, 0) = 0.0;
  for (uint32_t p = 1; p <= P; p++)
    for (uint32_t i = 0; i <= nb; i++)          /* groups 1..p cover buckets [0, i) */
      for (uint32_t j = 0; j <= i; j++) {       /* group p covers [j, i), possibly empty */
        if (BEST(j, p - 1) >= 1e300) continue;
        uint64_t rs = 0, ss = 0;
        for (uint32_t t = j; t < i; t++) { rs += h[t]; ss += s[t]; }
        double c = orc_split_cost(rs, T, ss);
        double v = BEST(j, p - 1) > c ? BEST(j, p - 1) : c;
        if (v < BEST(i, p)) { BEST(i, p) = v; ARG(i, p) = j; }
      }
  double opt = BEST(nb, P);
  uint32_t i = nb;
  for (uint32_t p = P; p >= 1; p--) { uint32_t j = ARG(i, p); first[p - 1] = j; i = j; }
#undef BEST
#undef ARG
  free(best); free(arg);
  return opt;
}

/* ------------------------------------------- B-MPSM (the basic variant) */

/* B-MPSM (Section 2.1, Fig. 3) with T workers: both inputs cut into T
 * chunks, each chunk sorted into a run; worker i merge-joins its private run
 * R_i with every public run S_j from the start (no range partitioning, so
 * every pair of runs is merged over its whole length).  out4 as in
 * orc_join.  Must equal orc_join on any input. */
int orc_bmpsm_join(const uint64_t* R, uint64_t nR, const uint64_t* S, uint64_t nS, uint32_t T, uint64_t* out4) {
  if (T == 0) return -2;
  uint64_t lr = nR ? (nR + T - 1) / T : 1, ls = nS ? (nS + T - 1) / T : 1;
  uint64_t* Rr = (uint64_t*)malloc((2 * nR + 2) * sizeof(uint64_t));
  uint64_t* Sr = (uint64_t*)malloc((2 * nS + 2) * sizeof(uint64_t));
  if (!Rr || !Sr) { free(Rr); free(Sr); return -1; }
  orc_sort_runs(R, nR, lr, Rr);
  orc_sort_runs(S, nS, ls, Sr);
  orc_acc a = {0, 0, 0, 0};
  for (uint64_t i0 = 0; i0 < nR; i0 += lr) {
    const uint64_t* Ri = Rr + 2 * i0;
    uint64_t ni = nR - i0 < lr ? nR - i0 : lr;
    for (uint64_t j0 = 0; j0 < nS; j0 += ls) {
      const uint64_t* Sj = Sr + 2 * j0;
      uint64_t nj = nS - j0 < ls ? nS - j0 : ls;
      uint64_t x = 0, y = 0;
      while (x < ni && y < nj) {
        if (Ri[2 * x] < Sj[2 * y]) x++;
        else if (Ri[2 * x] > Sj[2 * y]) y++;
        else {
          uint64_t k = Ri[2 * x], x2 = x, y2 = y;
          while (x2 < ni && Ri[2 * x2] == k) x2++;
          while (y2 < nj && Sj[2 * y2] == k) y2++;
          for (uint64_t p = x; p < x2; p++)
            for (uint64_t q = y; q < y2; q++) acc_pair(&a, k, Ri[2 * p + 1], Sj[2 * q + 1], NULL, 0);
          x = x2; y = y2;
        }
      }
    }
  }
  acc_out(&a, out4);
  free(Rr); free(Sr);
  return 0;
}

/* --------------------------------------------- the whole P-MPSM on the CPU */

/* P-MPSM (Section 3.2, Fig. 5) with T workers, R private and S public:
 *   phase 1: S in T chunks, each sorted into a run S_j;
 *   phase 2: R chunks C_i radix-clustered on B leading bits (after the
 *            domain shift) through splitter vector sp into T partitions with
 *            histograms and prefix sums (orc_radix_partition);
 *   phase 3: each partition R_i sorted;
 *   phase 4: for every R_i and every S_j, the merge start in S_j is found by
 *            interpolation search for the first key of R_i (Fig. 7), then
 *            R_i and S_j are merge-joined from there until S_j's key passes
 *            the last key of R_i.
 * sp == NULL means sp[d] = d * T >> B (equal key ranges).  out4 as in
 * orc_join.  Must equal orc_join on any input. */
int orc_pmpsm_join(const uint64_t* R, uint64_t nR, const uint64_t* S, uint64_t nS, uint32_t T, int B, int shift,
                   const uint32_t* sp_in, uint64_t* out4) {
  if (T == 0 || B < 1 || B > 24) return -2;
  uint64_t nd = (uint64_t)1 << B;
  uint32_t* sp = (uint32_t*)malloc(nd * sizeof(uint32_t));
  for (uint64_t d = 0; d < nd; d++) sp[d] = sp_in ? sp_in[d] : (uint32_t)((d * T) >> B);
  /* phase 1 */
  uint64_t run_len = nS ? (nS + T - 1) / T : 1;
  uint64_t* Sr = (uint64_t*)malloc((2 * nS + 2) * sizeof(uint64_t));
  orc_sort_runs(S, nS, run_len, Sr);
  /* phase 2 */
  uint64_t chunk = nR ? (nR + T - 1) / T : 1;
  uint64_t nchunk = nR ? (nR + chunk - 1) / chunk : 0;
  uint64_t* hist = (uint64_t*)malloc((nchunk * T + 1) * sizeof(uint64_t));
  uint64_t* ps = (uint64_t*)malloc((nchunk * T + 1) * sizeof(uint64_t));
  uint64_t* base = (uint64_t*)malloc((T + 1) * sizeof(uint64_t));
  uint64_t* Rp = (uint64_t*)malloc((2 * nR + 2) * sizeof(uint64_t));
  int rc = orc_radix_partition(R, nR, chunk, B, shift, sp, T, hist, ps, base, Rp);
  if (rc) { free(sp); free(Sr); free(hist); free(ps); free(base); free(Rp); return rc; }
  orc_acc a = {0, 0, 0, 0};
  for (uint32_t i = 0; i < T; i++) {
    /* phase 3 */
    uint64_t* Ri = Rp + 2 * base[i];
    uint64_t ni = base[i + 1] - base[i];
    orc_sort_by_key(Ri, ni);
    if (ni == 0) continue;
    /* phase 4 */
    for (uint64_t j0 = 0; j0 < nS; j0 += run_len) {
      const uint64_t* Sj = Sr + 2 * j0;
      uint64_t nj = nS - j0 < run_len ? nS - j0 : run_len;
      uint64_t y = orc_interp_search(Sj, nj, Ri[0], NULL);
      uint64_t x = 0;
      while (x < ni && y < nj) {
        if (Ri[2 * x] < Sj[2 * y]) x++;
        else if (Ri[2 * x] > Sj[2 * y]) y++;
        else {
          uint64_t k = Ri[2 * x], x2 = x, y2 = y;
          while (x2 < ni && Ri[2 * x2] == k) x2++;
          while (y2 < nj && Sj[2 * y2] == k) y2++;
          for (uint64_t p = x; p < x2; p++)
            for (uint64_t q = y; q < y2; q++) acc_pair(&a, k, Ri[2 * p + 1], Sj[2 * q + 1], NULL, 0);
          x = x2; y = y2;
        }
      }
    }
  }
  acc_out(&a, out4);
  free(sp); free(Sr); free(hist); free(ps); free(base); free(Rp);
  return 0;
}
