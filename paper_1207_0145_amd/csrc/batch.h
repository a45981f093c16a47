// Batched joins (many independent equi-joins in one launch sequence).  The
// sort and partitioning phases run over segment tables that span the joins
// of the batch (S runs of every join; one R segment per join), so each phase
// is one launch for the whole batch.  The kernels here are the join-aware
// ones: the start offsets of a partition are searched only in the runs of
// its own join, work items and results are accounted per join, and every
// join records when its first work item started and its last one finished.
#pragma once
#include "kernels.h"

#include "mpsm.h"

// The batch reads its joins from a device array of descriptors
// (mpsm_join_desc); the host knows only their number and bounds on their
// sizes, so every launch is sized by those bounds and the kernels below
// build the tables on the device.  Joins are taken in waves: ordered by
// their tuples (nR + nS, ties by index) and cut into W groups of equal
// count, the smallest first, so that small joins finish early instead of
// waiting for the whole batch.

constexpr int BPLAN_NT = 1024;
constexpr uint32_t BATCH_RANK_MAX = 4096;   // joins that can be ordered into waves
constexpr uint32_t NO_WAVE = 0xFFFFFFFFu;

// S runs of one join and R buckets of one join (as k_seg_plan counts them).
__device__ __forceinline__ uint32_t batch_runs_of(uint64_t nS, uint32_t L) { return (uint32_t)((nS + L - 1) / L); }
__device__ __forceinline__ uint32_t batch_buckets_of(uint64_t nR, uint32_t BT) {
  const uint64_t nb = (nR + BT - 1) / BT;
  return nb < 1 ? 1u : (nb > (uint64_t)MAX_NB ? (uint32_t)MAX_NB : (uint32_t)nb);
}

// Checks the descriptors and assigns every join to a wave (wave[b]).  A
// join with an empty side is in wave 0, where its result (0, 0) is
// written.  status[0] = MPSM_OK, or MPSM_EINVAL when a descriptor is
// malformed (NULL or misaligned pointers, a size of 2^32 or more) or the
// joins exceed the bounds the launches were sized for: then no join is in
// any wave and no output is written.  Also stamps the batch start time.
__global__ void __launch_bounds__(BPLAN_NT) k_batch_check(const mpsm_join_desc* d, uint32_t n, uint32_t W,
                                                          uint64_t max_sum_nR, uint64_t max_sum_nS, uint64_t max_nS,
                                                          uint32_t* wave, uint32_t* status,
                                                          unsigned long long* t_start) {
  __shared__ unsigned long long sumR, sumS;
  __shared__ uint32_t bad, nact;
  __shared__ uint64_t work[BATCH_RANK_MAX];
  const uint32_t tid = threadIdx.x;
  if (tid == 0) { sumR = 0; sumS = 0; bad = 0; nact = 0; *t_start = wall_clock64(); }
  __syncthreads();
  const bool rank = W > 1 && n <= BATCH_RANK_MAX;
  for (uint32_t b = tid; b < n; b += BPLAN_NT) {
    const mpsm_join_desc x = d[b];
    bool ok = (!x.nR || x.d_R) && (!x.nS || x.d_S) && x.d_out_count && x.d_out_checksum &&
              !((uintptr_t)x.d_R & 15) && !((uintptr_t)x.d_S & 15) && !((uintptr_t)x.d_out_count & 7) &&
              !((uintptr_t)x.d_out_checksum & 7) && !((uintptr_t)x.d_out_times & 7) && x.nR < (1ull << 32) &&
              x.nS < (1ull << 32);
    const bool act = x.nR && x.nS;
    if (act) {
      ok = ok && x.nS <= max_nS;
      atomicAdd(&sumR, (unsigned long long)x.nR);
      atomicAdd(&sumS, (unsigned long long)x.nS);
      atomicAdd(&nact, 1u);
    }
    if (!ok) atomicOr(&bad, 1u);
    if (rank) work[b] = act ? x.nR + x.nS : 0;
  }
  __syncthreads();
  const bool fail = bad || sumR > max_sum_nR || sumS > max_sum_nS || sumR >= (1ull << 32) || sumS >= (1ull << 32);
  const uint32_t na = nact;
  for (uint32_t b = tid; b < n; b += BPLAN_NT) {
    uint32_t w = 0;
    if (fail) {
      w = NO_WAVE;
    } else if (rank && work[b]) {
      const uint64_t wb = work[b];
      uint32_t r = 0;   // rank among the joins with work
      for (uint32_t q = 0; q < n; q++) {
        const uint64_t wq = work[q];
        r += wq && (wq < wb || (wq == wb && q < b));
      }
      w = (uint32_t)((uint64_t)r * W / na);
    }
    wave[b] = w;
  }
  if (tid == 0) status[0] = fail ? (uint32_t)MPSM_EINVAL : (uint32_t)MPSM_OK;
}

// Tables of wave w: the join table (every join; only the wave's joins get
// runs and buckets), the S segments (the runs of the wave's joins, in join
// order, then empty runs up to Qmax) and the R segments (one per joined
// join, then empty ones up to n), with each segment's source array; zeroes
// the counter words.
__global__ void __launch_bounds__(BPLAN_NT) k_batch_plan(const mpsm_join_desc* d, uint32_t n, const uint32_t* wave,
                                                         uint32_t w, uint32_t L, uint32_t BT, uint32_t Qmax,
                                                         BatchJoin* J, uint32_t* segS_start, uint32_t* segS_len,
                                                         const tup_t** srcS, uint32_t* segR_start,
                                                         uint32_t* segR_len, const tup_t** srcR,
                                                         uint32_t* zero_words, uint32_t nzero) {
  __shared__ uint32_t wsum[5][BPLAN_NT / 64 + 2];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < nzero; i += BPLAN_NT) zero_words[i] = 0;
  uint32_t cQ = 0, cG = 0, cA = 0, cS = 0, cR = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += BPLAN_NT) {
    const uint32_t b = b0 + tid;
    mpsm_join_desc x;
    bool member = false, act = false;
    if (b < n) {
      x = d[b];
      member = wave[b] == w;
      act = member && x.nR && x.nS;
    }
    const uint32_t Q = act ? batch_runs_of(x.nS, L) : 0, G = act ? batch_buckets_of(x.nR, BT) : 0;
    const uint32_t nS = act ? (uint32_t)x.nS : 0, nR = act ? (uint32_t)x.nR : 0;
    uint32_t t[5];
    const uint32_t eQ = block_excl_scan<BPLAN_NT>(Q, wsum[0], &t[0]);
    const uint32_t eG = block_excl_scan<BPLAN_NT>(G, wsum[1], &t[1]);
    const uint32_t eA = block_excl_scan<BPLAN_NT>(act ? 1u : 0u, wsum[2], &t[2]);
    const uint32_t eS = block_excl_scan<BPLAN_NT>(nS, wsum[3], &t[3]);
    const uint32_t eR = block_excl_scan<BPLAN_NT>(nR, wsum[4], &t[4]);
    if (b < n) {
      BatchJoin& j = J[b];
      j.r0 = cQ + eQ; j.Q = Q; j.g0 = cG + eG; j.G = G;
      j.member = member ? 1u : 0u; j.s0 = cS + eS;
      j.p0 = 0xFFFFFFFFu; j.P = 0; j.obase = 0; j.items = 0; j.done = 0;
      j.count = 0; j.checksum = 0; j.t_first = ~0ull; j.t_done = 0;
      j.out_count = x.d_out_count; j.out_checksum = x.d_out_checksum; j.out_times = x.d_out_times;
      if (act) {
        const uint32_t a = cA + eA;
        segR_start[a] = cR + eR;
        segR_len[a] = nR;
        srcR[a] = reinterpret_cast<const tup_t*>(x.d_R);
      }
    }
    cQ += t[0]; cG += t[1]; cA += t[2]; cS += t[3]; cR += t[4];
    __syncthreads();
  }
  // empty segments after the joined ones: they start at the end
  for (uint32_t a = cA + tid; a < n; a += BPLAN_NT) { segR_start[a] = cR; segR_len[a] = 0; srcR[a] = nullptr; }
  for (uint32_t q = cQ + tid; q < Qmax; q += BPLAN_NT) { segS_start[q] = cS; segS_len[q] = 0; srcS[q] = nullptr; }
  __syncthreads();   // the join table above is read back below
  // the runs of every joined join: run q belongs to the last join whose
  // first run is at or below q (joins without runs share the next start)
  for (uint32_t q = tid; q < cQ; q += BPLAN_NT) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) { const uint32_t m = (lo + hi) >> 1; if (J[m].r0 <= q) lo = m; else hi = m; }
    const BatchJoin& j = J[lo];
    const uint32_t r = q - j.r0;
    const uint64_t nSj = d[lo].nS;
    segS_start[q] = j.s0 + r * L;
    segS_len[q] = (uint32_t)((uint64_t)(r + 1) * L <= nSj ? L : nSj - (uint64_t)r * L);
    srcS[q] = reinterpret_cast<const tup_t*>(d[lo].d_S) + (uint64_t)r * L;
  }
}

// Join whose range [x0, x0 + xn) holds position x: the last join with
// start <= x (joins with empty ranges share the next join's start).
template <typename F>
__device__ __forceinline__ uint32_t batch_join_of(uint32_t n, uint64_t x, F start) {
  uint32_t lo = 0, hi = n;   // last b with start(b) <= x
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start(mid) <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Non-empty R buckets become the partitions (in bucket order, so those of a
// join are contiguous); each remembers its join.
__global__ void __launch_bounds__(1024) k_partitions_batch(const uint32_t* bstart, const uint64_t* bkey,
                                                           const uint32_t* Gcount, BatchJoin* J, uint32_t n,
                                                           uint32_t* Pcount, uint32_t* pstart, uint32_t* plen,
                                                           uint64_t* pkey, uint32_t* pjoin) {
  __shared__ uint32_t wsum[1024 / 64 + 2];
  const uint32_t G = *Gcount;
  uint32_t carry = 0;
  for (uint32_t b = 0; b < G; b += 1024) {
    const uint32_t g = b + threadIdx.x;
    const uint32_t len = g < G ? bstart[g + 1] - bstart[g] : 0;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>(len ? 1u : 0u, wsum, &tot);
    if (len) {
      const uint32_t p = carry + ex;
      const uint32_t jb = batch_join_of(n, g, [&](uint32_t i) { return (uint64_t)J[i].g0; });
      pstart[p] = bstart[g]; plen[p] = len; pkey[p] = bkey[g]; pjoin[p] = jb;
      atomicAdd(&J[jb].P, 1u);
      atomicMin(&J[jb].p0, p);
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *Pcount = carry;
}

// Offsets of the joins' blocks of start offsets: join b owns (P_b + 1) rows
// of Q_b entries (the last row holds the run lengths).
__global__ void k_batch_blocks(BatchJoin* J, uint32_t n, unsigned long long* o_total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long run = 0;
  for (uint32_t b = 0; b < n; b++) {
    J[b].obase = run;
    if (J[b].P == 0) J[b].p0 = 0;
    run += (unsigned long long)(J[b].P + 1) * J[b].Q;
  }
  *o_total = run;
}

// o[obase_b + row * Q_b + j] = lower bound of the first key of the join's
// partition `row` in run j of the join (row P_b: the run's length).  Threads
// walk a join's block run by run, consecutive threads taking consecutive
// partitions of one run, so that a wave's bisections share their first
// index entries and end in neighbouring lines.
__global__ void __launch_bounds__(256) k_search_batch(const tup_t* __restrict__ U, const uint32_t* run_start,
                                                      const uint32_t* run_len, const uint64_t* run_idx,
                                                      uint32_t idx_stride, uint32_t idx_per_run, const BatchJoin* J,
                                                      uint32_t n, const uint64_t* pkey, uint32_t* o,
                                                      const unsigned long long* o_total, int mode,
                                                      const uint8_t* span) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= *o_total) return;
  const uint32_t jb = batch_join_of(n, gid, [&](uint32_t i) { return (uint64_t)J[i].obase; });
  const BatchJoin& j = J[jb];
  const uint64_t local = gid - j.obase;
  const uint32_t rows = j.P + 1;
  const uint32_t row = (uint32_t)(local % rows), q = (uint32_t)(local / rows);
  if (row < j.P && !span[j.p0 + row]) return;   // inside a join unit: never read
  const uint32_t run = j.r0 + q;
  const uint32_t len = run_len[run];
  uint32_t probes = 0;
  o[j.obase + (uint64_t)row * j.Q + q] = row == j.P ? len
                      : run_lower_bound(mode, U + run_start[run], len, pkey[j.p0 + row],
                                        run_idx + (uint64_t)run * idx_per_run, idx_stride, &probes);
}

// Work items of every partition (as k_join_items) and their count per join.
// Join units of every partition (as k_join_units; a unit never spans two joins).
__global__ void k_join_units_batch(const uint32_t* Pcount, const uint32_t* plen, const uint32_t* pjoin,
                                   uint32_t Pmax, uint8_t* span) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t P = *Pcount;
  if (p < P && p < Pmax)
    span[p] = (uint8_t)join_span(plen, P, p, [&](uint32_t q) { return pjoin[q] == pjoin[q + 1]; });
}

// Work items of every join unit (as k_join_items) and the item count per join.
__global__ void k_join_items_batch(const uint32_t* Pcount, const uint32_t* pjoin, BatchJoin* J, const uint32_t* o,
                                   const uint32_t* run_len, uint32_t Pmax, uint32_t JCH, const uint8_t* span,
                                   uint32_t* items) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > Pmax + 1) return;
  const uint32_t P = *Pcount;
  uint32_t it = 0;
  if (p < P) {
    const uint32_t jb = pjoin[p];
    const uint32_t sp = span[p];
    if (sp) {
      const uint32_t Q = J[jb].Q;
      const uint32_t* a = o + J[jb].obase + (uint64_t)(p - J[jb].p0) * Q;
      const uint32_t* b = a + (uint64_t)sp * Q;
      uint64_t np = 0;
      const uint32_t* rl = run_len + J[jb].r0;
      for (uint32_t q = 0; q < Q; q++) np += slice_len(a[q], b[q], rl[q]);   // as in k_join
      it = (uint32_t)((np + JCH - 1) / JCH);
      if (it) atomicAdd(&J[jb].items, it);
    }
  }
  items[p] = it;
}

// Results and times of the wave's joins to the caller's slots.
__global__ void k_finalize_batch(const BatchJoin* J, uint32_t n, const unsigned long long* t_start) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const BatchJoin& j = J[b];
  if (!j.member) return;
  *j.out_count = j.count;
  *j.out_checksum = j.checksum;
  if (j.out_times) {
    const uint64_t t0 = *t_start;
    j.out_times[0] = t0;
    j.out_times[1] = j.items ? j.t_first : t0;
    j.out_times[2] = j.items ? j.t_done : t0;
  }
}
