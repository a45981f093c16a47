// Batched joins (many independent equi-joins in one launch sequence).  The
// sort and partitioning phases run over segment tables that span the joins
// of the batch (S runs of every join; one R segment per join), so each phase
// is one launch for the whole batch.  The kernels here are the join-aware
// ones: the start offsets of a partition are searched only in the runs of
// its own join, work items and results are accounted per join, and every
// join records when its first work item started and its last one finished.
#pragma once
#include "kernels.h"

// Fresh join table (all but the host-filled fields) and the batch start time.
__global__ void k_batch_init(BatchJoin* J, uint32_t n, unsigned long long* t_start, uint32_t* zero_words,
                             uint32_t nzero) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *t_start = wall_clock64();
  for (uint32_t b = t; b < n; b += gridDim.x * blockDim.x) {
    BatchJoin& j = J[b];
    j.p0 = 0xFFFFFFFFu; j.P = 0; j.obase = 0; j.items = 0; j.done = 0;
    j.count = 0; j.checksum = 0; j.t_first = ~0ull; j.t_done = 0;
  }
  for (uint32_t i = t; i < nzero; i += gridDim.x * blockDim.x) zero_words[i] = 0;
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

// Results and times of every join to the caller's slots.
__global__ void k_finalize_batch(const BatchJoin* J, uint32_t n, const unsigned long long* t_start) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const BatchJoin& j = J[b];
  *j.out_count = j.count;
  *j.out_checksum = j.checksum;
  if (j.out_times) {
    const uint64_t t0 = *t_start;
    j.out_times[0] = t0;
    j.out_times[1] = j.items ? j.t_first : t0;
    j.out_times[2] = j.items ? j.t_done : t0;
  }
}
