// HIP kernels of the range-partitioned MPSM join on gfx950.
//
// Data: tuples of 16 bytes {u64 key, u64 payload} (paper Section 5.1).
// Positions and counts are u32 (inputs are limited to < 2^32 tuples).
//
// Both relations are sorted by the same two-step scheme, per segment:
//   1. sampled splitters per segment (equi-depth quantiles of a seeded
//      sample) define NB buckets that are non-decreasing in the key;
//   2. histogram per tile -> exclusive scan -> scatter with LDS staging
//      (the paper's histogram / prefix-sum / synchronisation-free scatter,
//      Section 3.2.1) puts every bucket contiguously;
//   3. every bucket (<= one LDS tile) is radix-sorted in LDS.
// For S the segments are the runs S_j (phase 1, Section 3.2); for R one
// global level (and, for large R, a second level inside each coarse bucket)
// is the range partitioning of phase 2 and the per-bucket sort is phase 3.
// Phase 4 searches the first key of every R partition in every S run
// (Section 3.2.2) and joins each R partition, held in LDS, with its slices.
#pragma once
#include "block_sort.h"
#include "join_slices.h"
#include "search_window.h"

// ------------------------------------------------------------------ config
// bucket sort instances: small tiles for S buckets, large tiles (= the join's
// LDS partition capacity) for R partitions and for S buckets that overflow
constexpr int BS_NT = 1024, BS_IPT = 4, BS_M = 2048;     // 4096 tuples
constexpr int BL_NT = 1024, BL_IPT = 8, BL_M = 4096;     // 8192 tuples
constexpr int BS_CAP = BS_NT * BS_IPT;
constexpr int BL_CAP = BL_NT * BL_IPT;
constexpr int LSD_NT = 512, LSD_IPT = 16;                // fallback radix sort, 8192 tuples

constexpr int SMP_NT = 1024;   // splitter sample sort: up to 16384 keys
constexpr int SMP_IPT = 16;
using SampleSorter = BlockSort<SMP_NT, SMP_IPT, 4>;
constexpr int SMP_CAP = SMP_NT * SMP_IPT;

constexpr int SMP_NT_S = 256;  // small samples: up to 2048 keys
constexpr int SMP_IPT_S = 8;
using SampleSorterS = BlockSort<SMP_NT_S, SMP_IPT_S, 4>;

constexpr int HIST_NT = 256;
constexpr int SCAT_NT = 1024;
constexpr int SCAT_IPT = 7;
constexpr int SCAT_CH = SCAT_NT * SCAT_IPT;  // tuples staged in LDS per chunk (with their buckets)
constexpr int MAX_NB = 1024;                 // buckets per segment
constexpr uint32_t S_BUCKET_MEAN = 2400;   // mean tuples per S-run bucket
constexpr int SPLIT_DIR = 2048;              // cells of the splitter directory

constexpr int JOIN_NT = 1024;
constexpr int JOIN_CAP = 8192;               // R partition held in LDS
constexpr int JOIN_QMAX = 2048;              // S runs
constexpr int JOIN_DIR = 4096;               // cells of the R-partition directory
constexpr int JOIN_RDIR = 1024;              // run directory of a work item (one entry per 64 or 256 positions)
constexpr int JOIN_CHUNK_MAX = 256 * (JOIN_RDIR - 1);

constexpr int SCAN_NT = 256;
constexpr int SCAN_IPT = 16;
constexpr int SCAN_BLOCK = SCAN_NT * SCAN_IPT;

#include "learned.h"

// ------------------------------------------------------------ small kernels

struct Result {              // device result block
  unsigned long long count, checksum, maxsum, nonempty;
  unsigned long long big_buckets, search_probes, fallbacks, spare;   // spare: largest R partition
  unsigned long long truncated;   // status word: 1 if pairs were requested and count > their capacity
};

// One join of a batch (device table), rewritten for every wave of the batch
// by k_batch_plan: the run and bucket ranges (empty unless the join is
// joined in this wave) and the output pointers; the other kernels fill the
// rest.
struct BatchJoin {
  uint32_t r0, Q;                     // S runs [r0, r0 + Q)
  uint32_t g0, G;                     // R buckets [g0, g0 + G)
  uint32_t member, s0;                // joined in this wave; first position of its S tuples
  uint32_t p0, P;                     // partitions [p0, p0 + P)
  unsigned long long obase;           // first entry of the join's (P + 1) x Q block of start offsets
  uint32_t items, done;               // join work items; items finished
  unsigned long long count, checksum;
  unsigned long long t_first, t_done; // wall clock: first work item started, last one finished
  uint64_t* out_count;
  uint64_t* out_checksum;
  uint64_t* out_times;                // NULL, or 3 u64: batch start, t_first, t_done
};

__global__ void k_init_result(Result* res, uint32_t* zero_words, uint32_t nzero) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    res->count = 0; res->checksum = 0; res->maxsum = 0; res->nonempty = 0;
    res->big_buckets = 0; res->search_probes = 0; res->fallbacks = 0; res->spare = 0;
    res->truncated = 0;
  }
  for (uint32_t i = t; i < nzero; i += gridDim.x * blockDim.x) zero_words[i] = 0;
}

// Results to the caller's slots; with pairs requested (pairs_cap > 0) the
// status word records whether the pair buffer was too small.
__global__ void k_finalize(Result* res, uint64_t* out_count, uint64_t* out_checksum, uint64_t pairs_cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *out_count = res->count;
    *out_checksum = res->checksum;
    res->truncated = (pairs_cap && res->count > pairs_cap) ? 1ull : 0ull;
  }
}

// Per-segment plan: tiles, bucket count and their prefixes.  The segments
// are runs of run_len tuples over [0, n) (run_len != 0), or the buckets of
// a previous pass (src_bstart, nseg + 1 entries), both written here, or
// already in seg_start / seg_len.
//   seg_nb[s]    buckets of segment s: NBmax, or (BT != 0) ceil(len/BT)
//                clamped to [1, NBmax], so buckets average at most BT tuples
//   seg_tile0    prefix of tile counts (nseg + 1 entries)
//   seg_cnt0     prefix of seg_nb * tiles (count-matrix offsets)
//   seg_b0       prefix of seg_nb (global bucket ids)
__global__ void __launch_bounds__(1024) k_seg_plan(uint32_t nseg, uint32_t NBmax, uint32_t BT, uint32_t TILE,
                                                   uint32_t n, uint32_t run_len, const uint32_t* src_bstart,
                                                   uint32_t* seg_start, uint32_t* seg_len, uint32_t* seg_tile0,
                                                   uint32_t* seg_cnt0, uint32_t* seg_nb, uint32_t* seg_b0) {
  __shared__ uint32_t wsum[3][1024 / 64 + 2];
  uint32_t c1 = 0, c2 = 0, c3 = 0;
  for (uint32_t b = 0; b < nseg; b += 1024) {
    const uint32_t s = b + threadIdx.x;
    uint32_t len = 0;
    if (s < nseg) {
      if (run_len) {
        const uint64_t a = (uint64_t)s * run_len;
        len = (uint32_t)(a + run_len <= n ? run_len : (n > a ? n - a : 0));
        seg_start[s] = (uint32_t)a;
        seg_len[s] = len;
      } else if (src_bstart) {
        len = src_bstart[s + 1] - src_bstart[s];
        seg_start[s] = src_bstart[s];
        seg_len[s] = len;
      } else {
        len = seg_len[s];
      }
    }
    const uint32_t nt = (len + TILE - 1) / TILE;
    uint32_t nb = 0;
    if (s < nseg) {
      nb = BT ? (len + BT - 1) / BT : NBmax;
      nb = nb < 1 ? 1 : (nb > NBmax ? NBmax : nb);
    }
    uint32_t t1, t2, t3;
    const uint32_t e1 = block_excl_scan<1024>(nt, wsum[0], &t1);
    const uint32_t e2 = block_excl_scan<1024>(nt * nb, wsum[1], &t2);
    const uint32_t e3 = block_excl_scan<1024>(nb, wsum[2], &t3);
    if (s < nseg) { seg_tile0[s] = c1 + e1; seg_cnt0[s] = c2 + e2; seg_nb[s] = nb; seg_b0[s] = c3 + e3; }
    c1 += t1; c2 += t2; c3 += t3;
    __syncthreads();
  }
  if (threadIdx.x == 0) { seg_tile0[nseg] = c1; seg_cnt0[nseg] = c2; seg_b0[nseg] = c3; }
}

// ------------------------------------------------------------------- scan

// With enable set, a scan runs only if *enable is non-zero.
__global__ void __launch_bounds__(SCAN_NT) k_scan_reduce(const uint32_t* in, uint32_t n, uint32_t* bsum,
                                                         const uint32_t* enable) {
  __shared__ uint64_t red[SCAN_NT / 64 + 1];
  if (enable && !*enable) return;
  const uint32_t base = blockIdx.x * SCAN_BLOCK;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; k++) {
    const uint32_t i = base + k * SCAN_NT + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = block_sum64<SCAN_NT>(s, red);
  if (threadIdx.x == 0) bsum[blockIdx.x] = (uint32_t)s;
}

// Exclusive scan of one SCAN_BLOCK-sized block, offset by the block prefix:
// the sum of the totals (from k_scan_reduce) of the blocks before it, which
// every block adds up itself (a few thousand blocks at most, so this costs
// less than a launch that scans the totals).
__global__ void __launch_bounds__(SCAN_NT) k_scan_apply(const uint32_t* in, uint32_t* out, uint32_t n,
                                                        const uint32_t* bsum, const uint32_t* enable) {
  __shared__ uint32_t wsum[SCAN_NT / 64 + 2];
  __shared__ uint64_t red[SCAN_NT / 64 + 1];
  if (enable && !*enable) return;
  uint64_t pre = 0;
  for (uint32_t i = threadIdx.x; i < blockIdx.x; i += SCAN_NT) pre += bsum[i];
  pre = block_sum64<SCAN_NT>(pre, red);
  const uint32_t base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_IPT;
  uint32_t v[SCAN_IPT];
  uint32_t run = 0;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; k++) {
    const uint32_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    const uint32_t x = v[k];
    v[k] = run;
    run += x;
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan<SCAN_NT>(run, wsum, &tot) + (uint32_t)pre;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; k++) {
    const uint32_t i = base + k;
    if (i < n) out[i] = v[k] + ex;
  }
}

// ------------------------------------------------------- sampled splitters

// One workgroup per segment: draw nb*OS keys at uniform positions of the
// segment (SplitMix64 stream seg_seed = splitmix_at(level_seed, s)), sort
// them, and keep every OS-th as the nb-1 splitters of the segment
// (nb = seg_nb[s]; splitters of segment s start at s*(NBmax-1)).  A key that
// is the only splitter equal to it but also fills the sample OS/2 ranks
// before or after its rank gets a bucket of its own: the next splitter
// becomes key + 1 when that is below it; along a run of such splitters
// every other one moves (a moved splitter no longer carries its key).
//
// With regions (a bucket pass without a histogram, see k_bucket_scatter)
// the kernel also sizes every bucket's region of the segment's area
// (pad_area of its start up to pad_area of its end): from the sample keys c that fall
// in the bucket (by the final splitters and the bucket function), an upper
// bound on its tuples, len/M (c + 4 sqrt(c) + 10) + 16 (the sample count is
// about Poisson with mean len/M of the bucket's size; the bound holds except
// for about one bucket in 10^4, and a bucket past it only sends its segment
// through the exact path).  Regions are scaled down if they would not fit
// the area.
struct Regions {
  uint32_t* cap;     // per global bucket: region size
  uint32_t* start;   // per global bucket: region start (tuple index into the padded array)
  uint32_t* fill;    // per global bucket: tuples claimed (zeroed here)
  uint32_t* dirty;   // per segment: 1 if a bucket outgrew its region (zeroed here)
  uint32_t* any;     // 1 if any segment is dirty (zeroed by the call's init)
};

// Area of a padded pass: the segment that starts at (compact) position x
// has its regions from pad_area(x) up to pad_area of its end, 2.75 times
// its length rounded to 64 tuples, so the areas of consecutive segments
// tile the padded array in order.
__host__ __device__ inline uint64_t pad_area(uint64_t x) { return ((x * 11) / 4 + 63) & ~63ull; }

template <int NT>
__device__ void size_regions(const Regions& rg, uint32_t s, uint32_t g0, uint32_t nb, uint32_t start, uint32_t len,
                             uint32_t M, const uint32_t* bcnt, uint32_t* wsum, uint64_t* red) {
  constexpr int PER = (MAX_NB + NT - 1) / NT;
  const uint32_t tid = threadIdx.x;
  const float scale = M ? (float)len / (float)M : 0.f;
  const uint64_t base = pad_area(start);
  const uint32_t area = (uint32_t)(pad_area((uint64_t)start + len) - base);
  uint32_t c[PER];
  uint64_t tot = 0;
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const uint32_t b = tid * PER + q;
    c[q] = 0;
    if (b < nb) {
      const float x = (float)bcnt[b];
      const float bound = nb == 1 ? (float)len : scale * (x + 4.f * __builtin_sqrtf(x) + 10.f) + 16.f;
      c[q] = bound >= (float)area ? area : (uint32_t)bound + 1u;
      tot += c[q];
    }
  }
  tot = block_sum64<NT>(tot, red);
  // fit the area: scale every region down by the same factor
  if (tot > area) {
#pragma unroll
    for (int q = 0; q < PER; q++) c[q] = (uint32_t)((uint64_t)c[q] * area / tot);
  }
  uint32_t run = 0, loc[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) { loc[q] = run; run += c[q]; }
  uint32_t all;
  const uint32_t ex = block_excl_scan<NT>(run, wsum, &all);
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const uint32_t b = tid * PER + q;
    if (b < nb) {
      rg.cap[g0 + b] = c[q];
      rg.start[g0 + b] = (uint32_t)(base + loc[q] + ex);
      rg.fill[g0 + b] = 0;
    }
  }
  if (tid == 0) rg.dirty[s] = 0;
}

template <int NT, int IPT>
__global__ void __launch_bounds__(NT) k_sample_splitters(const tup_t* __restrict__ src, const uint32_t* seg_start,
                                                         const uint32_t* seg_len, const uint32_t* seg_nb,
                                                         uint32_t NBmax, uint32_t OS, uint64_t level_seed,
                                                         uint64_t* spl, const tup_t* const* seg_src,
                                                         uint64_t* full, Regions rg, const uint32_t* seg_b0) {
  using Sorter = BlockSort<NT, IPT, 4>;
  __shared__ uint64_t buf[Sorter::BUF_WORDS];
  __shared__ uint32_t wsum[Sorter::WSUM_WORDS];
  __shared__ uint64_t red[NT / 64 + 1];
  __shared__ uint64_t lspl[MAX_NB];
  __shared__ uint32_t bcnt[MAX_NB];
  const uint32_t s = blockIdx.x, tid = threadIdx.x;
  const uint32_t len = seg_len[s], start = seg_start[s], nb = seg_nb[s];
  if (len == 0 || nb < 2) {
    if (rg.cap) {   // one bucket holds the segment (or nothing)
      for (uint32_t b = tid; b < MAX_NB; b += NT) bcnt[b] = 0;
      __syncthreads();
      size_regions<NT>(rg, s, seg_b0[s], nb, start, len, 0, bcnt, wsum, red);
    }
    return;
  }
  // a segment may be read in place from its own array
  const gtup_t* const gsrc = as_global(seg_src ? seg_src[s] - start : src);
  const uint32_t M = nb * OS;
  uint64_t* out = spl + (uint64_t)s * (NBmax - 1);
  const uint64_t seed = splitmix_at(level_seed, s);
  uint64_t key[IPT], dummy[IPT];
#pragma unroll
  for (int k = 0; k < IPT; k++) {
    const uint32_t t = k * NT + tid;
    if (t < M) {
      const uint64_t pos = start + draw_below(splitmix_at(seed, t), len);
      key[k] = gsrc[pos].key;
    } else {
      key[k] = ~0ull;
    }
    dummy[k] = 0;
  }
  Sorter::template sort<false>(key, dummy, (int)M, buf, wsum, red);
  __syncthreads();   // the sort's exchange buffer now holds the sorted sample
#pragma unroll
  for (int k = 0; k < IPT; k++) {
    const uint32_t r = k * NT + tid;
    if (r < M) buf[r] = key[k];
    if (full && r < M) full[r] = key[k];   // the whole sorted sample (one segment)
  }
  uint8_t* const moves = reinterpret_cast<uint8_t*>(buf + Sorter::CAP);   // nb - 1 flags
  __syncthreads();
  const uint32_t h = OS / 2;
  for (uint32_t j = tid; j + 1 < nb; j += NT) {
    const uint32_t pos = (j + 1) * OS;
    const uint64_t c = buf[pos];
    bool f = false;
    if (h && j + 2 < nb && !(j > 0 && buf[pos - OS] == c) && buf[pos + OS] - c > 1)
      f = (pos >= h && buf[pos - h] == c) || (pos + h < M && buf[pos + h] == c);
    moves[j] = f;
  }
  __syncthreads();
  for (uint32_t j = tid; j + 1 < nb; j += NT) {
    // splitter j-1 moved this one if it starts a run of candidates of odd length
    uint32_t t = 0;
    while (t < j && moves[j - 1 - t]) t++;
    const uint32_t pos = (j + 1) * OS;
    const uint64_t v = (t & 1) ? buf[pos - OS] + 1 : buf[pos];
    out[j] = v;
    lspl[j] = v;
  }
  if (!rg.cap) return;
  // the sample keys per bucket, by the final splitters and the bucket function
  for (uint32_t b = tid; b < nb; b += NT) bcnt[b] = 0;
  __syncthreads();
  for (uint32_t r = tid; r < M; r += NT) atomicAdd(&bcnt[bucket_of(lspl, nb - 1, buf[r])], 1u);
  __syncthreads();
  size_regions<NT>(rg, s, seg_b0[s], nb, start, len, M, bcnt, wsum, red);
}

// ------------------------------------------------- cost-balanced splitters

// The global S distribution (Section 4.1): the runs' equi-height bounds
// (every stride-th key of each sorted run) merged by counting, for each
// sorted sample key x of R, the S tuples below x: in run j about
// lb * stride - stride / 2, lb = number of bounds below x.  s_below[i] for
// sample key i; s_below[M] = all S tuples.
__global__ void __launch_bounds__(256) k_cost_s_cdf(const uint64_t* sample, uint32_t M, const uint64_t* run_idx,
                                                    const uint32_t* run_len, uint32_t Q, uint32_t idx_per_run,
                                                    uint32_t stride, uint64_t nS, uint64_t* s_below) {
  // one wave per sample key; its lanes take the runs in turn
  const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i > M) return;
  if (i == M) { if (lane == 0) s_below[M] = nS; return; }
  const uint64_t x = sample[i];
  uint64_t tot = 0;
  for (uint32_t j = lane; j < Q; j += 64) {
    const uint64_t* idx = run_idx + (uint64_t)j * idx_per_run;
    const uint32_t n = run_len[j], nidx = (n + stride - 1) / stride;
    uint32_t lo = 0, hi = nidx;
    while (lo < hi) { const uint32_t m = (lo + hi) >> 1; if (idx[m] < x) lo = m + 1; else hi = m; }
    const uint64_t est = lo ? (uint64_t)lo * stride - stride / 2 : 0;
    tot += est < n ? est : n;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, 64);
  if (lane == 0) s_below[i] = tot;
}

// Cost of a partition of r R tuples and s S tuples (Section 4.3): sorting
// it, r log2 r, plus joining it, T r + s (T = S runs).
// The logarithm is the hardware's single-precision log2 (its relative
// error, about 2^-22, only moves a group border where two costs tie).
__device__ __forceinline__ double cost_of(double r, double s, double T) {
  return (r > 1.0 ? r * (double)__builtin_amdgcn_logf((float)r) : 0.0) + T * r + s;
}

constexpr int COST_NT = 1024;
constexpr int COST_MAX = SMP_CAP;  // sample keys (cells) held in LDS

// Cells: sample key i starts cell i, which holds about RC(i+1) - RC(i) R
// tuples, RC(i) = floor(i nR / M), and s_below[i+1] - s_below[i] S tuples
// (cell 0 also takes the S tuples below the first sample key).  Group g of
// consecutive cells [c_g, c_{g+1}) becomes bucket g, split at the first key
// of cell c_{g+1}.  The groups minimise the largest group cost: the smallest
// threshold C whose greedy partition (each group as long as its cost stays
// <= C; optimal for contiguous min-max partitions) needs at most NB groups
// is searched on a geometric grid of COST_NT thresholds at a time (each
// thread checks one), twice (the second grid between the last infeasible
// and the first feasible threshold); the result is the greedy partition of
// the smallest feasible threshold.  Unused splitters repeat the largest key.
__global__ void __launch_bounds__(COST_NT) k_cost_splitters(const uint64_t* sample, const uint64_t* s_below,
                                                           uint32_t M, uint64_t nR, uint32_t NB, uint32_t T,
                                                           uint64_t* spl, double* best_cost) {
  __shared__ uint64_t sc[COST_MAX + 1];
  __shared__ double lohi[2];
  __shared__ uint32_t first_ok;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i <= M; i += COST_NT) sc[i] = i == 0 ? 0 : s_below[i];
  __syncthreads();
  const double dT = (double)T;
  // R tuples below cell i: floor(i nR / M); M = buckets x oversample is a
  // power of two here (both are), so the division is a shift
  const bool pow2 = (M & (M - 1)) == 0;
  const uint32_t msh = pow2 ? (uint32_t)__builtin_ctz(M) : 0u;
  auto rc = [&](uint32_t i) -> double {
    return (double)(pow2 ? ((uint64_t)i * nR) >> msh : (uint64_t)i * nR / M);
  };
  auto cost = [&](uint32_t a, uint32_t b) -> double {
    return cost_of(rc(b) - rc(a), (double)(sc[b] - sc[a]), dT);
  };
  // number of groups the greedy needs for threshold C (M + 1 if a cell alone exceeds it)
  auto groups = [&](double C) -> uint32_t {
    uint32_t a = 0, g = 0;
    while (a < M) {
      if (cost(a, a + 1) > C || g > NB) return M + 1;
      uint32_t lo = a + 1, hi = M;   // largest b with cost(a, b) <= C
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (cost(a, mid) <= C) lo = mid; else hi = mid - 1;
      }
      a = lo;
      g++;
    }
    return g;
  };
  {
    // the largest single cell: the lower end of the threshold search
    double mx = 0.0;
    for (uint32_t i = tid; i < M; i += COST_NT) { const double c = cost(i, i + 1); mx = c > mx ? c : mx; }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) { const double o = __shfl_xor(mx, d, 64); mx = o > mx ? o : mx; }
    if (tid == 0) { lohi[0] = 0.0; first_ok = 0; }
    __syncthreads();
    // doubles are non-negative here, so their bit patterns order like u64
    if ((tid & 63) == 0) atomicMax(reinterpret_cast<unsigned long long*>(&lohi[0]), __double_as_longlong(mx));
    __syncthreads();
    if (tid == 0) {
      lohi[0] = lohi[0] > 0.0 ? lohi[0] : 1.0;
      lohi[1] = cost(0, M) > lohi[0] ? cost(0, M) : lohi[0];
    }
  }
  __syncthreads();
  // threshold t of a geometric grid of COST_NT over [lo, hi] (single-precision
  // exponent: the grid only has to be monotone and reach both ends)
  auto grid = [&](double lo, double hi, uint32_t t) -> double {
    if (t == 0) return lo;
    if (t == COST_NT - 1) return hi;
    const float e = __builtin_amdgcn_logf((float)(hi / lo)) * ((float)t / (float)(COST_NT - 1));
    const double c = lo * (double)__builtin_amdgcn_exp2f(e);
    return c < lo ? lo : (c > hi ? hi : c);
  };
  for (int round = 0; round < 2; round++) {
    const double lo = lohi[0], hi = lohi[1];
    if (tid == 0) first_ok = COST_NT;
    __syncthreads();
    const double C = grid(lo, hi, tid);
    if (groups(C) <= NB) atomicMin(&first_ok, tid);
    __syncthreads();
    const uint32_t f = first_ok < COST_NT ? first_ok : COST_NT - 1;
    const double Cf = grid(lo, hi, f);
    const double Cp = f == 0 ? lo : grid(lo, hi, f - 1);
    __syncthreads();
    if (tid == 0) { lohi[0] = Cp; lohi[1] = Cf; }
    __syncthreads();
  }
  if (tid == 0) {
    const double C = lohi[1];
    uint32_t a = 0, g = 0;
    double worst = 0.0;
    while (a < M) {
      uint32_t lo = a + 1, hi = M;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (cost(a, mid) <= C) lo = mid; else hi = mid - 1;
      }
      const double c = cost(a, lo);
      worst = c > worst ? c : worst;
      if (lo < M && g + 1 < NB) spl[g] = sample[lo];
      a = lo;
      g++;
    }
    for (uint32_t k = g > 0 ? g - 1 : 0; k + 1 < NB; k++) spl[k] = ~0ull;
    if (best_cost) *best_cost = worst;
  }
}

// ------------------------------------------------ histogram and scatter

__device__ __forceinline__ uint32_t seg_of_tile(const uint32_t* seg_tile0, uint32_t nseg, uint32_t g) {
  uint32_t lo = 0, hi = nseg;  // last s with seg_tile0[s] <= g
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (seg_tile0[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Per-tile bucket histogram; cnt layout [segment][bucket][tile].
__global__ void __launch_bounds__(HIST_NT) k_bucket_hist(const tup_t* __restrict__ src, const uint32_t* seg_start,
                                                         const uint32_t* seg_len, const uint32_t* seg_tile0,
                                                         const uint32_t* seg_cnt0, const uint32_t* seg_nb,
                                                         uint32_t nseg, const uint64_t* spl, uint32_t NBmax,
                                                         uint32_t TILE, uint32_t* cnt, const tup_t* const* seg_src,
                                                         const uint32_t* only_dirty) {
  __shared__ uint64_t sp[MAX_NB];
  __shared__ uint32_t h[MAX_NB];
  __shared__ SplitDir<SPLIT_DIR, MAX_NB> dir;
  const uint32_t g = blockIdx.x;
  if (g >= seg_tile0[nseg]) return;
  const uint32_t s = seg_of_tile(seg_tile0, nseg, g);
  if (only_dirty && !only_dirty[s]) return;   // redo of the segments a padded scatter could not place
  // a segment may be read in place from its own array
  const gtup_t* const gsrc = as_global(seg_src ? seg_src[s] - seg_start[s] : src);
  const uint32_t t = g - seg_tile0[s], ntiles = seg_tile0[s + 1] - seg_tile0[s];
  const uint32_t segend = seg_start[s] + seg_len[s];
  const uint32_t a = seg_start[s] + t * TILE;
  const uint32_t b = min(a + TILE, segend);
  const uint32_t NB = seg_nb[s], nspl = NB - 1;
  for (uint32_t i = threadIdx.x; i < nspl; i += HIST_NT) sp[i] = spl[(uint64_t)s * (NBmax - 1) + i];
  for (uint32_t i = threadIdx.x; i < NB; i += HIST_NT) h[i] = 0;
  __syncthreads();
  if (nspl) dir.build<HIST_NT>(sp, nspl);
  const SplitView sv = dir.view(nspl);
  constexpr int HU = 8;   // keys per thread in flight
  for (uint32_t base = a; base < b; base += HIST_NT * HU) {
    uint64_t kk[HU];
#pragma unroll
    for (int u = 0; u < HU; u++) {
      const uint32_t i = base + u * HIST_NT + threadIdx.x;
      kk[u] = i < b ? gsrc[i].key : 0;
    }
#pragma unroll
    for (int u = 0; u < HU; u++)
      if (base + u * HIST_NT + threadIdx.x < b) atomicAdd(&h[dir.bucket(sv, sp, kk[u])], 1u);
  }
  __syncthreads();
  uint32_t* c = cnt + seg_cnt0[s] + t;
  for (uint32_t i = threadIdx.x; i < NB; i += HIST_NT) c[(uint64_t)i * ntiles] = h[i];
}

// Scatter of every tile to its precomputed sub-ranges (pos = scanned cnt),
// staged in LDS so that consecutive lanes write consecutive addresses.
//
// PAD (a bucket pass without a histogram): instead of the scanned counts,
// every chunk claims room for its tuples of each bucket in that bucket's
// region (Regions; one atomic per bucket and chunk) and writes them there;
// a claim that outgrows the region writes nothing and marks the segment
// dirty.  The tuples of a bucket then sit at the start of its region in
// the order of the claims.
// The segments it marks dirty are redone by k_redo_scatter.
constexpr uint32_t NO_ROOM = 0xFFFFFFFFu;

template <bool PAD>
__global__ void __launch_bounds__(SCAT_NT) k_bucket_scatter(const tup_t* __restrict__ src, tup_t* __restrict__ dst,
                                                            const uint32_t* seg_start, const uint32_t* seg_len,
                                                            const uint32_t* seg_tile0, const uint32_t* seg_cnt0,
                                                            const uint32_t* seg_nb, uint32_t nseg, const uint64_t* spl,
                                                            uint32_t NBmax, uint32_t TILE, const uint32_t* pos,
                                                            const tup_t* const* seg_src, Regions rg,
                                                            const uint32_t* seg_b0) {
  __shared__ uint64_t sp[MAX_NB];
  __shared__ uint32_t cursor[MAX_NB], lcnt[MAX_NB], lofs[MAX_NB];
  __shared__ tup_t stage[SCAT_CH];
  __shared__ uint16_t sbk[SCAT_CH];   // bucket of every staged tuple
  __shared__ uint32_t wsum[SCAT_NT / 64 + 2];
  __shared__ SplitDir<SPLIT_DIR, MAX_NB> dir;
  const uint32_t tid = threadIdx.x;
  // the tiles of a segment write neighbouring pieces of its buckets: one XCD takes them
  const uint32_t g = xcd_item(blockIdx.x, seg_tile0[nseg]);
  if (g >= seg_tile0[nseg]) return;
  const uint32_t s = seg_of_tile(seg_tile0, nseg, g);
  // a segment may be read in place from its own array
  const gtup_t* const gsrc = as_global(seg_src ? seg_src[s] - seg_start[s] : src);
  const uint32_t t = g - seg_tile0[s], ntiles = seg_tile0[s + 1] - seg_tile0[s];
  const uint32_t segend = seg_start[s] + seg_len[s];
  const uint32_t a = seg_start[s] + t * TILE;
  const uint32_t b = min(a + TILE, segend);
  const uint32_t NB = seg_nb[s], nspl = NB - 1;
  const uint32_t g0 = PAD ? seg_b0[s] : 0u;
  for (uint32_t i = tid; i < nspl; i += SCAT_NT) sp[i] = spl[(uint64_t)s * (NBmax - 1) + i];
  if (PAD) {
    for (uint32_t i = tid; i < NB; i += SCAT_NT) lcnt[i] = 0;
  } else {
    const uint32_t* p = pos + seg_cnt0[s] + t;
    for (uint32_t i = tid; i < NB; i += SCAT_NT) { cursor[i] = p[(uint64_t)i * ntiles]; lcnt[i] = 0; }
  }
  __syncthreads();
  if (nspl) dir.build<SCAT_NT>(sp, nspl);
  const SplitView sv = dir.view(nspl);
  constexpr int PER = (MAX_NB + SCAT_NT - 1) / SCAT_NT;
  tup_t nv[SCAT_IPT];   // next chunk, loaded while the current one is placed
#pragma unroll
  for (int k = 0; k < SCAT_IPT; k++) {
    const uint32_t i = a + k * SCAT_NT + tid;
    if (i < b) nv[k] = load_tup(gsrc + i);
  }
  for (uint32_t c0 = a; c0 < b; c0 += SCAT_CH) {
    tup_t v[SCAT_IPT];
    uint32_t bk[SCAT_IPT], lr[SCAT_IPT];
#pragma unroll
    for (int k = 0; k < SCAT_IPT; k++) v[k] = nv[k];
#pragma unroll
    for (int k = 0; k < SCAT_IPT; k++) {
      const uint32_t i = c0 + SCAT_CH + k * SCAT_NT + tid;
      if (i < b) nv[k] = load_tup(gsrc + i);
    }
#pragma unroll
    for (int k = 0; k < SCAT_IPT; k++) {
      const uint32_t i = c0 + k * SCAT_NT + tid;
      if (i < b) {
        bk[k] = dir.bucket(sv, sp, v[k].key);
        lr[k] = atomicAdd(&lcnt[bk[k]], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of lcnt over NB buckets (PER consecutive buckets per
    // thread); with PAD each thread also claims its buckets' room
    uint32_t loc[PER], run = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const uint32_t i = tid * PER + q;
      const uint32_t c = (i < NB) ? lcnt[i] : 0;
      loc[q] = run;
      run += c;
      if (PAD && c) {
        const uint32_t at = atomicAdd(&rg.fill[g0 + i], c);
        if (at + c <= rg.cap[g0 + i]) {
          cursor[i] = rg.start[g0 + i] + at;
        } else {
          cursor[i] = NO_ROOM;
          rg.dirty[s] = 1u;
          *rg.any = 1u;
        }
      }
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<SCAT_NT>(run, wsum, &tot);
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const uint32_t i = tid * PER + q;
      if (i < NB) lofs[i] = loc[q] + ex;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAT_IPT; k++) {
      const uint32_t i = c0 + k * SCAT_NT + tid;
      if (i < b) {
        const uint32_t q = lofs[bk[k]] + lr[k];
        stage[q] = v[k];
        sbk[q] = (uint16_t)bk[k];
      }
    }
    __syncthreads();
    const uint32_t m = min((uint32_t)SCAT_CH, b - c0);
    for (uint32_t q = tid; q < m; q += SCAT_NT) {
      // the bucket is staged with the tuple rather than looked up again
      // (two or more splitter compares on skewed keys): 7 K tuples per
      // chunk, so that every bucket still gets a run of several tuples
      const tup_t tq = stage[q];
      const uint32_t bb = sbk[q];
      const uint32_t cb = cursor[bb];
      if (!PAD || cb != NO_ROOM) store_tup(dst + cb + (q - lofs[bb]), tq);
    }
    __syncthreads();
    for (uint32_t i = tid; i < NB; i += SCAT_NT) {
      if (!PAD) cursor[i] += lcnt[i];
      lcnt[i] = 0;
    }
    __syncthreads();
  }
}

// Redo of the segments that a scatter into regions marked dirty (a bucket
// outgrew its region; rare): every tile of a dirty segment writes its
// tuples straight to their places, compactly from the start of the
// segment's area (pad_area of its start), by the scanned counts of the
// segment's tiles (k_bucket_hist with only_dirty), each tuple taking its
// place within its tile's share of its bucket by one LDS atomic.  Unstaged,
// so slower than k_bucket_scatter, but with the LDS of the histogram: the
// launch, which most often has nothing to do, needs no whole CU (the staged
// scatter's workgroups, even those that exit at once, each wait for a CU
// with all its LDS free, which the bucket sort running beside R's passes
// rarely leaves).
__global__ void __launch_bounds__(HIST_NT) k_redo_scatter(const tup_t* __restrict__ src, tup_t* __restrict__ dst,
                                                          const uint32_t* seg_start, const uint32_t* seg_len,
                                                          const uint32_t* seg_tile0, const uint32_t* seg_cnt0,
                                                          const uint32_t* seg_nb, uint32_t nseg, const uint64_t* spl,
                                                          uint32_t NBmax, uint32_t TILE, const uint32_t* pos,
                                                          const tup_t* const* seg_src, const uint32_t* dirty) {
  __shared__ uint64_t sp[MAX_NB];
  __shared__ uint32_t cur[MAX_NB];
  __shared__ SplitDir<SPLIT_DIR, MAX_NB> dir;
  const uint32_t g = blockIdx.x;
  if (g >= seg_tile0[nseg]) return;
  const uint32_t s = seg_of_tile(seg_tile0, nseg, g);
  if (!dirty[s]) return;
  const gtup_t* const gsrc = as_global(seg_src ? seg_src[s] - seg_start[s] : src);
  const uint32_t t = g - seg_tile0[s], ntiles = seg_tile0[s + 1] - seg_tile0[s];
  const uint32_t segend = seg_start[s] + seg_len[s];
  const uint32_t a = seg_start[s] + t * TILE;
  const uint32_t b = min(a + TILE, segend);
  const uint32_t NB = seg_nb[s], nspl = NB - 1;
  // the segment's counts were scanned with every other segment's: positions
  // relative to its first count, from the start of its own area
  const uint32_t rel = pos[seg_cnt0[s]];
  const uint32_t base = (uint32_t)pad_area(seg_start[s]);
  const uint32_t* p = pos + seg_cnt0[s] + t;
  for (uint32_t i = threadIdx.x; i < nspl; i += HIST_NT) sp[i] = spl[(uint64_t)s * (NBmax - 1) + i];
  for (uint32_t i = threadIdx.x; i < NB; i += HIST_NT) cur[i] = base + (p[(uint64_t)i * ntiles] - rel);
  __syncthreads();
  if (nspl) dir.build<HIST_NT>(sp, nspl);
  const SplitView sv = dir.view(nspl);
  for (uint32_t i = a + threadIdx.x; i < b; i += HIST_NT) {
    const tup_t v = load_tup(gsrc + i);
    store_tup(dst + atomicAdd(&cur[dir.bucket(sv, sp, v.key)], 1u), v);
  }
}

// Start and key bounds of every global bucket g = seg_b0[s] + b.  bstart has
// G + 1 entries, G = seg_b0[nseg].  Every key of bucket b of segment s lies
// in [blo[g], bhi[g]]: the splitters around it (bucket b holds keys from
// spl[b-1] up to spl[b], the upper end for a key moved down by the
// equal-splitter rule), or the bounds of the enclosing segment, which are
// the splitters of the previous level (outer, with outer_nspl entries), or
// [0, 2^64-1] at the first level.
__global__ void k_bucket_table(uint32_t nseg, uint32_t NBmax, const uint32_t* seg_start, const uint32_t* seg_tile0,
                               const uint32_t* seg_cnt0, const uint32_t* seg_nb, const uint32_t* seg_b0,
                               const uint32_t* seg_len, const uint32_t* pos, const uint64_t* spl,
                               const uint64_t* outer, uint32_t outer_nspl, uint32_t* bstart, uint64_t* blo,
                               uint64_t* bhi) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t G = seg_b0[nseg];
  if (g > G) return;
  // the segments tile [0, n) in order (trailing empty ones start at n)
  if (g == G) { bstart[G] = seg_start[nseg - 1] + seg_len[nseg - 1]; return; }
  uint32_t lo = 0, hi = nseg;   // last s with seg_b0[s] <= g
  while (hi - lo > 1) { const uint32_t m = (lo + hi) >> 1; if (seg_b0[m] <= g) lo = m; else hi = m; }
  const uint32_t s = lo, b = g - seg_b0[s], nb = seg_nb[s];
  const uint32_t nt = seg_tile0[s + 1] - seg_tile0[s];
  bstart[g] = nt ? pos[seg_cnt0[s] + b * nt] : seg_start[s];
  const uint64_t olo = (outer && s > 0) ? outer[s - 1] : 0ull;
  const uint64_t ohi = (outer && s < outer_nspl) ? outer[s] : ~0ull;
  const uint64_t* sp = spl + (uint64_t)s * (NBmax - 1);
  blo[g] = b > 0 ? sp[b - 1] : olo;
  bhi[g] = b + 1 < nb ? sp[b] : ohi;
}

// Bucket table of a padded pass (one workgroup per segment): bucket g of
// segment s holds fill[g] tuples.  Its sorted output starts at the segment
// start plus the tuples of the segment's earlier buckets (bstart; bstart[G]
// = the end of the last segment), and its tuples are read from its region
// (bsrc = region start), or, for a segment the exact path redid, from the
// same compact offset inside the segment's area.  Key bounds as in
// k_bucket_table.
template <int NT>
__global__ void __launch_bounds__(NT) k_region_table(uint32_t nseg, uint32_t NBmax, const uint32_t* seg_start,
                                                     const uint32_t* seg_len, const uint32_t* seg_nb,
                                                     const uint32_t* seg_b0, Regions rg, const uint64_t* spl,
                                                     const uint64_t* outer, uint32_t outer_nspl, uint32_t* bstart,
                                                     uint32_t* bsrc, uint64_t* blo, uint64_t* bhi) {
  constexpr int PER = (MAX_NB + NT - 1) / NT;
  __shared__ uint32_t wsum[NT / 64 + 2];
  const uint32_t s = blockIdx.x, tid = threadIdx.x;
  const uint32_t nb = seg_nb[s], g0 = seg_b0[s];
  const bool redone = rg.dirty[s] != 0;
  uint32_t c[PER], loc[PER], run = 0;
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const uint32_t b = tid * PER + q;
    c[q] = b < nb ? rg.fill[g0 + b] : 0;
    loc[q] = run;
    run += c[q];
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan<NT>(run, wsum, &tot);
  const uint64_t* sp = spl + (uint64_t)s * (NBmax - 1);
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const uint32_t b = tid * PER + q;
    if (b < nb) {
      const uint32_t g = g0 + b, pre = loc[q] + ex;
      bstart[g] = seg_start[s] + pre;
      bsrc[g] = redone ? (uint32_t)pad_area(seg_start[s]) + pre : rg.start[g];
      blo[g] = b > 0 ? sp[b - 1] : ((outer && s > 0) ? outer[s - 1] : 0ull);
      bhi[g] = b + 1 < nb ? sp[b] : ((outer && s < outer_nspl) ? outer[s] : ~0ull);
    }
  }
  if (s == nseg - 1 && tid == 0) bstart[g0 + nb] = seg_start[s] + seg_len[s];
}

// ------------------------------------------------------------ bucket sort

struct SortOut {
  // S runs: every idx_stride-th key of each run (equi-height bounds)
  uint64_t* run_idx;
  const uint32_t* run_start;
  uint32_t idx_stride, idx_shift, idx_per_run, NB;   // idx_stride = 2^idx_shift
  // R buckets: first (smallest) key of every bucket
  uint64_t* bkey;
};

// Tuple of sorted rank r of bucket g (which starts at a): its key goes to
// the run index at every idx_stride-th run position, and to bkey at rank 0.
// The run's start is read through the constant address space (no kernel
// that sorts writes it), so it is a scalar load: a vector load issued after
// the bucket's stores would wait for every one of them.
__device__ __forceinline__ void emit_sorted(const SortOut& so, uint32_t g, uint32_t a, uint32_t r, uint64_t key) {
  if (so.run_idx) {
    const uint32_t s = g / so.NB;
    const uint32_t rs = *(__attribute__((address_space(4))) const uint32_t*)(so.run_start + s);
    const uint32_t rel = a + r - rs;
    if ((rel & (so.idx_stride - 1)) == 0) so.run_idx[(uint64_t)s * so.idx_per_run + (rel >> so.idx_shift)] = key;
  }
  if (so.bkey && r == 0) so.bkey[g] = key;
}

// Bucket sort by one counting pass plus a rank fix-up (the paper's sort is
// an MSD radix pass whose small partitions are finished by insertion sort,
// Section 2.3).  Keys of the bucket are mapped monotonically onto M
// sub-buckets by linear interpolation over the bucket's key bounds; one LDS
// counting sort groups the keys by sub-bucket, and every tuple is stored
// straight from registers to its final position (payloads never pass
// through LDS).  Inside a group a tuple's rank is the number of smaller
// keys plus the number of equal keys placed before it, so ranks form a
// permutation.  By group size:
//   * at most PIVMIN keys: ranked by comparing with every key of the group;
//   * at most GMAX keys: split three ways around the key at the group's first
//     position (a random member, so most often the group's most frequent
//     key): its copies count themselves, and only the other keys are ranked
//     by comparison;
//   * all keys equal (found from the group's min and max): positions stand;
//   * otherwise the group is sorted by a second counting pass that
//     interpolates over the group's own [min, max] into as many cells as it
//     has keys (keys clustered inside the bucket, duplicates of several
//     keys).  Second-level cells are ranked like first-level groups, and a
//     cell of more than GMAX keys is split three ways around a pivot key
//     taken from the cell: the copies of the pivot take the middle, the at
//     most SIDE other keys are ranked by comparison.
// A bucket that still has an unresolved cell, or more large groups than
// there are slots, goes to redo_list for the LSD radix sort
// (k_bucket_sort_lsd).  A bucket whose bounds admit one key is copied as is,
// whatever its size; other buckets larger than CAP go to over_list.  With
// in_list the kernel walks a list of bucket ids instead of all G buckets.
constexpr int CS_PIVMIN = 8;
constexpr int CS_GMAX = 32;
constexpr int CS_SIDE = 64;
constexpr int CS_SLOTS = 128;

enum : uint8_t { CS_DONE = 0, CS_BIG = 1, CS_SMALL2 = 2, CS_SMALL = 3 };

// Rank of key (at group position p) among the gs keys sk[gl, gl+gs).
__device__ __forceinline__ uint32_t cs_group_rank(const uint64_t* sk, uint32_t gl, uint32_t gs, uint32_t p,
                                                  uint64_t key) {
  uint32_t r = gl;
  if (gs <= 4) {   // common case: independent reads
#pragma unroll
    for (uint32_t t = 0; t < 4; t++) {
      const uint32_t q = gl + t;
      if (t < gs) { const uint64_t kq = sk[q]; r += (kq < key) || (kq == key && q < p); }
    }
  } else {
    for (uint32_t q = gl; q < gl + gs; q++) {
      const uint64_t kq = sk[q];
      r += (kq < key) || (kq == key && q < p);
    }
  }
  return r;
}

// bsrc (or NULL): where a bucket's tuples are read, when not at its output
// start in src (the regions of a padded pass).
template <int NT, int IPT, int M, int MINB, bool STAGE, bool TIGHT>
__global__ void __launch_bounds__(NT, MINB) k_bucket_sort_cs(const tup_t* __restrict__ src, tup_t* __restrict__ dst,
                                                       const uint32_t* bstart, const uint32_t* bsrc, const uint64_t* blo,
                                                       const uint64_t* bhi, const uint32_t* Gcount,
                                                       const uint32_t* in_list, const unsigned long long* in_count,
                                                       uint32_t* over_list, unsigned long long* over_count,
                                                       uint32_t* redo_list, unsigned long long* redo_count,
                                                       SortOut so) {
  constexpr int CAP = NT * IPT;
  constexpr int PER = M / NT;
  static_assert(M % NT == 0, "sub-buckets per thread");
  static_assert(CAP < (1 << 16), "positions fit 16 bits");
  // One LDS area holds the working arrays while ranks are computed and
  // then (STAGE), once every rank is known, the whole bucket in sorted order,
  // so the output leaves in fully coalesced stores; without STAGE every tuple
  // is stored straight from registers to its rank (fewer live registers).
  constexpr uint32_t OFF_SLOT1 = ((M + 1) * 4 + 15) / 16 * 16;
  constexpr uint32_t OFF_CNT2 = OFF_SLOT1 + (M * 2 + 15) / 16 * 16;
  constexpr uint32_t OFF_SK = OFF_CNT2 + ((CAP + 1) * 4 + 15) / 16 * 16;
  constexpr uint32_t WORK_BYTES = OFF_SK + CAP * 8;
  constexpr uint32_t AREA = WORK_BYTES > CAP * 16 ? WORK_BYTES : CAP * 16;
  // One LDS block in a fixed order: the small per-slot arrays first and the
  // counters at the front of the work area, so that the lane-indexed
  // accesses all fall within the 64 KiB an LDS instruction's immediate
  // offset reaches from one lane-scaled base register.
  struct __align__(16) Lds {
    uint64_t smin[CS_SLOTS], smax[CS_SLOTS], sC[CS_SLOTS];
    uint32_t sgs[CS_SLOTS];
    // per group in the pivot pass, at index (first position)/4: copies of
    // its pivot (bits 0..15) and other keys (bits 16..31) counted so far
    uint32_t gcnt[CAP / 4];
    uint32_t wsum[NT / 64 + 2];
    uint32_t nslot[2];   // large first-level groups (one spare word)
    uint32_t anyf[8];    // block_any flags, one per test below
    uint64_t wmin[NT / 64], wmax[NT / 64];   // per-wave key range (TIGHT)
    __align__(16) unsigned char area[AREA];
  };
  __shared__ Lds lds;
  unsigned char* const area = lds.area;
  uint32_t* const cnt = reinterpret_cast<uint32_t*>(area);                // first-level counters, then group starts
  uint16_t* const slot1 = reinterpret_cast<uint16_t*>(area + OFF_SLOT1);  // slot of a large first-level group
  uint32_t* const cnt2 = reinterpret_cast<uint32_t*>(area + OFF_CNT2);    // second-level counters, by position
  uint64_t* const sk = reinterpret_cast<uint64_t*>(area + OFF_SK);        // keys grouped by (sub-)group
  tup_t* const stage = reinterpret_cast<tup_t*>(area);                    // the sorted bucket
  uint64_t* const smin = lds.smin;
  uint64_t* const smax = lds.smax;
  uint64_t* const sC = lds.sC;
  uint32_t* const sgs = lds.sgs;
  uint32_t* const gcnt = lds.gcnt;
  uint32_t* const wsum = lds.wsum;
  uint32_t* const nslot = lds.nslot;
  uint32_t* const anyf = lds.anyf;
  const uint32_t tid = threadIdx.x;
  const uint32_t nitems = in_list ? (uint32_t)*in_count : *Gcount;
  // a grid of one workgroup per bucket takes the buckets XCD by XCD
  // (neighbouring buckets share an output line); a smaller grid strides
  const bool once = !in_list && gridDim.x >= nitems;
  for (uint32_t it = once ? xcd_item(blockIdx.x, nitems) : blockIdx.x; it < nitems;
       it += once ? nitems : gridDim.x) {
    const uint32_t g = in_list ? in_list[it] : it;
    const uint32_t a = bstart[g], n = bstart[g + 1] - a;
    if (n == 0) continue;
    // the bucket's tuples (uniform: kept in scalar registers)
    const uint32_t ain = __builtin_amdgcn_readfirstlane(bsrc ? bsrc[g] : a);
    const tup_t* const in = src + ain;
    uint64_t lo = blo[g], span = bhi[g] - lo;
    if (span == 0) {   // one key: input order is sorted order
      // Lane indexes pass through an empty asm where the lane's addresses
      // would otherwise be hoisted out of the bucket loop: live across the
      // whole loop they are spilled to scratch at every workgroup's start,
      // and those dead scratch lines are later written back to HBM.
      uint32_t i = tid;
      asm volatile("" : "+v"(i));
      for (; i + 3 * NT < n; i += 4 * NT) {   // four loads in flight
        tup_t t[4];
#pragma unroll
        for (int u = 0; u < 4; u++) t[u] = load_tup(in + i + u * NT);
#pragma unroll
        for (int u = 0; u < 4; u++) {
          store_tup(dst + a + i + u * NT, t[u]);
          emit_sorted(so, g, a, i + u * NT, lo);
        }
      }
      for (; i < n; i += NT) {
        store_tup(dst + a + i, load_tup(in + i));
        emit_sorted(so, g, a, i, lo);
      }
      continue;
    }
    if (n > (uint32_t)CAP) {
      if (tid == 0) over_list[atomicAdd(over_count, 1ull)] = g;
      continue;
    }
    uint64_t key[IPT], val[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      const uint32_t i = k * NT + tid;
      if (i < n) {
        const tup_t v = load_tup(in + i);
        key[k] = v.key; val[k] = v.pay;
      } else {
        key[k] = ~0ull; val[k] = 0;
      }
    }
    // LDS of the previous bucket is free (a workgroup that takes one bucket has none)
    if (!once) __syncthreads();
    for (uint32_t b = tid; b <= (uint32_t)M; b += NT) cnt[b] = 0;
    for (uint32_t b = tid; b < (uint32_t)(CAP / 4); b += NT) gcnt[b] = 0;
    if (tid < 2) nslot[tid] = 0;
    if (tid < 8) anyf[tid] = 0;
    __syncthreads();
    if constexpr (TIGHT) {
      // per-wave key range; the keys are first used here, two barriers
      // after their loads were issued, so that the loads overlap
      uint64_t mn = ~0ull, mx = 0;
#pragma unroll
      for (int k = 0; k < IPT; k++)
        if (k * NT + tid < n) { mn = key[k] < mn ? key[k] : mn; mx = key[k] > mx ? key[k] : mx; }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t x = __shfl_xor(mn, d, 64), y = __shfl_xor(mx, d, 64);
        mn = x < mn ? x : mn;
        mx = y > mx ? y : mx;
      }
      if ((tid & 63) == 0) { lds.wmin[tid >> 6] = mn; lds.wmax[tid >> 6] = mx; }
      __syncthreads();
      // interpolate over the keys' own range: the splitter bounds may enclose
      // empty key space (a segment's outer buckets, or a splitter that falls
      // in a gap between clusters), which would crowd the keys into few cells
      uint64_t bmn = lds.wmin[0], bmx = lds.wmax[0];
#pragma unroll
      for (int w = 1; w < NT / 64; w++) {
        bmn = lds.wmin[w] < bmn ? lds.wmin[w] : bmn;
        bmx = lds.wmax[w] > bmx ? lds.wmax[w] : bmx;
      }
      lo = bmn;
      span = bmx - bmn;
    }
    const bool exact = span < (uint64_t)M;   // one key per sub-bucket
    // sub-bucket: k - lo, or as a CellMap
    const uint32_t csh = cell_shift(span);
    const uint32_t C = cell_scale(M, (span >> csh) + 1);
    auto sub = [&](uint64_t k) -> uint32_t {
      const uint64_t x = k - lo;
      const uint32_t dd = exact ? (uint32_t)x : __umulhi((uint32_t)(x >> csh), C);
      return dd < (uint32_t)M ? dd : (uint32_t)(M - 1);
    };
    uint32_t fin[IPT];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      if (k * NT + tid < n) {
        bad |= key[k] - lo > span;            // outside the bucket's bounds: never expected
        fin[k] = atomicAdd(&cnt[sub(key[k])], 1u);
      }
    }
    __syncthreads();
    {
      uint32_t loc[PER], run = 0;
#pragma unroll
      for (int q = 0; q < PER; q++) { loc[q] = run; run += cnt[tid * PER + q]; }
      uint32_t tot;
      const uint32_t ex = block_excl_scan<NT>(run, wsum, &tot);
#pragma unroll
      for (int q = 0; q < PER; q++) cnt[tid * PER + q] = loc[q] + ex;
      if (tid == 0) cnt[M] = n;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      if (k * NT + tid < n) {
        fin[k] += cnt[sub(key[k])];
        if (!exact) sk[fin[k]] = key[k];
      }
    }
    bool any_bad;
    if (!exact) {
      // gs_[k]: start of the item's current group (bits 0..27) and its state
      // (bits 28..31).  aux[k], in the pivot pass: the group's size (bits
      // 0..13), the item's arrival index (bits 14..27) and whether its key
      // differs from the pivot (bit 28); in a second-level cell: the item's
      // arrival index, then for a small cell the cell's size.
      uint32_t gs_[IPT], aux[IPT];
      bool big = false, piv = false;
#define GL(k) (gs_[k] & 0x0FFFFFFFu)
#define ST(k) (gs_[k] >> 28)
#define SET(k, v) (gs_[k] = GL(k) | ((uint32_t)(v) << 28))
      // the group's pivot: the key found at two of three spread positions,
      // else the middle one
      auto pivot_of = [&](uint32_t gl, uint32_t gs) -> uint64_t {
        const uint64_t a0 = sk[gl], a1 = sk[gl + (gs >> 1)], a2 = sk[gl + gs - 1];
        return (a0 == a1 || a0 == a2) ? a0 : a1;
      };
      // whether two of the three agree in their low halves (a false match
      // only sends a group through the pivot pass, which counts exactly)
      auto may_agree = [&](uint32_t gl, uint32_t gs) -> bool {
        const uint32_t* lo32 = reinterpret_cast<const uint32_t*>(sk);
        const uint32_t a0 = lo32[2 * gl], a1 = lo32[2 * (gl + (gs >> 1))], a2 = lo32[2 * (gl + gs - 1)];
        return a0 == a1 || a0 == a2 || a1 == a2;
      };
      // a large first-level group's slot, opened by the item at its first position
      auto open_slot = [&](int k, uint32_t gl, uint32_t gs) {
        if (fin[k] == gl) {
          const uint32_t s = atomicAdd(&nslot[0], 1u);
          if (s < (uint32_t)CS_SLOTS) {
            slot1[sub(key[k])] = (uint16_t)s; smin[s] = key[k]; smax[s] = key[k]; sgs[s] = gs;
          }
        }
      };
      // Three-way split of the groups in state SMALL (keys at sk[gl, gl + gs))
      // around their pivots: the copies of the pivot count themselves and
      // follow the other keys that are smaller, and the at most SIDE other
      // keys are ranked by comparison among themselves.  A group with more
      // other keys goes, at the first level, to the second-level counting;
      // at the second level it makes the bucket a redo.
      auto pivot_pass = [&](bool first_level) {
#pragma unroll
        for (int k = 0; k < IPT; k++)
          if (ST(k) == CS_SMALL) {
            const uint32_t gl = GL(k);
            const bool other = key[k] != pivot_of(gl, aux[k] & 0x3FFFu);
            const uint32_t old = atomicAdd(&gcnt[gl >> 2], other ? 0x10000u : 1u);
            aux[k] |= ((other ? old >> 16 : old & 0xFFFFu) << 14) | ((uint32_t)other << 28);
          }
        __syncthreads();
        // the other keys move to the group's end, in arrival order from the
        // last position; the first copy of the pivot writes it at the start
#pragma unroll
        for (int k = 0; k < IPT; k++)
          if (ST(k) == CS_SMALL) {
            const uint32_t gl = GL(k), gs = aux[k] & 0x3FFFu, q = (aux[k] >> 14) & 0x3FFFu;
            if ((gcnt[gl >> 2] >> 16) <= (uint32_t)CS_SIDE) {
              if (aux[k] >> 28) sk[gl + gs - 1 - q] = key[k];
              else if (q == 0) sk[gl] = key[k];
            }
          }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; k++)
          if (ST(k) == CS_SMALL) {
            const uint32_t gl = GL(k), gs = aux[k] & 0x3FFFu, q = (aux[k] >> 14) & 0x3FFFu;
            const uint32_t c = gcnt[gl >> 2], no = c >> 16;
            if (no > (uint32_t)CS_SIDE) {
              if (first_level) {
                SET(k, CS_BIG);
                big = true;
                aux[k] = 0;
                open_slot(k, gl, gs);
              } else {
                bad = true;
              }
              continue;
            }
            const uint32_t ob = gl + gs - no;   // the other keys, at [ob, gl + gs)
            uint32_t r;
            if (aux[k] >> 28) {   // smaller other keys, then the pivot's copies if it is larger
              r = gl + (key[k] > sk[gl] ? (c & 0xFFFFu) : 0u);
#pragma unroll 2
              for (uint32_t t = 0; t < no; t++) {
                const uint64_t kq = sk[ob + t];
                r += (kq < key[k]) || (kq == key[k] && no - 1 - t < q);
              }
            } else {              // a copy of the pivot: after the other keys that are smaller
              r = gl + q;
#pragma unroll 2
              for (uint32_t t = 0; t < no; t++) r += sk[ob + t] < key[k];
            }
            fin[k] = r;
            SET(k, CS_DONE);
          }
      };
      __syncthreads();
#pragma unroll
      for (int k = 0; k < IPT; k++) {
        gs_[k] = 0;
        aux[k] = 0;
        if (k * NT + tid < n) {
          const uint32_t dd = sub(key[k]);
          const uint32_t l = cnt[dd], gs = cnt[dd + 1] - l;
          cnt2[fin[k]] = 0;
          gs_[k] = l;
          if (gs > (uint32_t)CS_PIVMIN) {
            // a large group whose three sampled keys all differ holds many
            // keys: straight to the second level
            if (gs > (uint32_t)CS_GMAX && !may_agree(l, gs)) {
              gs_[k] = l | ((uint32_t)CS_BIG << 28);
              big = true;
              open_slot(k, l, gs);
            } else {
              gs_[k] = l | ((uint32_t)CS_SMALL << 28);
              aux[k] = gs;
              piv = true;
            }
          } else if (gs > 1) {
            fin[k] = cs_group_rank(sk, l, gs, fin[k], key[k]);
          }
        }
      }
      bool any_big;
      if (block_any2(piv, big, &anyf[0], &anyf[1], &any_big)) {
        pivot_pass(true);
        any_big = block_any(big, &anyf[2]);
      }
      bool piv2 = false;
      if (any_big) {
        const uint32_t nbig = nslot[0];
        if (nbig > (uint32_t)CS_SLOTS) {
          bad = true;
        } else {
          // group bounds; a group's first item also clears the pivot-pass
          // counter at its start for the cells that may start there
#pragma unroll
          for (int k = 0; k < IPT; k++)
            if (ST(k) == CS_BIG) {
              const uint32_t s = slot1[sub(key[k])];
              atomicMin(reinterpret_cast<unsigned long long*>(&smin[s]), (unsigned long long)key[k]);
              atomicMax(reinterpret_cast<unsigned long long*>(&smax[s]), (unsigned long long)key[k]);
              if (fin[k] == GL(k)) gcnt[GL(k) >> 2] = 0;
            }
          __syncthreads();
          // second-level cells, as many as the group has keys; C = 0 marks a
          // span narrower than that (one key per cell)
          bool mixed = false;
          for (uint32_t s = tid; s < nbig; s += NT) {
            const uint64_t sp2 = smax[s] - smin[s];
            mixed |= sp2 != 0;
            sC[s] = sp2 < (uint64_t)sgs[s] ? 0ull : interp_scale(sgs[s], sp2);
          }
          // when every large group holds one key, their positions stand
          if (block_any(mixed, &anyf[3])) {
          auto cell = [&](uint32_t s, uint64_t k) -> uint32_t {
            const uint64_t x = k - smin[s], c = sC[s];
            const uint32_t c2 = c ? (uint32_t)__umul64hi(x, c) : (uint32_t)x;
            return c2 < sgs[s] ? c2 : sgs[s] - 1;
          };
#pragma unroll
          for (int k = 0; k < IPT; k++) {
            bool w = false;
            uint32_t c = 0;
            if (ST(k) == CS_BIG) {
              const uint32_t s = slot1[sub(key[k])];
              if (smin[s] == smax[s]) SET(k, CS_DONE);   // one key: positions stand
              else { w = true; c = GL(k) + cell(s, key[k]); }
            }
            if (w) aux[k] = atomicAdd(&cnt2[c], 1u);
          }
          __syncthreads();
          // exclusive scan of the second-level counters over the bucket
          {
            uint32_t t = tid;   // the lane's addresses are formed here, not hoisted
            asm volatile("" : "+v"(t));
            uint32_t loc[IPT], run = 0;
#pragma unroll
            for (int q = 0; q < IPT; q++) {
              const uint32_t i = t * IPT + q;
              loc[q] = run;
              run += i < n ? cnt2[i] : 0u;
            }
            uint32_t tot;
            const uint32_t ex = block_excl_scan<NT>(run, wsum, &tot);
#pragma unroll
            for (int q = 0; q < IPT; q++) {
              const uint32_t i = t * IPT + q;
              if (i < n) cnt2[i] = loc[q] + ex;
            }
            if (tid == 0) cnt2[n] = tot;
          }
          __syncthreads();
#pragma unroll
          for (int k = 0; k < IPT; k++)
            if (ST(k) == CS_BIG) {
              const uint32_t s = slot1[sub(key[k])];
              const uint32_t c2 = GL(k) + cell(s, key[k]);
              const uint32_t c0 = cnt2[c2];
              const uint32_t g2 = GL(k) + (c0 - cnt2[GL(k)]), gs2 = cnt2[c2 + 1] - c0;
              fin[k] = g2 + aux[k];
              sk[fin[k]] = key[k];
              if (gs2 <= 1) {
                SET(k, CS_DONE);
              } else if (gs2 <= (uint32_t)CS_PIVMIN) {
                gs_[k] = g2 | ((uint32_t)CS_SMALL2 << 28);
                aux[k] = gs2;
              } else {
                gs_[k] = g2 | ((uint32_t)CS_SMALL << 28);
                aux[k] = gs2;
                piv2 = true;
              }
            }
          __syncthreads();
#pragma unroll
          for (int k = 0; k < IPT; k++)
            if (ST(k) == CS_SMALL2) {
              fin[k] = cs_group_rank(sk, GL(k), aux[k], fin[k], key[k]);
              SET(k, CS_DONE);
            }
          }
        }
      }
      if (block_any2(piv2, bad, &anyf[4], &anyf[5], &any_bad)) {
        pivot_pass(false);
        any_bad = block_any(bad, &anyf[6]);
      }
#undef GL
#undef ST
#undef SET
    } else {
      any_bad = block_any(bad, &anyf[5]);
    }
    if (any_bad) {
      if (tid == 0) redo_list[atomicAdd(redo_count, 1ull)] = g;
      continue;
    }
    if constexpr (STAGE) {
      // every rank is known and the working arrays are free: stage, then copy
#pragma unroll
      for (int k = 0; k < IPT; k++) {
        if (k * NT + tid < n) {
          tup_t v; v.key = key[k]; v.pay = val[k];
          stage[fin[k]] = v;
        }
      }
      __syncthreads();
      uint32_t t = tid;   // the staged addresses are formed here, not hoisted
      asm volatile("" : "+v"(t));
#pragma unroll
      for (int k = 0; k < IPT; k++) {
        const uint32_t i = k * NT + t;
        if (i < n) {
          const tup_t v = stage[i];
          store_tup(dst + a + i, v);
          emit_sorted(so, g, a, i, v.key);
        }
      }
    } else {
      // every byte offset is formed before the first store and the index
      // entries follow the tuples: a register written between two stores
      // would be taken from a stored tuple, and writing it waits for that
      // store to complete
      tup_t* const out = dst + a;
#pragma unroll
      for (int k = 0; k < IPT; k++) {
        fin[k] *= (uint32_t)sizeof(tup_t);
        asm volatile("" : "+v"(fin[k]));
      }
      // the payloads arrive here, once: a load still pending at a store
      // that sits behind a branch makes that store wait for every earlier
      // store as well
#pragma unroll
      for (int k = 0; k < IPT; k++) asm volatile("" ::"v"(val[k]));
#pragma unroll
      for (int k = 0; k < IPT; k++) {
        if (k * NT + tid < n) {
          tup_t v; v.key = key[k]; v.pay = val[k];
          store_tup(reinterpret_cast<tup_t*>(reinterpret_cast<char*>(out) + fin[k]), v);
        }
      }
#pragma unroll
      for (int k = 0; k < IPT; k++)
        if (k * NT + tid < n) emit_sorted(so, g, a, fin[k] / (uint32_t)sizeof(tup_t), key[k]);
    }
  }
}

// LSD radix sort (BlockSort) of the buckets on a list, one workgroup per
// bucket; buckets larger than the tile go to over_list.
__global__ void __launch_bounds__(LSD_NT) k_bucket_sort_lsd(const tup_t* __restrict__ src, tup_t* __restrict__ dst,
                                                            const uint32_t* bstart, const uint32_t* bsrc,
                                                            const uint32_t* in_list,
                                                            const unsigned long long* in_count, uint32_t* over_list,
                                                            unsigned long long* over_count, SortOut so) {
  using Sorter = BlockSort<LSD_NT, LSD_IPT, 4>;
  __shared__ uint64_t buf[Sorter::BUF_WORDS];
  __shared__ uint32_t wsum[Sorter::WSUM_WORDS];
  __shared__ uint64_t red[LSD_NT / 64 + 1];
  const uint32_t tid = threadIdx.x;
  const uint32_t nitems = (uint32_t)*in_count;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const uint32_t g = in_list[it];
    const uint32_t a = bstart[g], n = bstart[g + 1] - a;
    if (n > (uint32_t)(LSD_NT * LSD_IPT)) {
      if (tid == 0) over_list[atomicAdd(over_count, 1ull)] = g;
      continue;
    }
    uint64_t key[LSD_IPT], val[LSD_IPT];
#pragma unroll
    for (int k = 0; k < LSD_IPT; k++) {
      const uint32_t i = k * LSD_NT + tid;
      if (i < n) { const tup_t v = load_tup(src + (bsrc ? bsrc[g] : a) + i); key[k] = v.key; val[k] = v.pay; }
      else { key[k] = ~0ull; val[k] = 0; }
    }
    Sorter::sort<true>(key, val, (int)n, buf, wsum, red);
#pragma unroll
    for (int k = 0; k < LSD_IPT; k++) {
      const uint32_t r = k * LSD_NT + tid;
      if (r < n) {
        tup_t v; v.key = key[k]; v.pay = val[k];
        store_tup(dst + a + r, v);
        emit_sorted(so, g, a, r, key[k]);
      }
    }
    __syncthreads();
  }
}

// Oversize buckets: one workgroup sorts a whole bucket through global memory
// with stable 4-bit LSD passes (only over the nibbles in which the bucket's
// keys differ), ping-ponging between src and dst ranges.  Each pass counts
// the digits of the whole bucket, then ranks chunks of 8192 tuples in LDS
// (each thread holds 8 consecutive tuples, which keeps the ranks stable)
// and writes every tuple to its digit's cursor.
constexpr int BIG_NT = 1024, BIG_IPT = 8;
__global__ void __launch_bounds__(BIG_NT) k_big_sort(tup_t* __restrict__ src, tup_t* __restrict__ dst,
                                                     const uint32_t* bstart, const uint32_t* bsrc,
                                                     const uint32_t* big_list,
                                                     const unsigned long long* big_count, SortOut so) {
  using RS = BlockSort<BIG_NT, BIG_IPT, 4>;
  constexpr uint32_t CH = BIG_NT * BIG_IPT;
  __shared__ uint64_t buf[RS::BUF_WORDS];
  __shared__ uint32_t wsum[RS::WSUM_WORDS];
  __shared__ uint64_t red[BIG_NT / 64 + 1];
  __shared__ uint32_t cur[16], ccnt[16], cpre[17];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t nbig = (uint32_t)*big_count;
  for (uint32_t e = blockIdx.x; e < nbig; e += gridDim.x) {
    const uint32_t g = big_list[e];
    const uint32_t a = bstart[g], n = bstart[g + 1] - a;
    tup_t* const in = src + (bsrc ? bsrc[g] : a);   // the bucket's tuples (room for n: its region)
    const uint64_t k0 = in[0].key;
    uint64_t vary = 0;
    for (uint32_t i = tid; i < n; i += BIG_NT) vary |= in[i].key ^ k0;
    vary = RS::block_or(vary, red);
    tup_t* from = in;
    tup_t* to = dst + a;
    for (int sh = 0; sh < 64; sh += 4) {
      if (((vary >> sh) & 15ull) == 0) continue;
      // digit counts of the whole bucket: 16-bit fields per thread, then wave sums
      uint64_t hw[4] = {0, 0, 0, 0};
      for (uint32_t i = tid; i < n; i += BIG_NT) {
        const uint32_t d = (uint32_t)(from[i].key >> sh) & 15u;
        const uint64_t inc = 1ull << (16 * (d & 3));
#pragma unroll
        for (int q = 0; q < 4; q++) hw[q] += (d >> 2) == (uint32_t)q ? inc : 0ull;
      }
      if (tid < 16) ccnt[tid] = 0;
      __syncthreads();
#pragma unroll
      for (int d = 0; d < 16; d++) {
        uint32_t c = (uint32_t)(hw[d >> 2] >> (16 * (d & 3))) & 0xFFFFu;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0 && c) atomicAdd(&ccnt[d], c);
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t run = 0;
        for (int d = 0; d < 16; d++) { cur[d] = run; run += ccnt[d]; }
      }
      __syncthreads();
      for (uint32_t c0 = 0; c0 < n; c0 += CH) {
        const uint32_t nv = n - c0 < CH ? n - c0 : CH;   // tuples of this chunk
        tup_t v[BIG_IPT];
        uint32_t d[BIG_IPT], r[BIG_IPT];
#pragma unroll
        for (int k = 0; k < BIG_IPT; k++) {
          const uint32_t i = tid * BIG_IPT + k;
          v[k].key = ~0ull; v[k].pay = 0;
          if (i < nv) v[k] = from[c0 + i];
          d[k] = i < nv ? (uint32_t)(v[k].key >> sh) & 15u : 15u;   // past the end: last, after the valid 15s
        }
        RS::rank(d, r, buf, wsum);   // stable rank in the chunk, digit-major
        // the chunk's digit starts are the rank counters of thread 0
        if (tid < 16) cpre[tid] = reinterpret_cast<const uint16_t*>(buf)[tid * BIG_NT];
        if (tid == 0) cpre[16] = nv;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BIG_IPT; k++)
          if (tid * BIG_IPT + k < nv) to[cur[d[k]] + (r[k] - cpre[d[k]])] = v[k];
        __syncthreads();
        if (tid < 16) cur[tid] += cpre[tid + 1] - cpre[tid];
        __syncthreads();
      }
      tup_t* t = from; from = to; to = t;
    }
    // the sorted data is in `from`
    for (uint32_t i = tid; i < n; i += BIG_NT) {
      const tup_t v = from[i];
      if (from != dst + a) dst[a + i] = v;
      emit_sorted(so, g, a, i, v.key);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ partitions

// Compact the non-empty R buckets into partitions p = 0..P-1 (start,
// length, first key) over the whole grid of buckets at once: flags of the
// non-empty buckets (k_partition_flags), their exclusive scan (pre), then
// every non-empty bucket writes its partition (k_partition_write).  Gmax:
// buckets the grid covers (>= *Gcount).
__global__ void k_partition_flags(const uint32_t* bstart, const uint32_t* Gcount, uint32_t Gmax, uint32_t* flags) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= Gmax) return;
  flags[g] = (g < *Gcount && bstart[g + 1] > bstart[g]) ? 1u : 0u;
}

__global__ void k_partition_write(const uint32_t* bstart, const uint64_t* bkey, uint32_t Gmax, const uint32_t* flags,
                                  const uint32_t* pre, uint32_t* Pcount, uint32_t* pstart, uint32_t* plen,
                                  uint64_t* pkey, Result* res) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t len = 0;
  if (g < Gmax && flags[g]) {
    const uint32_t p = pre[g];
    len = bstart[g + 1] - bstart[g];
    pstart[p] = bstart[g]; plen[p] = len; pkey[p] = bkey[g];
  }
  if (g + 1 == Gmax) *Pcount = pre[g] + flags[g];
  if (res) {   // statistics only: the largest partition, one atomic per wave
    unsigned long long m = len;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) { const unsigned long long x = __shfl_xor(m, d, 64); m = x > m ? x : m; }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(&res->spare, m);
  }
}

// B-MPSM (Section 2.1, Fig. 3: no range partitioning; every sorted R run
// meets every sorted S run): the partitions are the non-empty buckets of
// every sorted R run (key ranges inside that run, in order; NB buckets per
// run), and every run is closed by an empty terminator partition (pterm)
// whose start offsets are the S runs' lengths, so that the last partition
// of a run is joined with the tail of every S run and no join unit spans
// two R runs.
__global__ void __launch_bounds__(1024) k_partitions_runs(const uint32_t* bstart, const uint64_t* bkey,
                                                          const uint32_t* Gcount, uint32_t NB, uint32_t* Pcount,
                                                          uint32_t* pstart, uint32_t* plen, uint64_t* pkey,
                                                          uint8_t* pterm, Result* res) {
  __shared__ uint32_t wsum[1024 / 64 + 2];
  const uint32_t G = *Gcount;
  uint32_t carry = 0;
  for (uint32_t b = 0; b < G; b += 1024) {
    const uint32_t g = b + threadIdx.x;
    const uint32_t len = g < G ? bstart[g + 1] - bstart[g] : 0;
    const bool last = g < G && g % NB == NB - 1;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>((len ? 1u : 0u) + (last ? 1u : 0u), wsum, &tot);
    if (len) {
      const uint32_t p = carry + ex;
      pstart[p] = bstart[g]; plen[p] = len; pkey[p] = bkey[g]; pterm[p] = 0;
      if (res) atomicMax(&res->spare, (unsigned long long)len);
    }
    if (last) {
      const uint32_t p = carry + ex + (len ? 1u : 0u);
      pstart[p] = bstart[g + 1]; plen[p] = 0; pkey[p] = ~0ull; pterm[p] = 1;
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *Pcount = carry;
}


// ------------------------------------------------------------------ search

enum { SEARCH_BINARY = 0, SEARCH_INTERP = 1, SEARCH_LEARNED = 2, SEARCH_INDEX = 3 };

__device__ __forceinline__ uint32_t lb_keys(const tup_t* run, uint32_t lo, uint32_t hi, uint64_t key, uint32_t* probes) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    (*probes)++;
    if (run[mid].key < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t lb_window(const tup_t* run, uint32_t a, uint32_t b, uint64_t klo, uint64_t khi,
                                              uint64_t key, uint32_t* probes) {
  return lb_window_at([run](uint32_t i) { return run[i].key; }, a, b, klo, khi, key, probes);
}

// Interpolation search (Section 3.2.2, Fig. 7) with the invariant
// run[lo] < key <= run[hi]; bisection once a probe fails to halve the range
// twice or the range is at most 16.  Same answer as lower_bound.
__device__ __forceinline__ uint32_t interp_search(const tup_t* run, uint32_t n, uint64_t key, uint32_t* probes) {
  if (n == 0) return 0;
  (*probes)++;
  if (run[0].key >= key) return 0;
  (*probes)++;
  if (run[n - 1].key < key) return n;
  uint32_t lo = 0, hi = n - 1;
  int slow = 0;
  while (hi - lo > 1) {
    uint32_t m;
    if (hi - lo <= 16 || slow >= 2) {
      m = lo + ((hi - lo) >> 1);
    } else {
      const uint64_t klo = run[lo].key, khi = run[hi].key;
      // the proportion only picks the probe; the invariant keeps the answer exact
      const double f = (double)(key - klo) / (double)(khi - klo);
      m = lo + (uint32_t)(f * (double)(hi - lo));
      if (m <= lo) m = lo + 1;
      if (m >= hi) m = hi - 1;
    }
    const uint32_t before = hi - lo;
    (*probes)++;
    if (run[m].key < key) lo = m; else hi = m;
    if (2 * (hi - lo) > before) slow++;
  }
  return hi;
}

// o[p][j] = first position of run j whose key >= pkey[p]; o[P][j] = |S_j|.
// Modes: BINARY bisects the run; INTERP is the paper's interpolation search;
// INDEX bisects the run's equi-height index (every idx_stride-th key) and
// then the idx_stride-wide window; LEARNED predicts the index slot from the
// learned CDF of S, checks that the answer is bracketed by a window of
// +-eps slots around the prediction, bisects that window (or, when the check
// fails, the whole index), then the run window.  All modes return the same
// lower bound.
// Lower bound of key in a sorted run of n tuples by BINARY, INTERP or INDEX
// (bisection of the run's equi-height index idx of nidx keys, every
// idx_stride-th key, then of the idx_stride-wide window).
__device__ __forceinline__ uint32_t run_lower_bound(int mode, const tup_t* run, uint32_t n, uint64_t key,
                                                    const uint64_t* idx, uint32_t idx_stride, uint32_t* probes) {
  if (mode == SEARCH_BINARY) return lb_keys(run, 0, n, key, probes);
  if (mode == SEARCH_INTERP) return interp_search(run, n, key, probes);
  const uint32_t nidx = (n + idx_stride - 1) / idx_stride;
  uint32_t lo = 0, hi = nidx;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    (*probes)++;
    if (idx[mid] < key) lo = mid + 1; else hi = mid;
  }
  const uint32_t a = lo ? (lo - 1) * idx_stride + 1 : 0;
  const uint32_t b = lo < nidx ? lo * idx_stride : n;
  return lb_window(run, a, b, lo ? idx[lo - 1] : 0ull, lo < nidx ? idx[lo] : ~0ull, key, probes);
}

// The learned search's prediction for every partition's first key and the
// model's error near it (one evaluation per partition, not per partition
// and run: the key is the same in every run).
__global__ void k_search_model(const CdfModel* model, const uint64_t* pkey, const uint32_t* Pcount, uint32_t Pmax,
                               float2* qe) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const CdfModel& m = *model;
  if (p >= *Pcount || p >= Pmax || !m.valid) return;
  const float q = cdf_eval(m, pkey[p]);
  qe[p] = make_float2(q, cdf_local_eps(m, q));
}

// Launch shape: a wave takes 64 consecutive partitions of one run, so the
// first levels of its lanes' bisections read the same index entries and the
// last ones neighbouring lines; a workgroup takes 16 runs, so that each row
// o[p][.] is written in 64-byte pieces.  Blocks: cdiv(Pmax + 1, 64) *
// cdiv(Q, SEARCH_RUNS), runs fastest.
constexpr int SEARCH_NT = 1024;
constexpr int SEARCH_RUNS = SEARCH_NT / 64;

__global__ void __launch_bounds__(SEARCH_NT) k_search(const tup_t* __restrict__ U, const uint32_t* run_start,
                                                const uint32_t* run_len, uint32_t Q, const uint64_t* run_idx,
                                                uint32_t idx_stride, uint32_t idx_per_run, const uint32_t* Pcount,
                                                const uint64_t* pkey, uint32_t Pmax, uint32_t* o, int mode,
                                                const CdfModel* model, const float2* qe, Result* res,
                                                const uint8_t* span, const uint8_t* pterm) {
  const bool learned = mode == SEARCH_LEARNED;
  const CdfModel& m = *model;   // read through the caches: its knots are shared by all threads
  const uint32_t njt = (Q + SEARCH_RUNS - 1) / SEARCH_RUNS;
  const uint32_t p = (blockIdx.x / njt) * 64 + (threadIdx.x & 63);
  const uint32_t j = (blockIdx.x % njt) * SEARCH_RUNS + (threadIdx.x >> 6);
  const uint32_t P = *Pcount;
  uint32_t probes = 0, fallbacks = 0;
  // rows of partitions that do not start a join unit are never read
  if (p <= P && p <= Pmax && j < Q && (p == P || span[p])) {
    const uint32_t n = run_len[j];
    const tup_t* run = U + run_start[j];
    uint32_t r;
    if (p == P || (pterm && pterm[p])) {   // the end of the runs (B-MPSM: of every R run)
      r = n;
    } else {
      const uint64_t key = pkey[p];
      if (mode == SEARCH_BINARY) {
        r = lb_keys(run, 0, n, key, &probes);
      } else if (mode == SEARCH_INTERP) {
        r = interp_search(run, n, key, &probes);
      } else {
        const uint64_t* idx = run_idx + (uint64_t)j * idx_per_run;
        const uint32_t nidx = (n + idx_stride - 1) / idx_stride;
        uint32_t lo = 0, hi = nidx;
        if (learned && m.valid) {
          // window: the model's error on its sample near the prediction, plus the sampling error of
          // a 2^16-key sample and of this run (two standard deviations each)
          const float2 pq = qe[p];   // the prediction for the key and the model's error near it
          const float q = pq.x;
          const float sd = sqrtf(q * (1.f - q) + 1e-4f);
          const float err = pq.y + 2.f * sd * (1.f / 256.f + rsqrtf((float)n + 1.f));
          const int64_t t = (int64_t)(q * (float)nidx);
          const int64_t w = (int64_t)(err * (float)nidx) + 2;
          const uint32_t a = (uint32_t)(t - w < 0 ? 0 : (t - w > (int64_t)nidx ? (int64_t)nidx : t - w));
          const uint32_t b = (uint32_t)(t + w > (int64_t)nidx ? (int64_t)nidx : (t + w < (int64_t)a ? (int64_t)a : t + w));
          bool ok = true;
          if (a > 0) { probes++; ok = idx[a - 1] < key; }
          if (ok && b < nidx) { probes++; ok = idx[b] >= key; }
          if (ok) { lo = a; hi = b; } else { fallbacks++; }
        }
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          probes++;
          if (idx[mid] < key) lo = mid + 1; else hi = mid;
        }
        const uint32_t a = lo ? (lo - 1) * idx_stride + 1 : 0;
        const uint32_t b = lo < nidx ? lo * idx_stride : n;
        r = lb_window(run, a, b, lo ? idx[lo - 1] : 0ull, lo < nidx ? idx[lo] : ~0ull, key, &probes);
      }
    }
    o[(uint64_t)p * Q + j] = r;
  }
  if (res) {  // statistics only: one atomic per wave
    unsigned long long pr = probes, fb = fallbacks;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) { pr += __shfl_xor(pr, d, 64); fb += __shfl_xor(fb, d, 64); }
    if ((threadIdx.x & 63) == 0) {
      if (pr) atomicAdd(&res->search_probes, pr);
      if (fb) atomicAdd(&res->fallbacks, fb);
    }
  }
}

// ------------------------------------------------------------------- join

// Join units: partitions 2i and 2i+1 are joined as one unit when together
// they fit the LDS tile (they are adjacent in key order and in the sorted
// R, and their slices of every run are adjacent too), which halves the
// per-item setup of the join for small partitions.  span[p] = partitions in
// the unit starting at p (2 or 1), 0 for the second partition of a unit.
// same(p) says whether partitions p and p + 1 may share a unit.
template <typename F>
__device__ __forceinline__ uint32_t join_span(const uint32_t* plen, uint32_t P, uint32_t p, F same) {
  if (p & 1) return (plen[p - 1] + plen[p] <= (uint32_t)JOIN_CAP && same(p - 1)) ? 0u : 1u;
  return (p + 1 < P && plen[p] + plen[p + 1] <= (uint32_t)JOIN_CAP && same(p)) ? 2u : 1u;
}

// The join units of all partitions (before the start search, which only
// needs the rows of partitions that start a unit).  With B-MPSM's
// terminators (pterm) a terminator never shares a unit.
__global__ void k_join_units(const uint32_t* Pcount, const uint32_t* plen, uint32_t Pmax, uint8_t* span,
                             const uint8_t* pterm) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t P = *Pcount;
  if (p < P && p < Pmax)
    span[p] = (uint8_t)join_span(plen, P, p, [&](uint32_t q) { return !pterm || (!pterm[q] && !pterm[q + 1]); });
}

// Work items: join unit u contributes ceil(n_u / JCH) items, n_u = S tuples
// in its slices (0 when nothing can match).  items has Pmax + 2 entries.
// One wave per partition: its lanes read the unit's two rows of offsets
// across the runs side by side (each row is Q consecutive words), then add.
__global__ void k_join_items(const uint32_t* Pcount, const uint32_t* o, uint32_t Q, const uint32_t* run_len,
                             uint32_t Pmax, uint32_t JCH, const uint8_t* span, uint32_t* items) {
  const uint32_t p = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t lane = threadIdx.x & 63;
  if (p > Pmax + 1) return;
  const uint32_t P = *Pcount;
  const uint32_t sp = p < P ? span[p] : 0u;
  uint64_t np = 0;
  if (sp) {
    const uint32_t* a = o + (uint64_t)p * Q;
    const uint32_t* b = a + (uint64_t)sp * Q;
    for (uint32_t j = lane; j < Q; j += 64) np += slice_len(a[j], b[j], run_len[j]);   // as in k_join
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) np += __shfl_xor(np, d, 64);
  if (lane == 0) items[p] = (uint32_t)((np + JCH - 1) / JCH);
}

enum { VAL_HR = 0, VAL_RAW = 1 };

struct JoinArgs {
  const tup_t* Rs;          // R sorted, partitions contiguous
  const tup_t* U;           // S runs sorted
  const uint32_t* run_start;
  const uint32_t* run_len;
  uint32_t Q;
  const uint32_t* Pcount;
  const uint32_t* pstart;
  const uint32_t* plen;
  const uint32_t* o;
  const uint32_t* item_pre; // exclusive prefix of items, Pmax + 2 entries
  uint32_t Pmax;
  uint32_t JCH;
  Result* res;
  // pairs
  uint64_t* pairs;          // 3 u64 per pair (key, caller-R payload, caller-S payload)
  uint64_t pairs_cap;
  uint32_t* item_cnt;       // per-item pair counts (count pass) / offsets (write pass)
  uint32_t item_cap;        // entries of item_cnt
  int swapped;              // internal R is the caller's S
  // batch: per-join table and the join of every partition
  BatchJoin* J;
  const uint32_t* pjoin;
  const uint8_t* span;      // partitions per join unit (see join_span)
};

__device__ __forceinline__ uint32_t item_partition(const uint32_t* item_pre, uint32_t np2, uint32_t item) {
  uint32_t lo = 0, hi = np2 - 1;  // last p with item_pre[p] <= item
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (item_pre[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// Join kernel (phase 4).  A work item is a range of partition p's S tuples,
// counted along the concatenation of its slices S_j[o[p][j], o[p+1][j]).  The
// workgroup holds R_p in LDS (keys plus, per key, either the R-side hash
// prefix or the raw payload), with a directory over R_p's key range; every S
// tuple of the item is matched by a lower-bound search that the directory
// narrows to a few keys, and each match adds one pair.  Every S tuple belongs
// to exactly one slice of one partition, so each pair is produced once.
// Partitions larger than the LDS tile are searched in global memory.
// MODE 0: count + checksum (+max); MODE 1: count pairs per item; MODE 2: write
// pairs.  VM: what the LDS holds next to each R key.
constexpr int JOIN_U = 4;     // S tuples per thread per batch (two batches in flight)

template <int MODE, int VM, bool BATCH = false>
__global__ void __launch_bounds__(JOIN_NT) k_join(JoinArgs A) {
  __shared__ uint64_t rk[JOIN_CAP];
  __shared__ uint64_t rv[JOIN_CAP];
  __shared__ uint32_t cum[JOIN_QMAX + 1];
  __shared__ uint32_t sbase[JOIN_QMAX];
  __shared__ uint16_t jdir[JOIN_DIR + 1];
  __shared__ uint16_t rdir[JOIN_RDIR];
  __shared__ uint32_t wsum[JOIN_NT / 64 + 2];
  __shared__ uint64_t red[JOIN_NT / 64 + 1];
  __shared__ unsigned long long item_acc;
  __shared__ uint64_t jhi;
  __shared__ CellMap jmap;
  const uint32_t tid = threadIdx.x;
  const uint32_t np2 = A.Pmax + 2;
  // the pair passes keep one entry per item
  const uint32_t total = MODE == 0 ? A.item_pre[np2 - 1] : min(A.item_pre[np2 - 1], A.item_cap);
  unsigned long long cnt = 0, sum = 0, mx = 0;
  bool any = false;
  constexpr int JPF = JOIN_CAP / JOIN_NT;   // R tuples per thread
  tup_t pre[JPF];                          // next item's R partition, loaded during this item
  bool have_pre = false;
  // Workgroup b runs on XCD b mod 8.  Items are taken in rounds of
  // gridDim.x consecutive items; within a round the workgroups of one XCD
  // take neighbouring items (neighbouring join units, whose slices of a run
  // share their end lines), so those lines meet in one L2.
  const uint32_t item0 = gridDim.x % N_XCD == 0 ? (blockIdx.x % N_XCD) * (gridDim.x / N_XCD) + blockIdx.x / N_XCD
                                                : blockIdx.x;
  for (uint32_t item = item0; item < total; item += gridDim.x) {
    const uint32_t p = item_partition(A.item_pre, np2, item);
    const uint32_t k = item - A.item_pre[p];
    const uint32_t pe = p + A.span[p];   // the item's join unit: partitions [p, pe)
    const uint32_t rs = A.pstart[p], rn = A.pstart[pe - 1] + A.plen[pe - 1] - rs;
    // the unit's rows of start offsets and its runs (in a batch: those of its join)
    uint32_t Q = A.Q, r0 = 0, jb = 0;
    const uint32_t* oa = A.o + (uint64_t)p * Q;
    if (BATCH) {
      jb = A.pjoin[p];
      Q = A.J[jb].Q;
      r0 = A.J[jb].r0;
      oa = A.o + A.J[jb].obase + (uint64_t)(p - A.J[jb].p0) * Q;
      if (tid == 0) atomicMin(&A.J[jb].t_first, (unsigned long long)wall_clock64());
    }
    const uint32_t* ob = oa + (uint64_t)(pe - p) * Q;
    __syncthreads();   // LDS of the previous item is free
    // prefix of slice lengths over the runs; sbase[j] + x = S position of
    // concatenated index x when x falls in run j
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < Q; j0 += JOIN_NT) {
      const uint32_t j = j0 + tid;
      // clamped so that every read stays inside run j whatever the offsets hold
      const uint32_t nj = j < Q ? A.run_len[r0 + j] : 0;
      const uint32_t len = j < Q ? slice_len(oa[j], ob[j], nj) : 0;
      uint32_t tot;
      const uint32_t ex = block_excl_scan<JOIN_NT>(len, wsum, &tot);
      if (j < Q) { cum[j] = carry + ex; sbase[j] = slice_base(A.run_start[r0 + j], oa[j], nj, carry + ex); }
      carry += tot;
      __syncthreads();
    }
    if (tid == 0) { cum[Q] = carry; item_acc = 0; }
    const bool in_lds = rn <= (uint32_t)JOIN_CAP;
    if (in_lds) {
#pragma unroll
      for (int r = 0; r < JPF; r++) {
        const uint32_t i = r * JOIN_NT + tid;
        if (i < rn) {
          const tup_t t = have_pre ? pre[r] : load_tup(A.Rs + rs + i);
          rk[i] = t.key;
          rv[i] = (VM == VAL_HR) ? r_prefix_hash(t.key, t.pay) : t.pay;
        }
      }
    }
    // start loading the next item's partition; it arrives while this one is joined
    have_pre = false;
    {
      const uint32_t nxt = item + gridDim.x;
      if (nxt < total) {
        const uint32_t p2 = item_partition(A.item_pre, np2, nxt);
        const uint32_t pe2 = p2 + A.span[p2];
        const uint32_t rs2 = A.pstart[p2], rn2 = A.pstart[pe2 - 1] + A.plen[pe2 - 1] - rs2;
        if (rn2 <= (uint32_t)JOIN_CAP) {
#pragma unroll
          for (int r = 0; r < JPF; r++) {
            const uint32_t i = r * JOIN_NT + tid;
            if (i < rn2) pre[r] = load_tup(A.Rs + rs2 + i);
          }
          have_pre = true;
        }
      }
    }
    __syncthreads();
    // directory over R_p's key range: jdir[c] = first position whose cell is
    // >= c (cells are monotone in the key); a key in cell c has its lower
    // bound in [jdir[c], jdir[c+1]].  Built in one pass over the keys.
    if (in_lds) {
      if (tid == 0) {
        jhi = rk[rn - 1];
        jmap.init(rk[0], rk[rn - 1] - rk[0], JOIN_DIR);
      }
      __syncthreads();
      const CellMap mp = jmap;
      // cells are clamped to the directory, so the fill stays bounded even
      // if the partition were not sorted
      auto cell_of = [&](uint64_t key) -> int {
        const uint32_t x = mp(key);
        return x < (uint32_t)JOIN_DIR ? (int)x : JOIN_DIR - 1;
      };
      for (uint32_t i = tid; i < rn; i += JOIN_NT) {
        const int ci = cell_of(rk[i]);
        const int cp = i ? cell_of(rk[i - 1]) : -1;
        for (int cc = cp + 1; cc <= ci; cc++) jdir[cc] = (uint16_t)i;
      }
      const int clast = cell_of(rk[rn - 1]);
      for (int cc = (int)tid; cc <= JOIN_DIR; cc += JOIN_NT)
        if (cc > clast) jdir[cc] = (uint16_t)rn;
      __syncthreads();
    }
    const CellMap dmap = jmap;
    const uint64_t dlo = dmap.lo, dhi = jhi;
    const uint32_t lo_item = k * A.JCH;
    const uint32_t hi_item = min(lo_item + A.JCH, cum[Q]);
    const tup_t* Rg = A.Rs + rs;
    // run directory of the item: rdir[d] = run of position lo_item + 2^rsh d
    // (64 positions per entry where the item allows: a slice is often
    // shorter than 256 positions when there are many runs),
    // so that a position's run is found between two neighbouring entries
    const uint32_t rsh = A.JCH <= 64u * (JOIN_RDIR - 1) ? 6u : 8u;
    const uint32_t nd = (hi_item - lo_item + (1u << rsh) - 1) >> rsh;
    for (uint32_t d = tid; d < nd; d += JOIN_NT) {
      const uint32_t x = lo_item + (d << rsh);
      uint32_t a0 = 0, b0 = Q;
      while (b0 - a0 > 1) { const uint32_t m = (a0 + b0) >> 1; if (cum[m] <= x) a0 = m; else b0 = m; }
      rdir[d] = (uint16_t)a0;
    }
    __syncthreads();
    // S tuples of the item, JOIN_U per thread per batch; the next batch is
    // loaded while the current one is matched
    auto load_batch = [&](uint32_t base, tup_t (&sv)[JOIN_U]) {
#pragma unroll
      for (int u = 0; u < JOIN_U; u++) {
        const uint32_t x = base + u * JOIN_NT + tid;
        if (x < hi_item) {
          const uint32_t d = (x - lo_item) >> rsh;   // run j: cum[j] <= x < cum[j+1]
          uint32_t a0 = rdir[d], b0 = d + 1 < nd ? rdir[d + 1] + 1u : Q;
          while (b0 - a0 > 1) { const uint32_t m = (a0 + b0) >> 1; if (cum[m] <= x) a0 = m; else b0 = m; }
          sv[u] = load_tup(A.U + sbase[a0] + x);
        }
      }
    };
    tup_t nsv[JOIN_U];
    if (lo_item < hi_item) load_batch(lo_item, nsv);
    for (uint32_t base = lo_item; base < hi_item; base += JOIN_NT * JOIN_U) {
      tup_t sv[JOIN_U];
#pragma unroll
      for (int u = 0; u < JOIN_U; u++) sv[u] = nsv[u];
      if (base + JOIN_NT * JOIN_U < hi_item) load_batch(base + JOIN_NT * JOIN_U, nsv);
#pragma unroll
      for (int u = 0; u < JOIN_U; u++) {
        const uint32_t x = base + u * JOIN_NT + tid;
        if (x >= hi_item) continue;
        const tup_t s = sv[u];
        uint32_t lo = 0, hi = rn;
        if (in_lds) {
          if (s.key <= dlo) {
            hi = 0;
          } else if (s.key > dhi) {
            lo = rn;
          } else {
            const uint32_t cell = dmap(s.key);   // dlo < key <= dhi: below JOIN_DIR
            lo = jdir[cell];
            hi = jdir[cell + 1];
            while (lo < hi) { const uint32_t mid = (lo + hi) >> 1; if (rk[mid] < s.key) lo = mid + 1; else hi = mid; }
          }
        } else {
          while (lo < hi) { const uint32_t mid = (lo + hi) >> 1; if (Rg[mid].key < s.key) lo = mid + 1; else hi = mid; }
        }
        const uint64_t hk = (VM == VAL_RAW) ? mix64(s.key + MPSM_GAMMA) : 0;
        for (uint32_t q = lo; q < rn; q++) {
          uint64_t rkey, rval;
          if (in_lds) { rkey = rk[q]; rval = rv[q]; }
          else { const tup_t t = load_tup(Rg + q); rkey = t.key; rval = (VM == VAL_HR) ? r_prefix_hash(t.key, t.pay) : t.pay; }
          if (rkey != s.key) break;
          // caller orientation: (key, R payload, S payload)
          uint64_t h, rp_c = 0, sp_c = 0;
          if (VM == VAL_HR) {
            h = mix64(rval + s.pay);
          } else {
            rp_c = A.swapped ? s.pay : rval;
            sp_c = A.swapped ? rval : s.pay;
            h = mix64(mix64(hk + rp_c) + sp_c);
          }
          if (MODE == 0) {
            cnt++; sum += h;
            if (VM == VAL_RAW) { const uint64_t ps = rp_c + sp_c; mx = (!any || ps > mx) ? ps : mx; any = true; }
          } else if (MODE == 1) {
            cnt++;
          } else {
            const unsigned long long at = atomicAdd(&item_acc, 1ull) + A.item_cnt[item];
            if (at < A.pairs_cap) {
              A.pairs[3 * at] = s.key; A.pairs[3 * at + 1] = rp_c; A.pairs[3 * at + 2] = sp_c;
            }
          }
        }
      }
    }
    if (MODE == 1) {
      const uint64_t c = block_sum64<JOIN_NT>(cnt, red);
      if (tid == 0) A.item_cnt[item] = (uint32_t)c;
      cnt = 0;
    }
    if (BATCH && MODE == 0) {
      // a batch flushes every item into its join, and the join's last item
      // stamps the finishing time
      const uint64_t c = block_sum64<JOIN_NT>(cnt, red);
      const uint64_t sm = block_sum64<JOIN_NT>(sum, red);
      if (tid == 0) {
        if (c) { atomicAdd(&A.J[jb].count, (unsigned long long)c); atomicAdd(&A.J[jb].checksum, (unsigned long long)sm); }
        __threadfence();
        if (atomicAdd(&A.J[jb].done, 1u) + 1 == A.J[jb].items) A.J[jb].t_done = wall_clock64();
      }
      cnt = 0;
      sum = 0;
    }
  }
  if (MODE == 0 && !BATCH) {
    const uint64_t c = block_sum64<JOIN_NT>(cnt, red);
    const uint64_t sm = block_sum64<JOIN_NT>(sum, red);
    if (tid == 0) {
      if (c) { atomicAdd(&A.res->count, (unsigned long long)c); atomicAdd(&A.res->checksum, (unsigned long long)sm); }
    }
    if (VM == VAL_RAW) {
      const uint64_t m = block_max64<JOIN_NT>(any ? mx : 0, red);
      const uint64_t an = block_sum64<JOIN_NT>(any ? 1 : 0, red);
      if (tid == 0 && an) { atomicMax(&A.res->maxsum, (unsigned long long)m); atomicOr(&A.res->nonempty, 1ull); }
    }
  }
}
