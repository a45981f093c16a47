// Device-side basics shared by the MPSM kernels: tuple type, SplitMix64,
// wave64 scans, and the bucket function of sampled splitters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MPSM_GAMMA 0x9E3779B97F4A7C15ull

struct __align__(16) tup_t {
  uint64_t key;
  uint64_t pay;
};

// SplitMix64 output function (Steele, Lea, Flood 2014).  Also the building
// block of the per-pair checksum term.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// i-th output (0-based) of SplitMix64 seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i) {
  return mix64(seed + (i + 1) * MPSM_GAMMA);
}

// floor(x * n / 2^64): uniform index in [0, n) from a 64-bit draw.
__device__ __forceinline__ uint64_t draw_below(uint64_t x, uint64_t n) { return __umul64hi(x, n); }

// Checksum of one output pair given the R-side prefix hr = mix(mix(k+g)+rp).
__device__ __forceinline__ uint64_t r_prefix_hash(uint64_t key, uint64_t rp) {
  return mix64(mix64(key + MPSM_GAMMA) + rp);
}

__device__ __forceinline__ tup_t load_tup(const tup_t* p) {
  ulonglong2 v = *reinterpret_cast<const ulonglong2*>(p);
  tup_t t; t.key = v.x; t.pay = v.y;
  return t;
}
// Tuples known to be in device (global) memory.  A pointer read from a
// table is generic to the compiler, which then issues flat loads; a flat
// load also counts in the LDS wait counter, so every later wait for an LDS
// access would wait for it too (and drain a prefetch).  Reads through this
// type are global loads.
typedef __attribute__((address_space(1))) const tup_t gtup_t;
__device__ __forceinline__ const gtup_t* as_global(const tup_t* p) { return (const gtup_t*)p; }
__device__ __forceinline__ tup_t load_tup(const gtup_t* p) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const u64x2 v = *reinterpret_cast<__attribute__((address_space(1))) const u64x2*>(p);
  tup_t t; t.key = v.x; t.pay = v.y;
  return t;
}
__device__ __forceinline__ void store_tup(tup_t* p, tup_t t) {
  ulonglong2 v; v.x = t.key; v.y = t.pay;
  *reinterpret_cast<ulonglong2*>(p) = v;
}

// The workgroups of a launch are handed to the 8 XCDs in turn (workgroup
// b to XCD b mod 8), and each XCD has its own L2.  xcd_item gives workgroup b
// the k-th item (k = b / 8) of its XCD's contiguous share of n items, so
// that neighbouring items (the tiles of one segment, the buckets of one
// run), whose outputs share cache lines at their ends, run on one XCD and
// those lines are completed in its L2 before they are written back.  A
// bijection of [0, n) for any grid of at least n workgroups; workgroups
// without an item get n.
constexpr uint32_t N_XCD = 8;
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t n) {
  const uint32_t x = b % N_XCD, k = b / N_XCD, per = n / N_XCD, rem = n % N_XCD;
  const uint32_t cnt = per + (x < rem ? 1u : 0u);
  return k < cnt ? x * per + (x < rem ? x : rem) + k : n;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Inclusive scan of a u32 across the 64 lanes of a wave, with DPP lane
// moves (no LDS round trip): shifts by 1, 2, 4, 8 inside each row of 16
// lanes, then the row totals are carried with the row broadcasts of lane 15
// (into rows 1 and 3) and lane 31 (into rows 2 and 3).  Lanes whose source
// is outside the row receive 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return (uint32_t)x;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of one u32 per thread across a block of NT threads.
// `wsum` is LDS scratch of NT/64 + 1 words.  Returns the exclusive prefix;
// *total gets the block total.  Contains two barriers.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    uint32_t x = lane < NW ? wsum[lane] : 0u;
    uint32_t xi = wave_incl_scan(x);
    if (lane < NW) wsum[lane] = xi - x;
    if (lane == NW - 1) wsum[NW] = xi;
  }
  __syncthreads();
  uint32_t r = wsum[w] + inc - v;
  *total = wsum[NW];
  return r;
}

// Workgroup-wide OR of v through one LDS word that is zero on entry and is
// not written again until every thread has returned (the caller clears it
// behind a later barrier).  Ends with a barrier.  Uses only threadIdx.x, so
// no other work-item id stays live in the caller's loops.
__device__ __forceinline__ bool block_any(bool v, uint32_t* flag) {
  if (__any(v) && (threadIdx.x & 63) == 0) *flag = 1u;
  __syncthreads();
  return *flag != 0u;
}

// block_any of two values behind one barrier; returns the first, *b2 the second.
__device__ __forceinline__ bool block_any2(bool v1, bool v2, uint32_t* f1, uint32_t* f2, bool* b2) {
  const bool w1 = __any(v1), w2 = __any(v2);
  if ((threadIdx.x & 63) == 0) {
    if (w1) *f1 = 1u;
    if (w2) *f2 = 1u;
  }
  __syncthreads();
  *b2 = *f2 != 0u;
  return *f1 != 0u;
}

template <int NT>
__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t* wsum) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  __syncthreads();
  if (lane == 0) wsum[w] = v;
  __syncthreads();
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) s += wsum[i];
  return s;
}

template <int NT>
__device__ __forceinline__ uint64_t block_max64(uint64_t v, uint64_t* wsum) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) { uint64_t o = __shfl_xor(v, d, 64); v = o > v ? o : v; }
  __syncthreads();
  if (lane == 0) wsum[w] = v;
  __syncthreads();
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) s = wsum[i] > s ? wsum[i] : s;
  return s;
}

// Bucket of `key` under nspl sorted splitters (bucket b = [spl[b-1], spl[b])):
// the number of splitters <= key, except that a key equal to two or more
// splitters goes to the otherwise empty bucket just below, so a key that the
// sample saw at least twice is isolated in a bucket of its own.  The map is
// non-decreasing in the key.
__device__ __forceinline__ uint32_t bucket_of(const uint64_t* spl, uint32_t nspl, uint64_t key) {
  uint32_t lo = 0, hi = nspl;  // first index with spl[i] > key
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (spl[mid] <= key) lo = mid + 1; else hi = mid;
  }
  uint32_t b = lo;
  if (b >= 2 && spl[b - 1] == key && spl[b - 2] == key) b--;
  return b;
}

// A multiplier C with C <= M * 2^64 / (span + 1) (span >= M), so that
// x -> mulhi(x, C) maps [0, span] monotonically into [0, M).  Taken from a
// single-precision reciprocal scaled down by 2^-18: the reciprocal (1 ulp)
// and the four roundings around it stay below 3 * 2^-23 relative, so C never
// exceeds the exact value, and its coarser resolution only moves cell
// borders a little.  A wide integer or double division needs several times
// the registers, which the kernels that call this do not have to spare.
__device__ __forceinline__ uint64_t interp_scale(uint32_t M, uint64_t span) {
  const float r = __builtin_amdgcn_rcpf((float)span + 1.0f);
  const float q = (float)M * r * 0x1p64f * (1.0f - 0x1p-18f);
  return q >= 0x1p64f ? ~0ull : (uint64_t)q;
}

// Monotone map of the keys [lo, lo + width] onto cells [0, D):
// cell(x) = hi32(((x - lo) >> sh) * C).  The shift brings the range under
// 2^32, so that a lookup costs one 32-bit multiply-high; C is at most
// D 2^32 / ((width >> sh) + 1) (rounded down with margin, as in
// interp_scale), so every cell is below D, and a range narrower than D gets
// about one key value per cell.
__device__ __forceinline__ uint32_t cell_shift(uint64_t width) {
  return (width >> 32) ? 32u - (uint32_t)__builtin_clzll(width) : 0u;
}
// w1 = (width >> shift) + 1, in [1, 2^32]
__device__ __forceinline__ uint32_t cell_scale(uint32_t D, uint64_t w1) {
  const float q = (float)D * 0x1p32f * __builtin_amdgcn_rcpf((float)w1) * (1.0f - 0x1p-18f);
  return q >= 0x1p32f ? 0xffffffffu : (uint32_t)q;
}
struct CellMap {
  uint64_t lo;
  uint32_t sh, C;
  __device__ __forceinline__ void init(uint64_t lo_, uint64_t width, uint32_t D) {
    lo = lo_;
    sh = cell_shift(width);
    C = cell_scale(D, (width >> sh) + 1);
  }
  // x in [lo, lo + width]
  __device__ __forceinline__ uint32_t operator()(uint64_t x) const {
    return __umulhi((uint32_t)((x - lo) >> sh), C);
  }
};

// Logarithmic cells for skewed key spans: x = key - lo (x <= the span,
// whose top bit is at position top) falls in cell (31 - d) * 64 + m, where d
// is how many bit positions x's top bit lies below the span's and m the six
// bits that follow x's top bit; x = 0 and x below 2^(top - 31) fall in cell 0.
// Monotone in x, cells [0, 2048).  Each binary order of magnitude of x gets
// 64 cells, so splitters crowded at the low end of a heavy-tailed span
// (log-normal keys) still spread over many cells.
__device__ __forceinline__ uint32_t log_cell(uint64_t x, uint32_t top) {
  if (x == 0) return 0;
  const uint32_t lz = (uint32_t)__builtin_clzll(x);
  const uint32_t d = top - (63u - lz);
  if (d >= 32u) return 0;
  const uint32_t m = ((uint32_t)((x << lz) >> 32) >> 25) & 63u;
  return (31u - d) * 64u + m;
}

// Directory over sorted splitters for fast bucket_of: the span [spl[0],
// spl[nspl-1]] is cut into D cells, by a CellMap (linear) or by log_cell,
// whichever puts fewer splitters into a cell that already holds one (the
// choice is made per directory from its splitters).  Cell c's entry packs
// the first splitter whose cell is >= c (bits 0..15), the number of
// splitters in cell c (bits 16..30) and whether they are all one key (bit
// 31: the copies of a frequent key, compared once).  A key in cell c has every splitter
// below the first under it and every splitter after the cell's above it, so
// only its cell's splitters (usually 0 or 1) are compared: one LDS read of
// the entry, then at most one of a splitter in the common case.  A splitter
// of an earlier cell is strictly smaller than the key (cells are monotone),
// so the equal-splitter rule of bucket_of only needs to look at the
// splitters compared here, and dup[m] (spl[m] == spl[m-1]) answers it.
// Same answer as bucket_of.  The per-workgroup constants of the map are
// copied to registers once (SplitView) instead of being re-read from LDS at
// every lookup.
struct SplitView {
  uint64_t lo, last;
  uint32_t sh, C, nspl;
  uint32_t logm, top;   // logarithmic cells (uniform over the workgroup), top bit of the span
};

template <int D, int NSPL>
struct SplitDir {
  static_assert(D == 2048, "log_cell fills 2048 cells");
  uint32_t ent[D];
  uint8_t dup[NSPL];
  CellMap map;
  uint64_t last;
  uint32_t top, logm;
  uint32_t coll[2];

  // All threads of the block call; spl (LDS) holds nspl sorted splitters,
  // 1 <= nspl <= NSPL < 2^16.
  template <int NT>
  __device__ void build(const uint64_t* spl, uint32_t nspl) {
    if (threadIdx.x == 0) {
      const uint64_t w = spl[nspl - 1] - spl[0];
      map.init(spl[0], w, D);
      last = spl[nspl - 1];
      top = w ? 63u - (uint32_t)__builtin_clzll(w) : 0u;
      coll[0] = coll[1] = 0;
    }
    __syncthreads();
    const CellMap mp = map;
    const uint32_t tp = top;
    // splitters that share a cell with a smaller predecessor, under either map
    uint32_t c0 = 0, c1 = 0;
    for (uint32_t m = threadIdx.x + 1; m < nspl; m += NT) {
      const uint64_t x = spl[m], y = spl[m - 1];
      if (x != y) {
        c0 += mp(x) == mp(y);
        c1 += log_cell(x - mp.lo, tp) == log_cell(y - mp.lo, tp);
      }
    }
    if (c0) atomicAdd(&coll[0], c0);
    if (c1) atomicAdd(&coll[1], c1);
    __syncthreads();
    // a logarithmic cell costs a few more instructions: taken when it halves the collisions
    const bool lg = 2 * coll[1] < coll[0];
    auto cell_of = [&](uint64_t k) -> uint32_t { return lg ? log_cell(k - mp.lo, tp) : mp(k); };
    auto first_at = [&](uint32_t cell) -> uint32_t {   // first m with cell(spl[m]) >= cell
      uint32_t a = 0, b = nspl;
      while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (cell_of(spl[m]) < cell) a = m + 1; else b = m;
      }
      return a;
    };
    for (uint32_t cell = threadIdx.x; cell < (uint32_t)D; cell += NT) {
      const uint32_t f0 = first_at(cell), f1 = first_at(cell + 1);
      const bool one = f1 - f0 >= 2 && spl[f0] == spl[f1 - 1];
      ent[cell] = f0 | ((f1 - f0) << 16) | (one ? 0x80000000u : 0u);
    }
    for (uint32_t m = threadIdx.x; m < nspl; m += NT) dup[m] = m > 0 && spl[m] == spl[m - 1];
    if (threadIdx.x == 0) logm = lg ? 1u : 0u;
    __syncthreads();
  }

  __device__ __forceinline__ SplitView view(uint32_t nspl) const {
    SplitView v;
    v.nspl = nspl;
    if (nspl) { v.lo = map.lo; v.last = last; v.sh = map.sh; v.C = map.C; v.top = top; v.logm = logm; }
    else { v.lo = ~0ull; v.last = ~0ull; v.sh = 0; v.C = 0; v.top = 0; v.logm = 0; }
    v.logm = __builtin_amdgcn_readfirstlane(v.logm);
    v.top = __builtin_amdgcn_readfirstlane(v.top);
    return v;
  }

  __device__ __forceinline__ uint32_t bucket(const SplitView& v, const uint64_t* spl, uint64_t key) const {
    if (v.nspl == 0 || key < v.lo) return 0;
    uint32_t b;
    bool eq;
    if (key >= v.last) {
      b = v.nspl;
      eq = key == v.last;
    } else {
      // below D
      const uint32_t cell = v.logm ? log_cell(key - v.lo, v.top) : __umulhi((uint32_t)((key - v.lo) >> v.sh), v.C);
      const uint32_t e = ent[cell];
      uint32_t a = e & 0xFFFFu;
      const uint32_t n = (e >> 16) & 0x7FFFu;
      if (n == 0) {
        b = a;
        eq = false;
      } else if (n == 1 || (e >> 31)) {   // one splitter, or n copies of one key
        const uint64_t s0 = spl[a];
        b = a + (s0 <= key ? n : 0u);
        eq = s0 == key;
      } else {
        uint32_t z = a + n;
        while (a < z) {
          const uint32_t m = (a + z) >> 1;
          if (spl[m] <= key) a = m + 1; else z = m;
        }
        b = a;
        eq = b > 0 && spl[b - 1] == key;
      }
    }
    if (eq && b >= 2 && dup[b - 1]) b--;
    return b;
  }
};
