// LDS-resident LSD radix sort of one tile held in registers by a workgroup.
//
// Layout: NT threads, IPT items per thread, capacity CAP = NT*IPT.  During a
// pass the items of thread t are the consecutive positions t*IPT .. t*IPT+IPT-1
// of the current order ("blocked").  Each pass ranks one RB-bit digit:
// every thread counts its own items per digit into private 16-bit counters
// laid out digit-major ([digit][thread]); one exclusive scan over those
// counters in that order gives every item its destination, which is stable
// with respect to the current order (earlier digit first, then earlier
// thread, then earlier item of the same thread).  Items then trade places
// through one LDS buffer.  The counters alias the exchange buffer, so one
// buffer of CAP u64 words (+1/16 padding against bank conflicts) is all the
// LDS a sort needs.  Passes whose digit is the same for every key of the
// tile are skipped.
#pragma once
#include "common.h"

template <int NT, int IPT, int RB>
struct BlockSort {
  static constexpr int CAP = NT * IPT;
  static constexpr int NDIG = 1 << RB;
  static constexpr int XCH_WORDS = CAP + CAP / 16;
  static constexpr int CNT_WORDS = NDIG * NT / 4;  // u16 counters, in u64 words
  static constexpr int BUF_WORDS = XCH_WORDS > CNT_WORDS ? XCH_WORDS : CNT_WORDS;
  static constexpr int WSUM_WORDS = NT / 64 + 2;
  static_assert(RB >= 1 && RB <= 8, "radix bits");
  static_assert(NT % 64 == 0, "whole waves");

  __device__ static __forceinline__ int pad(int i) { return i + (i >> 4); }

  // Stable destination of every item for its digit d[k] in [0, NDIG).
  __device__ static void rank(const uint32_t (&d)[IPT], uint32_t (&r)[IPT], uint64_t* buf, uint32_t* wsum) {
    uint16_t* cnt = reinterpret_cast<uint16_t*>(buf);
    uint32_t* cnt32 = reinterpret_cast<uint32_t*>(buf);
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NDIG / 2; i++) cnt32[i * NT + tid] = 0u;
    __syncthreads();
    uint32_t local[IPT];
#pragma unroll
    for (int k = 0; k < IPT; k++) {
      uint16_t* c = cnt + d[k] * NT + tid;
      uint32_t v = *c;
      local[k] = v;
      *c = (uint16_t)(v + 1);
    }
    __syncthreads();
    // raking: thread tid owns flattened counters [tid*NDIG, tid*NDIG + NDIG)
    uint32_t* my = cnt32 + tid * (NDIG / 2);
    uint32_t pre[NDIG];
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < NDIG / 2; i++) {
      uint32_t v = my[i];
      pre[2 * i] = run; run += v & 0xFFFFu;
      pre[2 * i + 1] = run; run += v >> 16;
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<NT>(run, wsum, &tot);
#pragma unroll
    for (int i = 0; i < NDIG / 2; i++) my[i] = (pre[2 * i] + ex) | ((pre[2 * i + 1] + ex) << 16);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; k++) r[k] = (uint32_t)cnt[d[k] * NT + tid] + local[k];
    __syncthreads();
  }

  // Move one u64 per item to its rank; read back blocked (or striped).
  __device__ static void exchange(uint64_t (&v)[IPT], const uint32_t (&r)[IPT], uint64_t* buf, bool striped_out) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < IPT; k++) buf[pad((int)r[k])] = v[k];
    __syncthreads();
    if (striped_out) {
#pragma unroll
      for (int k = 0; k < IPT; k++) v[k] = buf[pad(k * NT + tid)];
    } else {
#pragma unroll
      for (int k = 0; k < IPT; k++) v[k] = buf[pad(tid * IPT + k)];
    }
    __syncthreads();
  }

  __device__ static uint64_t block_or(uint64_t v, uint64_t* red) {
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) s |= red[i];
    __syncthreads();
    return s;
  }

  // Sort the first n items by key, carrying val.  Input is striped (item k of
  // thread t is element k*NT + t of the tile); items beyond n must hold key
  // ~0.  The tile is first transposed to blocked order so that the element
  // order is the input order, which makes the whole sort stable and keeps
  // the padding items last.  On return the items are striped in sorted order:
  // item k of thread t has rank k*NT + t.  Returns the number of digit passes.
  // `red` is LDS scratch of NT/64 + 1 u64, `wsum` of WSUM_WORDS u32.
  template <bool HAS_VAL>
  __device__ static int sort(uint64_t (&key)[IPT], uint64_t (&val)[IPT], int n, uint64_t* buf, uint32_t* wsum,
                             uint64_t* red) {
    const int tid = threadIdx.x;
    if (n <= 1) return 0;
    // bits that differ between some key and the tile's first key
    if (tid == 0) red[NT / 64] = key[0];
    __syncthreads();
    const uint64_t k0 = red[NT / 64];
    uint64_t vary = 0;
#pragma unroll
    for (int k = 0; k < IPT; k++)
      if (k * NT + tid < n) vary |= key[k] ^ k0;
    vary = block_or(vary, red);
    if (vary == 0) return 0;  // all keys equal: input order is sorted order
    transpose_to_blocked(key, buf);
    if (HAS_VAL) transpose_to_blocked(val, buf);
    int last_sh = 0;
    for (int sh = 0; sh < 64; sh += RB)
      if ((vary >> sh) & (uint64_t)(NDIG - 1)) last_sh = sh;
    int passes = 0;
    for (int sh = 0; sh < 64; sh += RB) {
      if (((vary >> sh) & (uint64_t)(NDIG - 1)) == 0) continue;
      uint32_t d[IPT], r[IPT];
#pragma unroll
      for (int k = 0; k < IPT; k++) d[k] = (uint32_t)(key[k] >> sh) & (uint32_t)(NDIG - 1);
      rank(d, r, buf, wsum);
      const bool striped = (sh == last_sh);
      exchange(key, r, buf, striped);
      if (HAS_VAL) exchange(val, r, buf, striped);
      passes++;
    }
    return passes;
  }

  __device__ static void transpose_to_blocked(uint64_t (&v)[IPT], uint64_t* buf) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < IPT; k++) buf[pad(k * NT + tid)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; k++) v[k] = buf[pad(tid * IPT + k)];
    __syncthreads();
  }
};
