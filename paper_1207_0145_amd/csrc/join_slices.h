// Slices of the S runs that one join unit reads (Section 3.2.2: the start of
// a private partition in every public run is searched, and the partition is
// merged with the run from there on; the next partition's start ends it).
//
// For run j of n_j tuples, the unit's start offset oa and the next unit's
// start offset ob bound the slice [oa, ob).  The start search returns lower
// bounds, so for sorted runs 0 <= oa <= ob <= n_j.  Both offsets are clamped
// to the run here and a reversed pair gives an empty slice, so whatever the
// offsets hold (runs left unsorted, offsets of another join), every position
// the join reads stays inside run j.
//
// The slices of the Q runs are concatenated: cum[j] is the exclusive prefix
// of the slice lengths, and concatenated index x with cum[j] <= x < cum[j+1]
// is S position sbase[j] + x = run_start[j] + begin_j + (x - cum[j]).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

__host__ __device__ __forceinline__ uint32_t slice_begin(uint32_t oa, uint32_t n) { return oa < n ? oa : n; }

__host__ __device__ __forceinline__ uint32_t slice_len(uint32_t oa, uint32_t ob, uint32_t n) {
  const uint32_t a = oa < n ? oa : n, b = ob < n ? ob : n;
  return b > a ? b - a : 0u;
}

// sbase[j] for a slice that starts at concatenated index c (wraps mod 2^32;
// sbase[j] + x is formed only for x >= c).
__host__ __device__ __forceinline__ uint32_t slice_base(uint32_t run_start, uint32_t oa, uint32_t n, uint32_t c) {
  return run_start + slice_begin(oa, n) - c;
}
