// Lower bound of a key inside one window of a sorted run, line by line
// (the last step of the start search, Section 3.2.2: the start of a private
// partition in a public run).  Host and device share this code; the host
// build serves the library's CPU test entry point.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Lower bound of key in the run's [a, b) when every key before a is smaller
// and the key at b (if any) is not: the window between two index keys klo <
// key <= khi.  A bisection of a 256-tuple window touches about five
// different 128-byte lines (eight 16-byte tuples each) before its steps fall
// inside one, and the start search is bound by fetching them.  Here the
// first probe goes to the line that linear interpolation between klo and
// khi points at; the line's first and last key say whether the bound lies
// in it, or else in which direction to step to the next line; the bound is
// then bisected inside the line, where every probe hits the fetched line.
// Lines are counted from the run's start (a line start for the runs of one
// join, whose starts are multiples of 8 tuples).  Any klo, khi give the same
// result: they only choose the first line.  key_at(i) is the run's i-th key.
template <typename KeyAt>
__host__ __device__ __forceinline__ uint32_t lb_window_at(KeyAt key_at, uint32_t a, uint32_t b, uint64_t klo,
                                                          uint64_t khi, uint64_t key, uint32_t* probes) {
  if (a >= b) return a;
  uint32_t pos = a;
  if (khi > klo && key > klo) {
    const float f = (float)(key - klo) / (float)(khi - klo);
    const float d = f * (float)(b - a);
    pos = d < (float)(b - a - 1) ? a + (uint32_t)d : b - 1;
  }
  uint32_t line = pos & ~7u;
  for (;;) {
    const uint32_t s = line > a ? line : a;
    const uint32_t e = line + 8 < b ? line + 8 : b;
    (*probes)++;
    if (key_at(s) >= key) {             // the bound is at s or before
      if (s == a) return a;
      b = s;
      line = (s - 1) & ~7u;
    } else if (key_at(e - 1) < key) {   // after this line
      if (e == b) return b;
      a = e;
      line = e;
    } else {                            // in (s, e - 1]
      uint32_t lo = s + 1, hi = e - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (key_at(mid) < key) lo = mid + 1; else hi = mid;
      }
      return lo;
    }
  }
}
