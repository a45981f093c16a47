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
// in it, or else on which side.  On that side the search gallops: it
// probes one line further, then two, four, ... until it passes the bound,
// and bisects what is left.  An interpolation that is off by k lines costs
// about 2 log2(k) lines, never much more than a plain bisection (keys that
// interpolate badly, such as tight clusters).  Lines are counted from the
// run's start (a line start for the runs of one join, whose starts are
// multiples of 8 tuples).  Any klo, khi give the same result: they only
// choose the first line.  key_at(i) is the run's i-th key; *probes counts
// the lines read.
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
  const uint32_t line = pos & ~7u;
  const uint32_t s = line > a ? line : a;
  const uint32_t e = line + 8 < b ? line + 8 : b;
  uint32_t last = line;   // the line read last
  (*probes)++;
  if (key_at(s) >= key) {   // the bound is at s or before: gallop down
    b = s;
    for (uint32_t step = 8; b > a;) {
      const uint32_t t = b - a > step ? b - step : a;
      const uint32_t lt = t & ~7u;
      if (lt != last) { (*probes)++; last = lt; }
      if (key_at(t) < key) { a = t + 1; break; }
      b = t;
      step <<= 1;
    }
  } else if (key_at(e - 1) < key) {   // after this line: gallop up
    a = e;
    for (uint32_t step = 8; a < b;) {
      const uint32_t t = b - a > step ? a + step - 1 : b - 1;
      const uint32_t lt = t & ~7u;
      if (lt != last) { (*probes)++; last = lt; }
      if (key_at(t) >= key) { b = t; break; }
      a = t + 1;
      step <<= 1;
    }
  } else {                  // in (s, e - 1]
    a = s + 1;
    b = e - 1;
  }
  while (a < b) {
    const uint32_t mid = a + ((b - a) >> 1);
    if ((mid & ~7u) != last) { (*probes)++; last = mid & ~7u; }
    if (key_at(mid) < key) a = mid + 1; else b = mid;
  }
  return a;
}
