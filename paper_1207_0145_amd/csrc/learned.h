// Learned CDF of a relation's keys: a piecewise-linear CDF over K knots
// (sample quantiles -- the paper's global CDF with steps taken as equally
// high and interpolated linearly between them, Section 4.1) plus a small
// residual network r(q) = sum_h w2[h] tanh(w1[h] q + b1[h]) + b2 applied to
// the piecewise-linear estimate q.  Everything is fp32 except the knot keys
// (u64, so the segment of a key is found exactly).  The model only chooses
// splitters and search windows; every decision it feeds is re-checked with
// integer comparisons, so results never depend on it.
#pragma once
#include "block_sort.h"

constexpr int CDF_K = 256;          // knots
constexpr int CDF_H = 8;            // hidden units
constexpr int CDF_M = 1 << 16;      // sample keys
constexpr int CDF_TRAIN = 2048;     // training points (every 32nd sample)
constexpr int CDF_STEPS = 24;       // Adam steps
constexpr int CDF_CHUNK = 4096;     // sample keys sorted per workgroup

struct CdfModel {
  uint64_t kkey[CDF_K];             // knot keys, non-decreasing
  float w1[CDF_H], b1[CDF_H], w2[CDF_H], b2;
  float eps;                        // max |prediction - empirical CDF| over the sample
  uint32_t valid;                   // 0 if the sample was empty
  uint32_t pad;
};

// Piecewise-linear estimate: knot i has quantile i/(K-1).
__device__ __forceinline__ float cdf_pwl(const CdfModel& m, uint64_t key) {
  if (key <= m.kkey[0]) return 0.f;
  if (key >= m.kkey[CDF_K - 1]) return 1.f;
  uint32_t lo = 0, hi = CDF_K - 1;   // kkey[lo] <= key < kkey[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (m.kkey[mid] <= key) lo = mid; else hi = mid;
  }
  const uint64_t a = m.kkey[lo], b = m.kkey[hi];
  const float t = (float)((double)(key - a) / (double)(b - a));
  return ((float)lo + t) * (1.f / (float)(CDF_K - 1));
}

__device__ __forceinline__ float cdf_residual(const CdfModel& m, float q) {
  float r = m.b2;
#pragma unroll
  for (int h = 0; h < CDF_H; h++) r += m.w2[h] * tanhf(m.w1[h] * q + m.b1[h]);
  return r;
}

__device__ __forceinline__ float cdf_eval(const CdfModel& m, uint64_t key) {
  const float q = cdf_pwl(m, key);
  const float p = q + cdf_residual(m, q);
  return p < 0.f ? 0.f : (p > 1.f ? 1.f : p);
}

// A key whose predicted CDF is about `target`: q solves q + r(q) = target by
// fixed-point steps (the residual is small and smooth), then the
// piecewise-linear part is inverted exactly on its segment.  Callers only
// need some non-decreasing sequence of keys, and keep the results sorted.
__device__ __forceinline__ uint64_t cdf_inverse(const CdfModel& m, float target) {
  float q = target;
#pragma unroll
  for (int it = 0; it < 6; it++) {
    q = target - cdf_residual(m, q);
    q = q < 0.f ? 0.f : (q > 1.f ? 1.f : q);
  }
  const float pos = q * (float)(CDF_K - 1);
  uint32_t i = (uint32_t)pos;
  if (i >= (uint32_t)CDF_K - 1) return m.kkey[CDF_K - 1];
  const double t = (double)(pos - (float)i);
  const uint64_t a = m.kkey[i], b = m.kkey[i + 1];
  return a + (uint64_t)(t * (double)(b - a));
}

// Draw CDF_M keys of src[0, n) at SplitMix64 positions (stream seed).
__global__ void k_cdf_sample(const tup_t* __restrict__ src, uint32_t n, uint64_t seed, uint64_t* sample) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint32_t)CDF_M) return;
  sample[t] = n ? src[draw_below(splitmix_at(seed, t), n)].key : 0ull;
}

// Sort each CDF_CHUNK-key chunk of the sample in LDS.
__global__ void __launch_bounds__(1024) k_cdf_sort_chunks(uint64_t* sample) {
  using Sorter = BlockSort<1024, CDF_CHUNK / 1024, 4>;
  __shared__ uint64_t buf[Sorter::BUF_WORDS];
  __shared__ uint32_t wsum[Sorter::WSUM_WORDS];
  __shared__ uint64_t red[1024 / 64 + 1];
  uint64_t* c = sample + (uint64_t)blockIdx.x * CDF_CHUNK;
  uint64_t key[CDF_CHUNK / 1024], dummy[CDF_CHUNK / 1024];
#pragma unroll
  for (int k = 0; k < CDF_CHUNK / 1024; k++) { key[k] = c[k * 1024 + threadIdx.x]; dummy[k] = 0; }
  Sorter::sort<false>(key, dummy, CDF_CHUNK, buf, wsum, red);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < CDF_CHUNK / 1024; k++) c[k * 1024 + threadIdx.x] = key[k];
}

// Merge the sorted chunks by rank: a key's rank is its position in its chunk
// plus, in every other chunk, the number of keys below it (keys equal to it
// count when their chunk comes first), which orders equal keys by chunk.
__global__ void k_cdf_merge(const uint64_t* chunks, uint64_t* sorted) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint32_t)CDF_M) return;
  const uint32_t c = t / CDF_CHUNK, i = t % CDF_CHUNK;
  const uint64_t key = chunks[t];
  uint32_t rank = i;
  for (uint32_t o = 0; o < (uint32_t)(CDF_M / CDF_CHUNK); o++) {
    if (o == c) continue;
    const uint64_t* oc = chunks + (uint64_t)o * CDF_CHUNK;
    uint32_t lo = 0, hi = CDF_CHUNK;
    if (o < c) { while (lo < hi) { const uint32_t m = (lo + hi) >> 1; if (oc[m] <= key) lo = m + 1; else hi = m; } }
    else { while (lo < hi) { const uint32_t m = (lo + hi) >> 1; if (oc[m] < key) lo = m + 1; else hi = m; } }
    rank += lo;
  }
  sorted[rank] = key;
}

// Fit the model to the sorted sample (one workgroup of 1024 threads).
// Knots: kkey[i] = sorted[i (M-1)/(K-1)].  Residual network: full-batch Adam
// on the squared error between q + r(q) and the empirical CDF (rank+0.5)/M at
// CDF_TRAIN sample points.  eps: the largest error over all M sample points.
// Sum of a float over the 64 lanes of a wave (DPP row shifts and row
// broadcasts as in wave_incl_scan; the total ends in lane 63).
__device__ __forceinline__ float wave_sum_f(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__global__ void __launch_bounds__(1024) k_cdf_train(const uint64_t* sorted, uint32_t n_src, CdfModel* out) {
  constexpr int NP = 3 * CDF_H + 1;              // parameters
  __shared__ CdfModel m;
  __shared__ float gpart[1024 / 64][NP];
  __shared__ float grad[NP];
  __shared__ float mom1[NP], mom2[NP];
  __shared__ float emax[1024 / 64];
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (uint32_t i = tid; i < (uint32_t)CDF_K; i += 1024)
    m.kkey[i] = sorted[(uint64_t)i * (CDF_M - 1) / (CDF_K - 1)];
  if (tid < (uint32_t)CDF_H) {
    // deterministic start: hidden units spread over [0, 1], output weights 0 (pure PWL)
    m.w1[tid] = 6.f;
    m.b1[tid] = -6.f * ((float)tid + 0.5f) / (float)CDF_H;
    m.w2[tid] = 0.f;
  }
  if (tid == 0) { m.b2 = 0.f; m.valid = n_src ? 1u : 0u; m.pad = 0; }
  if (tid < (uint32_t)NP) { mom1[tid] = 0.f; mom2[tid] = 0.f; }
  __syncthreads();
  // two training points per thread
  float xq[2], yv[2];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const uint32_t j = (tid * 2 + u) * (CDF_M / CDF_TRAIN);
    xq[u] = cdf_pwl(m, sorted[j]);
    yv[u] = ((float)j + 0.5f) / (float)CDF_M;
  }
  const float lr = 0.01f, be1 = 0.9f, be2 = 0.999f;
  float b1t = 1.f, b2t = 1.f;
  for (int step = 0; step < CDF_STEPS; step++) {
    float g[NP];
#pragma unroll
    for (int q = 0; q < NP; q++) g[q] = 0.f;
#pragma unroll
    for (int u = 0; u < 2; u++) {
      float th[CDF_H];
      float pred = xq[u] + m.b2;
#pragma unroll
      for (int h = 0; h < CDF_H; h++) { th[h] = tanhf(m.w1[h] * xq[u] + m.b1[h]); pred += m.w2[h] * th[h]; }
      const float e = 2.f * (pred - yv[u]) / (float)CDF_TRAIN;
#pragma unroll
      for (int h = 0; h < CDF_H; h++) {
        const float dz = e * m.w2[h] * (1.f - th[h] * th[h]);
        g[h] += dz * xq[u];               // w1
        g[CDF_H + h] += dz;               // b1
        g[2 * CDF_H + h] += e * th[h];    // w2
      }
      g[3 * CDF_H] += e;                  // b2
    }
#pragma unroll
    for (int q = 0; q < NP; q++) {
      const float s = wave_sum_f(g[q]);
      if (lane == 0) gpart[w][q] = s;
    }
    __syncthreads();
    if (tid < (uint32_t)NP) {
      float s = 0.f;
      for (int i = 0; i < 1024 / 64; i++) s += gpart[i][tid];
      grad[tid] = s;
    }
    __syncthreads();
    b1t *= be1; b2t *= be2;
    if (tid < (uint32_t)NP) {
      const float gq = grad[tid];
      mom1[tid] = be1 * mom1[tid] + (1.f - be1) * gq;
      mom2[tid] = be2 * mom2[tid] + (1.f - be2) * gq * gq;
      const float step_v = lr * (mom1[tid] / (1.f - b1t)) / (sqrtf(mom2[tid] / (1.f - b2t)) + 1e-7f);
      float* p = tid < (uint32_t)CDF_H ? &m.w1[tid] : tid < 2u * CDF_H ? &m.b1[tid - CDF_H]
               : tid < 3u * CDF_H ? &m.w2[tid - 2 * CDF_H] : &m.b2;
      *p -= step_v;
    }
    __syncthreads();
  }
  // error bound over every 4th sample key
  float e = 0.f;
  for (uint32_t j = tid * 4; j < (uint32_t)CDF_M; j += 4096) {
    const float y = ((float)j + 0.5f) / (float)CDF_M;
    const float d = fabsf(cdf_eval(m, sorted[j]) - y);
    e = d > e ? d : e;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) { const float o = __shfl_xor(e, d, 64); e = o > e ? o : e; }
  if (lane == 0) emax[w] = e;
  __syncthreads();
  if (tid == 0) {
    float x = 0.f;
    for (int i = 0; i < 1024 / 64; i++) x = emax[i] > x ? emax[i] : x;
    m.eps = x;
  }
  __syncthreads();
  // publish
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&m);
  uint32_t* dst = reinterpret_cast<uint32_t*>(out);
  for (uint32_t i = tid; i < sizeof(CdfModel) / 4; i += 1024) dst[i] = src[i];
}

// Learned splitters: spl[b-1] = inverse CDF at b/NB (b = 1..NB-1), kept
// non-decreasing.  One thread per splitter, then a serial fix-up pass.
__global__ void k_learned_splitters(const CdfModel* model, uint32_t NB, uint64_t* spl) {
  __shared__ CdfModel m;
  const uint32_t tid = threadIdx.x;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(model);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&m);
  for (uint32_t i = tid; i < sizeof(CdfModel) / 4; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  for (uint32_t b = 1 + tid; b < NB; b += blockDim.x) spl[b - 1] = cdf_inverse(m, (float)b / (float)NB);
  __syncthreads();
  if (tid == 0)
    for (uint32_t b = 1; b + 1 < NB; b++)
      if (spl[b] < spl[b - 1]) spl[b] = spl[b - 1];
}
