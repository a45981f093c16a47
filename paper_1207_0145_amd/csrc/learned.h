// Learned CDF of a relation's keys: a piecewise-linear CDF over K knots
// (sample quantiles -- the paper's global CDF with steps taken as equally
// high and interpolated linearly between them, Section 4.1) plus a small
// residual network r(q) = sum_h w2[h] tanh(w1[h] q + b1[h]) + b2 applied to
// the piecewise-linear estimate q.  Everything is fp32 except the knot keys
// (u64, so the segment of a key is found exactly).  The model only chooses
// splitters and search windows; every decision it feeds is re-checked with
// integer comparisons, so results never depend on it.
//
// Up to two models (R and S) are built together: every kernel below takes
// the model index from blockIdx.y.
#pragma once
#include "block_sort.h"

constexpr int CDF_K = 4096;         // knots (16 sample keys per knot)
constexpr int CDF_H = 8;            // hidden units
constexpr int CDF_M = 1 << 16;      // sample keys
constexpr int CDF_TRAIN = 2048;     // training points (every 32nd sample)
constexpr int CDF_STEPS = 16;       // Adam steps
constexpr int CDF_CHUNK = 4096;     // sample keys sorted per workgroup
constexpr int CDF_SEG = 64;         // quantile segments with their own error bound

struct CdfModel {
  uint64_t kkey[CDF_K];             // knot keys, non-decreasing
  float w1[CDF_H], b1[CDF_H], w2[CDF_H], b2;
  float eps;                        // max |prediction - empirical CDF| over the sample
  uint32_t valid;                   // 0 if the sample was empty
  uint32_t pad;
  float eps_seg[CDF_SEG];           // the same over sample keys with empirical CDF in [i, i+1)/CDF_SEG
};

// Error bound of a prediction q: the largest segment bound around q (the
// segment of q and its neighbours, since q itself may be off by a little).
__device__ __forceinline__ float cdf_local_eps(const CdfModel& m, float q) {
  int i = (int)(q * (float)CDF_SEG);
  i = i < 0 ? 0 : (i >= CDF_SEG ? CDF_SEG - 1 : i);
  float e = m.eps_seg[i];
  if (i > 0) e = fmaxf(e, m.eps_seg[i - 1]);
  if (i + 1 < CDF_SEG) e = fmaxf(e, m.eps_seg[i + 1]);
  return e;
}

// What the model-building kernels work on (by value; index = blockIdx.y).
struct CdfJob {
  const tup_t* src[2];
  uint32_t n[2];
  uint64_t seed[2];
  CdfModel* model[2];
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
  const float t = (float)(key - a) / (float)(b - a);   // in [0, 1); single precision is ample
  return ((float)lo + (t < 1.f ? t : 1.f)) * (1.f / (float)(CDF_K - 1));
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

// Draw CDF_M keys of the model's input at SplitMix64 positions (its seed).
__global__ void k_cdf_sample(CdfJob job, uint64_t* sample) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (t >= (uint32_t)CDF_M) return;
  const uint32_t n = job.n[y];
  sample[(uint64_t)y * CDF_M + t] = n ? job.src[y][draw_below(splitmix_at(job.seed[y], t), n)].key : 0ull;
}

// Sort each CDF_CHUNK-key chunk of the sample in LDS.
__global__ void __launch_bounds__(1024) k_cdf_sort_chunks(uint64_t* sample) {
  using Sorter = BlockSort<1024, CDF_CHUNK / 1024, 4>;
  __shared__ uint64_t buf[Sorter::BUF_WORDS];
  __shared__ uint32_t wsum[Sorter::WSUM_WORDS];
  __shared__ uint64_t red[1024 / 64 + 1];
  uint64_t* c = sample + (uint64_t)blockIdx.y * CDF_M + (uint64_t)blockIdx.x * CDF_CHUNK;
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
__global__ void k_cdf_merge(const uint64_t* chunks_all, uint64_t* sorted_all) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint32_t)CDF_M) return;
  const uint64_t* chunks = chunks_all + (uint64_t)blockIdx.y * CDF_M;
  uint64_t* sorted = sorted_all + (uint64_t)blockIdx.y * CDF_M;
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

// Largest |cdf_eval - empirical CDF| over every 4th sample key (all threads
// of the 1024-thread block call; the result is in every thread).  With
// seg != NULL also the largest per quantile segment (seg: CDF_SEG floats of
// LDS, zeroed by the caller).
// (NET false: the piecewise-linear part alone, the model before training
// and after a network that did not help.)
template <bool NET>
__device__ float cdf_sample_error(const CdfModel& m, const uint64_t* sorted, float* emax, float* seg) {
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  float e = 0.f;
  for (uint32_t j = tid * 4; j < (uint32_t)CDF_M; j += 4096) {
    const float y = ((float)j + 0.5f) / (float)CDF_M;
    const float d = fabsf((NET ? cdf_eval(m, sorted[j]) : cdf_pwl(m, sorted[j])) - y);
    e = d > e ? d : e;
    // non-negative floats order like their bit patterns
    if (seg) atomicMax(reinterpret_cast<unsigned int*>(&seg[j / (CDF_M / CDF_SEG)]), __float_as_uint(d));
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) { const float o = __shfl_xor(e, d, 64); e = o > e ? o : e; }
  __syncthreads();
  if (lane == 0) emax[w] = e;
  __syncthreads();
  float x = 0.f;
  for (int i = 0; i < 1024 / 64; i++) x = emax[i] > x ? emax[i] : x;
  return x;
}

// Fit one model per blockIdx.y to its sorted sample (1024 threads).
// Knots: kkey[i] = sorted[i (M-1)/(K-1)].  Residual network: full-batch Adam
// on the squared error between q + r(q) and the empirical CDF (rank+0.5)/M at
// CDF_TRAIN sample points; the network is kept only if it lowers the largest
// error over the sample (else the model is the piecewise-linear CDF alone).
// eps: that largest error.
__global__ void __launch_bounds__(1024) k_cdf_train(const uint64_t* sorted_all, CdfJob job) {
  constexpr int NP = 3 * CDF_H + 1;              // parameters
  __shared__ CdfModel m;
  __shared__ float gpart[1024 / 64][NP];
  __shared__ float grad[NP];
  __shared__ float mom1[NP], mom2[NP];
  __shared__ float emax[1024 / 64];
  __shared__ float eseg[CDF_SEG];
  const uint64_t* sorted = sorted_all + (uint64_t)blockIdx.y * CDF_M;
  CdfModel* out = job.model[blockIdx.y];
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (uint32_t i = tid; i < (uint32_t)CDF_K; i += 1024)
    m.kkey[i] = sorted[(uint64_t)i * (CDF_M - 1) / (CDF_K - 1)];
  if (tid < (uint32_t)CDF_H) {
    // deterministic start: hidden units spread over [0, 1], output weights 0 (pure PWL)
    m.w1[tid] = 6.f;
    m.b1[tid] = -6.f * ((float)tid + 0.5f) / (float)CDF_H;
    m.w2[tid] = 0.f;
  }
  if (tid == 0) { m.b2 = 0.f; m.valid = job.n[blockIdx.y] ? 1u : 0u; m.pad = 0; }
  if (tid < (uint32_t)NP) { mom1[tid] = 0.f; mom2[tid] = 0.f; }
  __syncthreads();
  const float e_pwl = cdf_sample_error<false>(m, sorted, emax, nullptr);
  // two training points per thread
  float xq[2], yv[2];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const uint32_t j = (tid * 2 + u) * (CDF_M / CDF_TRAIN);
    xq[u] = cdf_pwl(m, sorted[j]);
    yv[u] = ((float)j + 0.5f) / (float)CDF_M;
  }
  const float lr = 1e-3f, be1 = 0.9f, be2 = 0.999f;
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
  // error bounds of the trained model, overall and per quantile segment
  if (tid < (uint32_t)CDF_SEG) eseg[tid] = 0.f;
  __syncthreads();
  float e = cdf_sample_error<true>(m, sorted, emax, eseg);
  if (!(e < e_pwl)) {   // the network did not help (or diverged): drop it
    __syncthreads();
    if (tid < (uint32_t)CDF_H) m.w2[tid] = 0.f;
    if (tid == 0) m.b2 = 0.f;
    if (tid < (uint32_t)CDF_SEG) eseg[tid] = 0.f;
    __syncthreads();
    e = cdf_sample_error<false>(m, sorted, emax, eseg);
  }
  __syncthreads();
  if (tid < (uint32_t)CDF_SEG) m.eps_seg[tid] = eseg[tid];
  if (tid == 0) m.eps = e;
  __syncthreads();
  // publish
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&m);
  uint32_t* dst = reinterpret_cast<uint32_t*>(out);
  for (uint32_t i = tid; i < sizeof(CdfModel) / 4; i += 1024) dst[i] = src[i];
}

// Learned splitters of every segment s (one workgroup each), written at
// spl + s (NBmax - 1): the inverse CDF at equally spaced quantiles of the
// segment's key range.  Without outer bounds the range is the whole
// relation and every segment gets the same NBmax - 1 splitters; with outer
// bounds (the previous level's splitters) segment s covers [outer[s-1],
// outer[s]) and gets seg_nb[s] - 1 splitters between F(lo) and F(hi),
// clamped into the range.  Made non-decreasing by a running maximum.
constexpr int LSPL_NT = 256;
__global__ void __launch_bounds__(LSPL_NT) k_learned_splitters(const CdfModel* model, uint32_t NBmax,
                                                               const uint32_t* seg_nb, const uint64_t* outer,
                                                               uint32_t outer_nspl, uint64_t* spl) {
  __shared__ uint64_t sp[MAX_NB];
  __shared__ uint64_t wmax[LSPL_NT / 64];
  const CdfModel& m = *model;
  const uint32_t s = blockIdx.x, tid = threadIdx.x;
  const uint32_t nb = outer ? seg_nb[s] : NBmax;
  if (nb < 2) return;
  uint64_t* out = spl + (uint64_t)s * (NBmax - 1);
  uint64_t lo = 0, hi = ~0ull;
  float qlo = 0.f, qhi = 1.f;
  if (outer) {
    if (s > 0) { lo = outer[s - 1]; qlo = cdf_eval(m, lo); }
    if (s < outer_nspl) { hi = outer[s]; qhi = cdf_eval(m, hi); }
  }
  // thread t owns the consecutive splitters [t*PER, t*PER + PER)
  constexpr int PER = MAX_NB / LSPL_NT;
  const uint32_t ns = nb - 1;
  uint64_t run = 0;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t i = tid * PER + k;
    if (i < ns) {
      uint64_t key = cdf_inverse(m, qlo + (qhi - qlo) * (float)(i + 1) / (float)nb);
      key = key < lo ? lo : (key > hi ? hi : key);
      run = key > run ? key : run;
      sp[i] = run;
    }
  }
  // exclusive running maximum over the threads before this one
  uint64_t incl = run;
  const uint32_t lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(incl, d, 64);
    if (lane >= (uint32_t)d) incl = o > incl ? o : incl;
  }
  if (lane == 63) wmax[w] = incl;
  __syncthreads();
  uint64_t before = __shfl_up(incl, 1, 64);
  if (lane == 0) before = 0;
  for (uint32_t v = 0; v < w; v++) before = wmax[v] > before ? wmax[v] : before;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t i = tid * PER + k;
    if (i < ns) out[i] = sp[i] > before ? sp[i] : before;
  }
}
