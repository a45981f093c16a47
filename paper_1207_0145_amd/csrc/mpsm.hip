// Host side of the C ABI: argument checks, the plan (sizes, workspace
// layout), and the launch sequence of the P-MPSM phases on one stream.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "kernels.h"
#include "mpsm.h"

namespace {

constexpr uint32_t HIST_TILE = 9 * SCAT_CH;   // tuples per histogram / scatter tile (9 chunks of the scatter)
constexpr uint32_t IDX_STRIDE = 256;          // equi-height index stride of S runs
constexpr uint64_t DEFAULT_SEED = 0x1207014500000000ull;
constexpr uint64_t TAG_S = 0x5300000000000001ull, TAG_R1 = 0x5200000000000001ull, TAG_R2 = 0x5200000000000002ull;
constexpr uint64_t TAG_CR = 0x4352000000000001ull, TAG_CS = 0x4353000000000001ull;  // learned-CDF samples

uint32_t next_pow2(uint64_t x) {
  uint32_t p = 1;
  while (p < x && p < (1u << 30)) p <<= 1;
  return p;
}
uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

struct Plan {
  int swapped;
  uint64_t nR, nS;           // internal roles
  uint32_t L, Q, NBs, OSs;
  uint32_t levels, NB1, OS1, NB2, OS2;
  uint32_t QR;                 // B-MPSM (no range partitioning): sorted R runs of L tuples
  // bucket passes without a histogram (sample-sized regions in areas of
  // pad_area tuples): S's runs, R's runs (B-MPSM), R's second level
  int padS, padR1, padR2;
  // S in host memory (the memory-constrained variant): S is sorted and
  // joined in chunks of nSc tuples (Qc runs each), whose sorted runs then go
  // back to host memory.  Otherwise nSc = nS and Qc = Q.
  int hostS;
  uint64_t nSc;
  uint32_t Qc;
  uint64_t runtab;   // hostS: start and length of every run (Q + 1 entries each)
  uint32_t Gs, Gr, Pmax;
  uint32_t idx_per_run;
  uint32_t JCH, BT;
  int search, splitter, want_max;
  uint64_t seed;
  uint32_t tilesS, tilesR1, tilesR2;       // upper bounds of histogram tiles
  uint64_t cntS, cntR1, cntR2;             // count-matrix lengths
  uint64_t item_cap;                       // upper bound of join work items
  // workspace offsets (bytes)
  uint64_t T, U, R1, R2;
  uint64_t cS, cR1, cR2, bsum, bsumR;
  uint64_t segS, segR1, segR2;             // 4 arrays each: start, len, tile0, cnt0
  uint64_t splS, splR1, splR2;
  uint64_t bstS, bstR1, bstR2;
  uint64_t bndS, bndR1, bndR2;             // per-bucket key bounds (lo array, then hi array)
  uint64_t bigS, midS, redoS, midR, redoR, redoR2, bigR, ctr;
  uint64_t bkey, Pc, pstart, plen, pkey;
  uint64_t ridx, o, items, item_pre, item_cnt, res, span, pterm, qe;
  uint64_t cdf_chunks, cdf_sorted, modelR, modelS;  // learned CDF samples and models
  uint64_t cost_sample, cost_s_below, cost_best;   // cost-balanced splitters
  uint64_t capS, rstS, fillS, bsrcS, dirtyS;        // S's regions (padS)
  uint64_t capR1, rstR1, fillR1, bsrcR1, dirtyR1;   // R's level-1 regions (padR1)
  uint64_t capR2, rstR2, fillR2, bsrcR2, dirtyR2;   // R's level-2 regions (padR2)
  uint64_t total;
};

struct Seg {  // device pointers of one segment table (nseg + 1 entries each)
  uint32_t *start, *len, *tile0, *cnt0, *nb, *b0;
};

bool config_valid(const mpsm_config* c) {
  if (c->struct_size != sizeof(mpsm_config)) return false;
  if (c->role < 0 || c->role > 2) return false;
  if (c->splitter != MPSM_SPLIT_SAMPLED && c->splitter != MPSM_SPLIT_LEARNED && c->splitter != MPSM_SPLIT_COST &&
      c->splitter != MPSM_SPLIT_NONE)
    return false;
  if (c->search < 0 || c->search > 3) return false;
  if (c->log2_run_len && (c->log2_run_len < 12 || c->log2_run_len > 24)) return false;
  if (c->bucket_target && (c->bucket_target < 256 || c->bucket_target > 4096)) return false;
  if (c->join_chunk && (c->join_chunk < 1024 || c->join_chunk > (uint32_t)JOIN_CHUNK_MAX)) return false;
  if (c->oversample > 64 || c->waves > 64) return false;
  return true;
}

bool make_plan(uint64_t nR_c, uint64_t nS_c, const mpsm_config* cfg, Plan* P, uint64_t chunk = 0) {
  memset(P, 0, sizeof(*P));
  if (nR_c >= (1ull << 32) || nS_c >= (1ull << 32)) return false;
  P->hostS = chunk != 0;
  // with S in host memory the roles stay as given (S is the public input)
  P->swapped = !P->hostS && (cfg->role == MPSM_ROLE_SWAP || (cfg->role == MPSM_ROLE_AUTO && nS_c < nR_c));
  P->nR = P->swapped ? nS_c : nR_c;
  P->nS = P->swapped ? nR_c : nS_c;
  P->search = cfg->search;
  P->splitter = cfg->splitter;
  P->want_max = cfg->want_max ? 1 : 0;
  P->seed = cfg->seed;
  const uint32_t BT = cfg->bucket_target ? cfg->bucket_target : 4096u;   // R partitions
  // S buckets: a mean of 2400 tuples (any count works: buckets are cut by
  // splitters, not by key bits).  Buckets up to 1.7x the mean fit the
  // two-per-CU sort's 4096-tuple tile.  A key that matches one splitter only
  // (under two buckets' worth of copies) stays in its bucket, which can then
  // hold about three means: 3 x 2400 leaves room below the 8192-tuple tile,
  // where 3 x 2730 already let Zipf-distributed keys overflow it.
  const uint32_t BTs = BT < S_BUCKET_MEAN ? BT : S_BUCKET_MEAN;
  // S runs
  uint64_t L;
  if (cfg->log2_run_len) L = 1ull << cfg->log2_run_len;
  else {
    // about 128 runs, but no longer than MAX_NB buckets of the mean size:
    // longer runs get larger buckets, half of which overflow the two-per-CU
    // sort's tile and go to the slower one-per-CU sort
    L = next_pow2(cdiv(P->nS ? P->nS : 1, 128));
    if (L < (1u << 16)) L = 1u << 16;
    while (L > (1u << 16) && L > (uint64_t)MAX_NB * S_BUCKET_MEAN) L >>= 1;
  }
  P->L = (uint32_t)L;
  P->Q = P->nS ? (uint32_t)cdiv(P->nS, L) : 1;
  if (P->Q > (uint32_t)JOIN_QMAX) return false;
  P->nSc = P->nS;
  if (P->hostS) {   // whole runs per chunk
    uint64_t c = chunk / L * L;
    if (c < L) c = L;
    if (c < P->nSc) P->nSc = c;
  }
  P->Qc = P->nSc ? (uint32_t)cdiv(P->nSc, L) : 1;
  P->NBs = (uint32_t)cdiv(L, BTs);
  if (P->NBs > (uint32_t)MAX_NB) P->NBs = MAX_NB;
  const uint32_t OSreq = cfg->oversample ? cfg->oversample : 32u;
  auto os_for = [&](uint32_t NB) { return NB > 1 ? (SMP_CAP / NB < OSreq ? SMP_CAP / NB : OSreq) : 1u; };
  P->OSs = os_for(P->NBs);
  // R partitioning levels
  const uint64_t F = cdiv(P->nR ? P->nR : 1, BT);
  P->QR = 1;
  if (P->splitter == MPSM_SPLIT_NONE) {
    // B-MPSM: R sorted into runs of L tuples exactly as S is (one bucket
    // pass per run, then the bucket sort); the buckets of a run are its
    // partitions, and every R run meets every S run
    P->levels = 1;
    P->QR = P->nR ? (uint32_t)cdiv(P->nR, L) : 1;
    P->NB1 = P->NBs;
    P->OS1 = P->OSs;
    P->NB2 = 1;
    P->OS2 = 1;
  } else if (F <= (uint64_t)MAX_NB) {
    P->levels = 1;
    P->NB1 = next_pow2(F);
    P->OS1 = os_for(P->NB1);
    P->NB2 = 1;
    P->OS2 = 1;
  } else {
    // first level: a modest fan-out (long write segments in the scatter);
    // second level: buckets sized from the data
    P->levels = 2;
    P->NB1 = 256;
    P->OS1 = os_for(P->NB1);
    // level-2 buckets per level-1 bucket: ceil(len / BT), at most twice the
    // average need (level-1 buckets are sampled, so their sizes vary)
    P->NB2 = 2 * next_pow2(cdiv(F, P->NB1));
    // cost-balanced first-level buckets differ in size by design (fewer R
    // tuples where S is dense): room for the largest to be cut to the target
    if (P->splitter == MPSM_SPLIT_COST || P->NB2 > (uint32_t)MAX_NB) P->NB2 = MAX_NB;
    // 16 samples per level-2 bucket while they fit the small sample sort
    // (NB2 <= 128), 24 once the larger sort is needed anyway: with 4, bucket
    // sizes spread so far that about 1% exceed the LDS tile, and on R with
    // many duplicate keys (2^28 log-normal keys) 24 against 16 balances the
    // partitions better (-0.7 ms of the whole join)
    const uint32_t OS2def = (uint64_t)P->NB2 * 16 <= (uint64_t)(SMP_NT_S * SMP_IPT_S) ? 16u : 24u;
    const uint32_t OS2req = cfg->oversample ? cfg->oversample : OS2def;
    P->OS2 = SMP_CAP / P->NB2 < OS2req ? SMP_CAP / P->NB2 : OS2req;
  }
  P->Gs = P->Qc * P->NBs;
  P->Gr = P->QR * P->NB1 * P->NB2;
  P->Pmax = P->Gr + (P->splitter == MPSM_SPLIT_NONE ? P->QR : 0u);   // B-MPSM: one terminator per R run
  P->idx_per_run = (uint32_t)cdiv(L, IDX_STRIDE);
  P->JCH = cfg->join_chunk ? cfg->join_chunk : 32768u;
  P->BT = BT;
  P->tilesS = (uint32_t)(P->nSc / HIST_TILE + P->Qc);
  P->tilesR1 = (uint32_t)(P->nR / HIST_TILE + P->QR);
  P->tilesR2 = (uint32_t)(P->nR / HIST_TILE + P->NB1);
  P->cntS = (uint64_t)P->tilesS * P->NBs;
  P->cntR1 = (uint64_t)P->tilesR1 * P->NB1;
  P->cntR2 = P->levels == 2 ? (uint64_t)P->tilesR2 * P->NB2 : 1;
  P->item_cap = P->nS / P->JCH + P->Pmax + 2;

  // Bucket passes scatter into sample-sized bucket regions without a
  // histogram pass when the relation is large enough for that pass to
  // matter; every segment gets an area of 2.75 times its length (the
  // regions' bound is about 2.5 times a bucket's mean size).  Every chunk
  // claims its room by one atomic per bucket, so the pass needs many
  // segments (S's runs, B-MPSM's R runs, R's level-1 buckets at the second
  // level): R's first level is one segment, all of R, and there the claims
  // of every chunk meet on the same 256 counters (measured: its scatter
  // 3x slower than histogram and scatter together).
  const bool big_r = P->nR >= (1u << 22) && pad_area(P->nR) < (1ull << 32);
  P->padS = P->nSc >= (1u << 22) && pad_area(P->nSc) < (1ull << 32);
  P->padR1 = big_r && P->splitter == MPSM_SPLIT_NONE;
  P->padR2 = big_r && P->levels == 2;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) { uint64_t o = off; off += (bytes + 255) & ~255ull; return o; };
  const uint64_t ts = sizeof(tup_t);
  P->T = take((P->padS ? pad_area(P->nSc) : P->nSc) * ts);
  // hostS: two chunks' runs (one copied in or out while the other is sorted)
  P->U = take(P->nSc * ts * (P->nSc < P->nS ? 2u : 1u));
  P->R1 = take((P->padR1 ? pad_area(P->nR) : P->nR) * ts);
  P->R2 = take((P->padR2 ? pad_area(P->nR) : P->nR) * ts);
  P->cS = take(P->cntS * 4);
  P->cR1 = take(P->cntR1 * 4);
  P->cR2 = take(P->cntR2 * 4);
  uint64_t maxscan = P->cntS;
  if (P->cntR1 > maxscan) maxscan = P->cntR1;
  if (P->cntR2 > maxscan) maxscan = P->cntR2;
  if (P->item_cap > maxscan) maxscan = P->item_cap;
  P->bsum = take((cdiv(maxscan, SCAN_BLOCK) + 1) * 4);
  P->bsumR = take((cdiv(maxscan, SCAN_BLOCK) + 1) * 4);   // R's scans, which may run beside S's
  P->segS = take(6ull * (P->Qc + 1) * 4);
  if (P->hostS) P->runtab = take(2ull * (P->Q + 1) * 4);
  P->segR1 = take(6ull * (P->QR + 1) * 4);
  P->segR2 = take(6ull * (P->NB1 + 1) * 4);
  P->splS = take((uint64_t)P->Qc * P->NBs * 8);
  P->splR1 = take((uint64_t)P->QR * P->NB1 * 8);
  P->splR2 = take((uint64_t)P->NB1 * P->NB2 * 8);
  P->bstS = take(((uint64_t)P->Gs + 1) * 4);
  P->bstR1 = take(((uint64_t)P->QR * P->NB1 + 1) * 4);
  P->bstR2 = take(((uint64_t)P->Gr + 1) * 4);
  P->bndS = take((uint64_t)P->Gs * 16);
  P->bndR1 = take((uint64_t)P->QR * P->NB1 * 16);
  P->bndR2 = take((uint64_t)P->Gr * 16);
  P->bigS = take((uint64_t)P->Gs * 4);
  P->midS = take((uint64_t)P->Gs * 4);
  P->redoS = take((uint64_t)P->Gs * 4);
  P->midR = take((uint64_t)P->Gr * 4);
  P->redoR = take((uint64_t)P->Gr * 4);
  P->redoR2 = take((uint64_t)P->Gr * 4);
  P->bigR = take((uint64_t)P->Gr * 4);
  P->ctr = take(16 * 8);
  P->bkey = take((uint64_t)P->Gr * 8);
  P->Pc = take(4);
  P->pstart = take((uint64_t)P->Pmax * 4);
  P->plen = take((uint64_t)P->Pmax * 4);
  P->pkey = take((uint64_t)P->Pmax * 8);
  P->ridx = take((uint64_t)P->Q * P->idx_per_run * 8);
  P->o = take(((uint64_t)P->Pmax + 1) * P->Q * 4);
  P->items = take(((uint64_t)P->Pmax + 2) * 4);
  P->item_pre = take(((uint64_t)P->Pmax + 2) * 4);
  P->item_cnt = take((P->item_cap + 1) * 4);
  P->span = take((uint64_t)P->Pmax + 2);
  P->qe = take(((uint64_t)P->Pmax + 1) * 8);
  P->pterm = take((uint64_t)P->Pmax + 2);
  P->cdf_chunks = take(2ull * CDF_M * 8);
  P->cdf_sorted = take(2ull * CDF_M * 8);
  P->modelR = take(sizeof(CdfModel));
  P->modelS = take(sizeof(CdfModel));
  P->cost_sample = take((uint64_t)COST_MAX * 8);
  P->cost_s_below = take(((uint64_t)COST_MAX + 1) * 8);
  P->cost_best = take(8);
  if (P->padS) {
    P->capS = take((uint64_t)P->Gs * 4);
    P->rstS = take((uint64_t)P->Gs * 4);
    P->fillS = take((uint64_t)P->Gs * 4);
    P->bsrcS = take(((uint64_t)P->Gs + 1) * 4);
    P->dirtyS = take((uint64_t)P->Qc * 4);
  }
  if (P->padR1) {
    const uint64_t g1 = (uint64_t)P->QR * P->NB1;
    P->capR1 = take(g1 * 4);
    P->rstR1 = take(g1 * 4);
    P->fillR1 = take(g1 * 4);
    P->bsrcR1 = take((g1 + 1) * 4);
    P->dirtyR1 = take((uint64_t)P->QR * 4);
  }
  if (P->padR2) {
    P->capR2 = take((uint64_t)P->Gr * 4);
    P->rstR2 = take((uint64_t)P->Gr * 4);
    P->fillR2 = take((uint64_t)P->Gr * 4);
    P->bsrcR2 = take(((uint64_t)P->Gr + 1) * 4);
    P->dirtyR2 = take((uint64_t)P->NB1 * 4);
  }
  P->res = take(sizeof(Result));
  P->total = off;
  return true;
}

Seg seg_at(char* ws, uint64_t off, uint32_t nseg) {
  uint32_t* b = reinterpret_cast<uint32_t*>(ws + off);
  Seg s;
  s.start = b;
  s.len = b + (nseg + 1);
  s.tile0 = b + 2 * (nseg + 1);
  s.cnt0 = b + 3 * (nseg + 1);
  s.nb = b + 4 * (nseg + 1);
  s.b0 = b + 5 * (nseg + 1);
  return s;
}

// Start and length of each of the Q runs of L tuples over [0, n) (entry Q:
// start n, length 0).
__global__ void k_run_table(uint32_t* start, uint32_t* len, uint32_t Q, uint32_t L, uint32_t n) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > Q) return;
  const uint64_t a = (uint64_t)q * L;
  const uint32_t s = (uint32_t)(a < n ? a : n);
  start[q] = s;
  len[q] = q < Q ? (n - s < L ? n - s : L) : 0u;
}

// Run index of sorted runs that are already in place: entry i of run q is
// the key at the run's position i * stride (the entries the bucket sorts
// emit when they write the runs).
__global__ void k_run_index(const tup_t* runs, const uint32_t* start, const uint32_t* len, uint32_t Q,
                            uint32_t idx_per_run, uint32_t stride, uint64_t* run_idx) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)Q * idx_per_run) return;
  const uint32_t q = (uint32_t)(t / idx_per_run), i = (uint32_t)(t % idx_per_run);
  if ((uint64_t)i * stride < len[q]) run_idx[t] = runs[start[q] + i * stride].key;
}

// Zeroes the 64-bit words w[i] whose bit i is set in mask.
__global__ void k_clear_words(unsigned long long* w, uint32_t mask) {
  const uint32_t i = threadIdx.x;
  if (i < 32 && ((mask >> i) & 1u)) w[i] = 0;
}

#define HIP_TRY(x)                        \
  do {                                    \
    if ((x) != hipSuccess) return MPSM_EHIP; \
  } while (0)
#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

mpsm_status scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* bsum, hipStream_t st,
                     const uint32_t* enable = nullptr) {
  if (n == 0) return MPSM_OK;
  const uint32_t nb = (uint32_t)cdiv(n, SCAN_BLOCK);
  k_scan_reduce<<<nb, SCAN_NT, 0, st>>>(in, (uint32_t)n, bsum, enable);
  LAUNCH_CHECK();
  k_scan_apply<<<nb, SCAN_NT, 0, st>>>(in, out, (uint32_t)n, bsum, enable);
  LAUNCH_CHECK();
  return MPSM_OK;
}

// Step markers of the launch sequence (events recorded after each step).
const char* const kMarkers[] = {
    "start",        "init",          "cdf_models",    "s_splitters",   "s_histogram", "s_scan",          "s_scatter",
    "s_bucket_sort", "s_oversize_sort", "r1_splitters", "r1_histogram", "r1_scan",       "r1_scatter",
    "r2_splitters", "r2_histogram",  "r2_scan",       "r2_scatter",  "r_bucket_sort",   "r_oversize_sort",
    "partitions",   "search",        "join_plan",     "join",        "finalize"};
constexpr uint32_t kNumMarkers = sizeof(kMarkers) / sizeof(kMarkers[0]);
enum {
  MK_START, MK_INIT, MK_CDF, MK_S_SPL, MK_S_HIST, MK_S_SCAN, MK_S_SCAT, MK_S_SORT, MK_S_BIG, MK_R1_SPL, MK_R1_HIST,
  MK_R1_SCAN, MK_R1_SCAT, MK_R2_SPL, MK_R2_HIST, MK_R2_SCAN, MK_R2_SCAT, MK_R_SORT, MK_R_BIG, MK_PART, MK_SEARCH,
  MK_ITEMS, MK_JOIN, MK_FIN
};

struct Marker {
  void** ev;
  uint32_t n;
  hipStream_t st;
  bool ok = true;
  void mark(uint32_t i) {
    if (ev && i < n && hipEventRecord((hipEvent_t)ev[i], st) != hipSuccess) ok = false;
  }
  void mark_range(uint32_t a, uint32_t b) {  // steps a..b that were not run
    for (uint32_t i = a; i <= b; i++) mark(i);
  }
};

// Buffers of one bucket pass.
struct Level {
  Seg seg;
  uint32_t nseg, NBmax, BT, OS, max_tiles, Gmax;
  uint64_t level_seed;
  uint64_t* spl;
  uint32_t* cnt;
  uint64_t ncnt;
  uint32_t* bstart;
  uint64_t *blo, *bhi;
  const uint64_t* outer;     // splitters of the previous level (NULL at the first level)
  uint32_t outer_nspl;
  const CdfModel* model;     // learned splitters from this model, or NULL
  const struct CostArgs* cost;  // cost-balanced splitters (one segment), or NULL
  // where the segment table comes from (see k_seg_plan): runs of run_len
  // tuples, the buckets of a previous level, or filled in beforehand
  uint32_t run_len = 0;
  const uint32_t* src_bstart = nullptr;
  // a pass without a histogram (rg.cap set): buckets in sample-sized regions
  // of dst, read through bsrc (see k_bucket_scatter)
  Regions rg{};
  uint32_t* bsrc = nullptr;
  const uint32_t* Gcount() const { return seg.b0 + nseg; }
};

Level make_level(char* ws, uint64_t seg_off, uint32_t nseg, uint32_t NBmax, uint32_t BT, uint32_t OS,
                 uint32_t max_tiles, uint64_t level_seed, uint64_t spl_off, uint64_t cnt_off, uint64_t ncnt,
                 uint64_t bst_off, uint64_t bnd_off, uint32_t Gmax) {
  Level L;
  L.seg = seg_at(ws, seg_off, nseg);
  L.nseg = nseg; L.NBmax = NBmax; L.BT = BT; L.OS = OS; L.max_tiles = max_tiles; L.Gmax = Gmax;
  L.level_seed = level_seed;
  L.spl = reinterpret_cast<uint64_t*>(ws + spl_off);
  L.cnt = reinterpret_cast<uint32_t*>(ws + cnt_off);
  L.ncnt = ncnt;
  L.bstart = reinterpret_cast<uint32_t*>(ws + bst_off);
  L.blo = reinterpret_cast<uint64_t*>(ws + bnd_off);
  L.bhi = L.blo + Gmax;
  L.outer = nullptr;
  L.outer_nspl = 0;
  L.model = nullptr;
  L.cost = nullptr;
  return L;
}

// Inputs of the cost-balanced splitters: the sorted S runs' equi-height
// bounds and room for the sorted R sample, the S counts and the result.
struct CostArgs {
  uint64_t* sample;
  uint64_t* s_below;
  double* best;
  const uint64_t* run_idx;
  const uint32_t* run_len;
  uint32_t Q, idx_per_run, stride;
  uint64_t nS, nR;
};

// One bucket pass over segments: splitters, histogram, scan, scatter, table.
// Markers mk0 .. mk0+3 follow splitters, histogram, scan and scatter.
mpsm_status bucket_pass(const tup_t* src, tup_t* dst, uint32_t n, const Level& L, uint32_t* bsum, hipStream_t st,
                        Marker& mk, uint32_t mk0, const tup_t* const* seg_src = nullptr) {
  const Seg& sg = L.seg;
  k_seg_plan<<<1, 1024, 0, st>>>(L.nseg, L.NBmax, L.BT, HIST_TILE, n, L.run_len, L.src_bstart, sg.start, sg.len,
                                 sg.tile0, sg.cnt0, sg.nb, sg.b0);
  LAUNCH_CHECK();
  if (L.NBmax > 1 && L.cost) {
    // the whole sorted sample, the S distribution at its keys, the min-max split
    const CostArgs& c = *L.cost;
    const uint32_t M = L.NBmax * L.OS;
    if (M <= (uint32_t)(SMP_NT_S * SMP_IPT_S))
      k_sample_splitters<SMP_NT_S, SMP_IPT_S><<<1, SMP_NT_S, 0, st>>>(src, sg.start, sg.len, sg.nb, L.NBmax, L.OS,
                                                                      L.level_seed, L.spl, seg_src, c.sample, L.rg,
                                                                      sg.b0);
    else
      k_sample_splitters<SMP_NT, SMP_IPT><<<1, SMP_NT, 0, st>>>(src, sg.start, sg.len, sg.nb, L.NBmax, L.OS,
                                                                L.level_seed, L.spl, seg_src, c.sample, L.rg, sg.b0);
    LAUNCH_CHECK();
    k_cost_s_cdf<<<(uint32_t)cdiv((uint64_t)M + 1, 4), 256, 0, st>>>(c.sample, M, c.run_idx, c.run_len, c.Q,
                                                                    c.idx_per_run, c.stride, c.nS, c.s_below);
    LAUNCH_CHECK();
    k_cost_splitters<<<1, COST_NT, 0, st>>>(c.sample, c.s_below, M, c.nR, L.NBmax, c.Q, L.spl, c.best);
    LAUNCH_CHECK();
  } else if (L.NBmax > 1 && L.model) {
    k_learned_splitters<<<L.nseg, 256, 0, st>>>(L.model, L.NBmax, sg.nb, L.outer, L.outer_nspl, L.spl);
    LAUNCH_CHECK();
  } else if (L.NBmax > 1) {
    if (L.NBmax * L.OS <= (uint32_t)(SMP_NT_S * SMP_IPT_S))
      k_sample_splitters<SMP_NT_S, SMP_IPT_S><<<L.nseg, SMP_NT_S, 0, st>>>(src, sg.start, sg.len, sg.nb, L.NBmax,
                                                                           L.OS, L.level_seed, L.spl, seg_src,
                                                                           nullptr, L.rg, sg.b0);
    else
      k_sample_splitters<SMP_NT, SMP_IPT><<<L.nseg, SMP_NT, 0, st>>>(src, sg.start, sg.len, sg.nb, L.NBmax, L.OS,
                                                                     L.level_seed, L.spl, seg_src, nullptr, L.rg, sg.b0);
    LAUNCH_CHECK();
  }
  mk.mark(mk0);
  if (L.rg.cap) {
    // no histogram: every chunk claims room in its buckets' regions; the
    // segments where a bucket outgrew its region are redone (histogram,
    // scan, unstaged scatter), whose launches end at once when no segment
    // needs it
    mk.mark_range(mk0 + 1, mk0 + 2);
    k_bucket_scatter<true><<<L.max_tiles, SCAT_NT, 0, st>>>(src, dst, sg.start, sg.len, sg.tile0, sg.cnt0, sg.nb,
                                                            L.nseg, L.spl, L.NBmax, HIST_TILE, nullptr, seg_src, L.rg,
                                                            sg.b0);
    LAUNCH_CHECK();
    k_bucket_hist<<<L.max_tiles, HIST_NT, 0, st>>>(src, sg.start, sg.len, sg.tile0, sg.cnt0, sg.nb, L.nseg, L.spl,
                                                   L.NBmax, HIST_TILE, L.cnt, seg_src, L.rg.dirty);
    LAUNCH_CHECK();
    mpsm_status rc = scan_u32(L.cnt, L.cnt, L.ncnt, bsum, st, L.rg.any);
    if (rc != MPSM_OK) return rc;
    k_redo_scatter<<<L.max_tiles, HIST_NT, 0, st>>>(src, dst, sg.start, sg.len, sg.tile0, sg.cnt0, sg.nb, L.nseg,
                                                    L.spl, L.NBmax, HIST_TILE, L.cnt, seg_src, L.rg.dirty);
    LAUNCH_CHECK();
    k_region_table<1024><<<L.nseg, 1024, 0, st>>>(L.nseg, L.NBmax, sg.start, sg.len, sg.nb, sg.b0, L.rg, L.spl,
                                                  L.outer, L.outer_nspl, L.bstart, L.bsrc, L.blo, L.bhi);
    LAUNCH_CHECK();
    mk.mark(mk0 + 3);
    return MPSM_OK;
  }
  if (L.max_tiles) {
    k_bucket_hist<<<L.max_tiles, HIST_NT, 0, st>>>(src, sg.start, sg.len, sg.tile0, sg.cnt0, sg.nb, L.nseg, L.spl,
                                                   L.NBmax, HIST_TILE, L.cnt, seg_src, nullptr);
    LAUNCH_CHECK();
    mk.mark(mk0 + 1);
    mpsm_status rc = scan_u32(L.cnt, L.cnt, L.ncnt, bsum, st);
    if (rc != MPSM_OK) return rc;
    mk.mark(mk0 + 2);
    k_bucket_scatter<false><<<L.max_tiles, SCAT_NT, 0, st>>>(src, dst, sg.start, sg.len, sg.tile0, sg.cnt0, sg.nb,
                                                             L.nseg, L.spl, L.NBmax, HIST_TILE, L.cnt, seg_src,
                                                             Regions{}, nullptr);
    LAUNCH_CHECK();
  } else {
    mk.mark_range(mk0 + 1, mk0 + 2);
  }
  k_bucket_table<<<(uint32_t)cdiv((uint64_t)L.Gmax + 1, 256), 256, 0, st>>>(
      L.nseg, L.NBmax, sg.start, sg.tile0, sg.cnt0, sg.nb, sg.b0, sg.len, L.cnt, L.spl, L.outer, L.outer_nspl,
      L.bstart, L.blo, L.bhi);
  LAUNCH_CHECK();
  mk.mark(mk0 + 3);
  return MPSM_OK;
}

// A stream of the calling thread's own for the work that runs beside phase 1
// (the learned-CDF kernels, R's partitioning and sort), and the events that
// order it against the caller's stream (created once per thread and device,
// on the device current at the call, default priority).
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, gate = nullptr, done = nullptr;
  // copies of S's chunks in and of their runs out (S in host memory), one
  // stream per direction, and the events that order them
  hipStream_t cin = nullptr, cout = nullptr;
  hipEvent_t c_start = nullptr, c_in = nullptr, c_sorted = nullptr, c_out = nullptr, c_joined = nullptr;
};
constexpr int SIDE_MAX_DEVICES = 64;
thread_local SideStream t_side[SIDE_MAX_DEVICES];

mpsm_status side_stream(SideStream** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SIDE_MAX_DEVICES) return MPSM_EUNSUPPORTED;
  SideStream& s = t_side[dev];
  if (!s.st) {
    HIP_TRY(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&s.fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&s.gate, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
  }
  *out = &s;
  return MPSM_OK;
}

// The side stream's copy streams and their events (each created on first
// use, so that a call after a failed creation makes the missing ones).
mpsm_status copy_streams(SideStream* s) {
  for (hipStream_t* q : {&s->cin, &s->cout})
    if (!*q) HIP_TRY(hipStreamCreateWithFlags(q, hipStreamNonBlocking));
  for (hipEvent_t* e : {&s->c_start, &s->c_in, &s->c_sorted, &s->c_out, &s->c_joined})
    if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return MPSM_OK;
}

// Sample CDF_M keys of each relation of the job, sort them, fit the learned
// CDFs (nmodel = 1 or 2 models built side by side).
mpsm_status train_cdf(const CdfJob& job, uint32_t nmodel, uint64_t* chunks, uint64_t* sorted, hipStream_t st) {
  k_cdf_sample<<<dim3(CDF_M / 256, nmodel), 256, 0, st>>>(job, chunks);
  LAUNCH_CHECK();
  k_cdf_sort_chunks<<<dim3(CDF_M / CDF_CHUNK, nmodel), 1024, 0, st>>>(chunks);
  LAUNCH_CHECK();
  k_cdf_merge<<<dim3(CDF_M / 256, nmodel), 256, 0, st>>>(chunks, sorted);
  LAUNCH_CHECK();
  k_cdf_train<<<dim3(1, nmodel), 1024, 0, st>>>(sorted, job);
  LAUNCH_CHECK();
  return MPSM_OK;
}

int g_num_cus = 0;

}  // namespace

extern "C" {

void mpsm_config_default(mpsm_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(mpsm_config);
  cfg->role = MPSM_ROLE_AUTO;
  cfg->splitter = MPSM_SPLIT_SAMPLED;
  cfg->search = MPSM_SEARCH_INDEX;
  cfg->seed = DEFAULT_SEED;
}

const char* mpsm_status_string(mpsm_status s) {
  switch (s) {
    case MPSM_OK: return "ok";
    case MPSM_EINVAL: return "invalid argument";
    case MPSM_ECAPACITY: return "pair buffer too small";
    case MPSM_ENOMEM: return "workspace too small";
    case MPSM_EHIP: return "HIP runtime error";
    case MPSM_EUNSUPPORTED: return "unsupported option";
  }
  return "unknown status";
}

uint64_t mpsm_workspace_bytes(uint64_t nR, uint64_t nS, const mpsm_config* cfg) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!config_valid(cfg)) return 0;
  Plan P;
  if (!make_plan(nR, nS, cfg, &P)) return 0;
  return P.total;
}

mpsm_status mpsm_workspace_layout(uint64_t nR, uint64_t nS, const mpsm_config* cfg, mpsm_layout* out) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!out || !config_valid(cfg)) return MPSM_EINVAL;
  Plan P;
  if (!make_plan(nR, nS, cfg, &P)) return MPSM_EINVAL;
  memset(out, 0, sizeof(*out));
  out->swapped = (uint32_t)P.swapped;
  out->levels = P.levels;
  out->run_len = P.L;
  out->runs = P.Q;
  out->s_buckets = P.NBs;
  out->r_buckets1 = P.NB1;
  out->r_buckets2 = P.NB2;
  out->s_oversample = P.OSs;
  out->r_oversample1 = P.OS1;
  out->r_oversample2 = P.OS2;
  out->s_level_seed = P.seed ^ TAG_S;
  out->r_level_seed1 = P.seed ^ TAG_R1;
  out->r_level_seed2 = P.seed ^ TAG_R2;
  out->off_s_sorted = P.U;
  out->off_r_sorted = P.levels == 2 ? P.R1 : P.R2;
  out->off_s_splitters = P.splS;
  out->off_r_splitters1 = P.splR1;
  out->off_r_splitters2 = P.splR2;
  out->off_s_bucket_start = P.bstS;
  out->off_r_bucket_start1 = P.bstR1;
  out->off_r_bucket_start = P.levels == 2 ? P.bstR2 : P.bstR1;
  out->off_partitions = P.Pc;
  out->off_part_start = P.pstart;
  out->off_part_len = P.plen;
  out->off_part_key = P.pkey;
  out->off_offsets = P.o;
  out->p_max = P.Pmax;
  out->idx_stride = IDX_STRIDE;
  out->off_run_index = P.ridx;
  out->idx_per_run = P.idx_per_run;
  out->padded_passes = (P.padS ? 1u : 0u) | (P.padR1 ? 2u : 0u) | (P.padR2 ? 4u : 0u);
  out->off_join_span = P.span;
  out->off_cost_sample = P.cost_sample;
  out->off_cost_s_below = P.cost_s_below;
  out->off_cost_best = P.cost_best;
  out->cost_cells = P.NB1 * P.OS1;
  out->off_cdf_model_r = P.modelR;
  out->off_cdf_model_s = P.modelS;
  out->cdf_seed_r = P.seed ^ TAG_CR;
  out->cdf_seed_s = P.seed ^ TAG_CS;
  out->cdf_sample = CDF_M;
  out->cdf_knots = CDF_K;
  return MPSM_OK;
}

}  // extern "C"

namespace {

// S in pinned host memory (the runs of S kept outside device memory, as the
// memory-constrained variant of Section 3.1 keeps them on disk): its tuples
// by host address (copies) and device address (the learned model's
// sample), where its sorted runs go, and the tuples of whole runs copied in,
// sorted and joined at a time.
struct HostS {
  const tup_t* S_host;
  const tup_t* S_dev;
  tup_t* runs_host;
  uint64_t chunk;
  // S's sorted runs are already in host memory (runs_dev, their device
  // address): no run generation, only the join, which reads them there
  bool spilled;
  const tup_t* runs_dev;
};

mpsm_status join_impl(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS, uint64_t* d_out_count,
                      uint64_t* d_out_checksum, mpsm_pair* d_pairs, uint64_t pairs_capacity, const mpsm_config* cfg,
                      void* d_workspace, uint64_t workspace_bytes, void* stream, mpsm_stats* stats, void** events,
                      uint32_t n_events, bool single_stream = false, const HostS* hs = nullptr) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!config_valid(cfg)) return MPSM_EINVAL;
  if ((nR && !d_R) || (nS && !d_S) || !d_out_count || !d_out_checksum || !d_workspace) return MPSM_EINVAL;
  if (((uintptr_t)d_R & 15) || ((uintptr_t)d_S & 15) || ((uintptr_t)d_workspace & 255) ||
      ((uintptr_t)d_out_count & 7) || ((uintptr_t)d_out_checksum & 7) || ((uintptr_t)d_pairs & 7))
    return MPSM_EINVAL;
  if (d_pairs && pairs_capacity == 0) d_pairs = nullptr;
  Plan P;
  if (!make_plan(nR, nS, cfg, &P, hs ? hs->chunk : 0)) return MPSM_EINVAL;
  if (workspace_bytes < P.total) return MPSM_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  if (!g_num_cus) {
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    g_num_cus = ncu > 0 ? ncu : 256;
  }
  // learned splitters use R's model, the learned search S's; both are built
  // on a side stream while phase 1 runs and joined before R's partitioning.
  const bool learn_r = P.splitter == MPSM_SPLIT_LEARNED && P.nR && P.nS;
  const bool learn_s = P.search == MPSM_SEARCH_LEARNED && P.nR && P.nS;
  // R's partitioning and sort run on the side stream too, beside S's run
  // generation (they are independent until the search), except with
  // cost-balanced splitters, which need S's runs.  They start once S's
  // tuples are scattered into runs: beside S's histogram and scatter, both
  // bound by HBM and on the critical path, R's passes took bandwidth from
  // them; S's bucket sort, bound by its ALU work, leaves more of it.
  const bool r_side = P.splitter != MPSM_SPLIT_COST && P.nR && P.nS && !single_stream;
  // the side stream and its events exist before anything is enqueued
  SideStream* side = nullptr;
  if ((learn_r || learn_s || r_side || P.hostS) && !single_stream) {
    mpsm_status rs = side_stream(&side);
    if (rs == MPSM_OK && P.hostS) rs = copy_streams(side);
    if (rs != MPSM_OK) return rs;
  }
  if (P.hostS && !side) return MPSM_EINVAL;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    HIP_TRY(hipEventRecord(ev0, st));
  }
  // the launch sequence; on a failure after the side stream was forked, the
  // caller's stream is made to wait for it before returning
  bool forked = false, copies_forked = false;
  Marker mk{events, n_events, st};
  char* ws = static_cast<char*>(d_workspace);
  const tup_t* Rin = reinterpret_cast<const tup_t*>(P.swapped ? d_S : d_R);
  const tup_t* Sin = reinterpret_cast<const tup_t*>(P.swapped ? d_R : d_S);
  tup_t* T = reinterpret_cast<tup_t*>(ws + P.T);
  tup_t* U = reinterpret_cast<tup_t*>(ws + P.U);
  tup_t* R1 = reinterpret_cast<tup_t*>(ws + P.R1);
  tup_t* R2 = reinterpret_cast<tup_t*>(ws + P.R2);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(ws + P.bsum);
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(ws + P.ctr);
  Result* res = reinterpret_cast<Result*>(ws + P.res);
  CdfModel* modelR = reinterpret_cast<CdfModel*>(ws + P.modelR);
  CdfModel* modelS = reinterpret_cast<CdfModel*>(ws + P.modelS);
  auto enqueue = [&]() -> mpsm_status {
    mk.mark(MK_START);
    k_init_result<<<1, 64, 0, st>>>(res, reinterpret_cast<uint32_t*>(ctr), 32);
    LAUNCH_CHECK();
    mk.mark(MK_INIT);
    // The side stream may start from here (fork); its kernels are enqueued
    // once phase 1's first long kernels are, so that the host time their
    // launches take never leaves the GPU waiting.  Without a side stream
    // the models are built on the caller's stream.
    if (side) {
      HIP_TRY(hipEventRecord(side->fork, st));
      forked = true;
    }
    auto start_models = [&]() -> mpsm_status {
      if (side) HIP_TRY(hipStreamWaitEvent(side->st, side->fork, 0));
      if (!learn_r && !learn_s) return MPSM_OK;
      CdfJob job;
      memset(&job, 0, sizeof(job));
      uint32_t nm = 0;
      if (learn_r) { job.src[nm] = Rin; job.n[nm] = (uint32_t)P.nR; job.seed[nm] = P.seed ^ TAG_CR; job.model[nm] = modelR; nm++; }
      if (learn_s) { job.src[nm] = hs ? hs->S_dev : Sin; job.n[nm] = (uint32_t)P.nS; job.seed[nm] = P.seed ^ TAG_CS; job.model[nm] = modelS; nm++; }
      mpsm_status rc = train_cdf(job, nm, reinterpret_cast<uint64_t*>(ws + P.cdf_chunks),
                                 reinterpret_cast<uint64_t*>(ws + P.cdf_sorted), side ? side->st : st);
      if (rc != MPSM_OK) return rc;
      if (side && !r_side) HIP_TRY(hipEventRecord(side->done, side->st));
      return MPSM_OK;
    };
    mk.mark(MK_CDF);
    if (P.nR == 0 || P.nS == 0) {
      mk.mark_range(MK_S_SPL, MK_JOIN);  // MK_CDF was recorded above
      k_finalize<<<1, 64, 0, st>>>(res, d_out_count, d_out_checksum, d_pairs ? pairs_capacity : 0);
      LAUNCH_CHECK();
      mk.mark(MK_FIN);
    } else {
      mpsm_status rc;
      // ---- phase 1: sort S into Q runs of L tuples
      Level LS = make_level(ws, P.segS, P.Qc, P.NBs, 0, P.OSs, P.tilesS, P.seed ^ TAG_S, P.splS, P.cS, P.cntS, P.bstS,
                            P.bndS, P.Gs);
      LS.run_len = P.L;
      // regions of a pass without a histogram; `any` is a word of ctr,
      // which k_init_result zeroes
      auto regions = [&](Level& Lv, uint64_t cap, uint64_t rst, uint64_t fill, uint64_t dirty, uint64_t bsrc,
                         uint32_t any_word) {
        Lv.rg.cap = reinterpret_cast<uint32_t*>(ws + cap);
        Lv.rg.start = reinterpret_cast<uint32_t*>(ws + rst);
        Lv.rg.fill = reinterpret_cast<uint32_t*>(ws + fill);
        Lv.rg.dirty = reinterpret_cast<uint32_t*>(ws + dirty);
        Lv.rg.any = reinterpret_cast<uint32_t*>(ctr + any_word);
        Lv.bsrc = reinterpret_cast<uint32_t*>(ws + bsrc);
      };
      uint64_t* const ridx = reinterpret_cast<uint64_t*>(ws + P.ridx);
      uint32_t* midS = reinterpret_cast<uint32_t*>(ws + P.midS);
      uint32_t* bigS = reinterpret_cast<uint32_t*>(ws + P.bigS);
      uint32_t* redoS = reinterpret_cast<uint32_t*>(ws + P.redoS);
      // the bucket sorts of a pass over S's runs (T to dst); run_idx: the
      // index entries of the pass's first run
      auto sort_runs = [&](const Level& Lv, tup_t* dst, uint64_t* run_idx) -> mpsm_status {
        SortOut so;
        so.run_idx = run_idx;
        so.run_start = Lv.seg.start;
        so.idx_stride = IDX_STRIDE;
        so.idx_shift = __builtin_ctz(IDX_STRIDE);
        so.idx_per_run = P.idx_per_run;
        so.NB = P.NBs;
        so.bkey = nullptr;
        k_bucket_sort_cs<BS_NT, BS_IPT, BS_M, 8, false, false><<<P.Gs, BS_NT, 0, st>>>(T, dst, Lv.bstart, Lv.bsrc, Lv.blo, Lv.bhi, Lv.Gcount(),
                                                                     nullptr, nullptr, midS, ctr + 2, redoS, ctr + 3, so);
        LAUNCH_CHECK();
        k_bucket_sort_cs<BL_NT, BL_IPT, BL_M, 1, true, false><<<g_num_cus, BL_NT, 0, st>>>(T, dst, Lv.bstart, Lv.bsrc, Lv.blo, Lv.bhi, Lv.Gcount(),
                                                                          midS, ctr + 2, bigS, ctr + 0, redoS, ctr + 3,
                                                                          so);
        LAUNCH_CHECK();
        k_bucket_sort_lsd<<<g_num_cus, LSD_NT, 0, st>>>(T, dst, Lv.bstart, Lv.bsrc, redoS, ctr + 3, bigS, ctr + 0, so);
        LAUNCH_CHECK();
        mk.mark(MK_S_SORT);
        k_big_sort<<<g_num_cus, BIG_NT, 0, st>>>(T, dst, Lv.bstart, Lv.bsrc, bigS, ctr + 0, so);
        LAUNCH_CHECK();
        mk.mark(MK_S_BIG);
        return MPSM_OK;
      };
      if (!P.hostS) {
        if (P.padS) regions(LS, P.capS, P.rstS, P.fillS, P.dirtyS, P.bsrcS, 7);
        rc = bucket_pass(Sin, T, (uint32_t)P.nS, LS, bsum, st, mk, MK_S_SPL);
        if (rc != MPSM_OK) return rc;
        if (r_side) HIP_TRY(hipEventRecord(side->gate, st));
        rc = start_models();
        if (rc != MPSM_OK) return rc;
        rc = sort_runs(LS, U, ridx);
        if (rc != MPSM_OK) return rc;
      } else {
        // S in host memory: R's phases and partitions come first, on the
        // side stream, and S's chunks are sorted and joined after them
        rc = start_models();
        if (rc != MPSM_OK) return rc;
      }

      // ---- phase 2: range-partition R (one or two levels); phase 3: sort partitions
      const bool bmpsm = P.splitter == MPSM_SPLIT_NONE;
      Level LR1 = make_level(ws, P.segR1, P.QR, P.NB1, 0, P.OS1, P.tilesR1, P.seed ^ TAG_R1, P.splR1, P.cR1, P.cntR1,
                             P.bstR1, P.bndR1, P.QR * P.NB1);
      if (learn_r) LR1.model = modelR;
      CostArgs cost_args;
      if (P.splitter == MPSM_SPLIT_COST) {
        cost_args.sample = reinterpret_cast<uint64_t*>(ws + P.cost_sample);
        cost_args.s_below = reinterpret_cast<uint64_t*>(ws + P.cost_s_below);
        cost_args.best = reinterpret_cast<double*>(ws + P.cost_best);
        cost_args.run_idx = ridx;
        cost_args.run_len = LS.seg.len;
        cost_args.Q = P.Q;
        cost_args.idx_per_run = P.idx_per_run;
        cost_args.stride = IDX_STRIDE;
        cost_args.nS = P.nS;
        cost_args.nR = P.nR;
        LR1.cost = &cost_args;
      }
      // the models are needed from here on; R's phase runs on the side stream
      // after them, or on this stream after S's
      if (side && !r_side) HIP_TRY(hipStreamWaitEvent(st, side->done, 0));
      const hipStream_t rst = r_side ? side->st : st;
      if (r_side && !P.hostS) HIP_TRY(hipStreamWaitEvent(rst, side->gate, 0));
      uint32_t* const rbsum = r_side ? reinterpret_cast<uint32_t*>(ws + P.bsumR) : bsum;
      Marker mkR{events, n_events, rst};
      LR1.run_len = bmpsm ? P.L : (uint32_t)P.nR;   // B-MPSM: R runs; else one segment, all of R
      if (P.padR1) regions(LR1, P.capR1, P.rstR1, P.fillR1, P.dirtyR1, P.bsrcR1, 8);
      rc = bucket_pass(Rin, R1, (uint32_t)P.nR, LR1, rbsum, rst, mkR, MK_R1_SPL);
      if (rc != MPSM_OK) return rc;
      SortOut soR;
      soR.run_idx = nullptr;
      soR.run_start = nullptr;
      soR.idx_stride = 1;
      soR.idx_shift = 0;
      soR.idx_per_run = 0;
      soR.NB = 1;
      soR.bkey = reinterpret_cast<uint64_t*>(ws + P.bkey);
      uint32_t* redoR = reinterpret_cast<uint32_t*>(ws + P.redoR);
      uint32_t* bigR = reinterpret_cast<uint32_t*>(ws + P.bigR);
      const Level* LRf = &LR1;   // level whose buckets are the R partitions
      Level LR2;
      tup_t* Rsrc = R1;          // partitioned, unsorted
      tup_t* Rsorted = R2;
      if (P.levels == 2) {
        // 3/4 of the target so that sampling noise rarely pushes a partition past the LDS tile
        LR2 = make_level(ws, P.segR2, P.NB1, P.NB2, P.BT * 3 / 4, P.OS2, P.tilesR2, P.seed ^ TAG_R2, P.splR2, P.cR2, P.cntR2,
                         P.bstR2, P.bndR2, P.Gr);
        LR2.outer = LR1.spl;
        LR2.outer_nspl = P.NB1 - 1;
        // the second level stays sampled: its buckets are finer than the model's knots
        LR2.src_bstart = LR1.bstart;   // segments: the level-1 buckets
        if (P.padR2) regions(LR2, P.capR2, P.rstR2, P.fillR2, P.dirtyR2, P.bsrcR2, 9);
        rc = bucket_pass(R1, R2, (uint32_t)P.nR, LR2, rbsum, rst, mkR, MK_R2_SPL);
        if (rc != MPSM_OK) return rc;
        LRf = &LR2;
        Rsrc = R2;
        Rsorted = R1;
      } else {
        mkR.mark_range(MK_R2_SPL, MK_R2_SCAT);
      }
      // as for S runs: the 2-per-CU sort takes the buckets up to its tile, the
      // larger ones go to the 1-per-CU sort
      uint32_t* midR = reinterpret_cast<uint32_t*>(ws + P.midR);
      k_bucket_sort_cs<BS_NT, BS_IPT, BS_M, 8, false, false><<<LRf->Gmax, BS_NT, 0, rst>>>(Rsrc, Rsorted, LRf->bstart, LRf->bsrc, LRf->blo,
                                                                        LRf->bhi, LRf->Gcount(), nullptr, nullptr, midR,
                                                                        ctr + 6, redoR, ctr + 4, soR);
      LAUNCH_CHECK();
      k_bucket_sort_cs<BL_NT, BL_IPT, BL_M, 1, true, false><<<g_num_cus, BL_NT, 0, rst>>>(Rsrc, Rsorted, LRf->bstart, LRf->bsrc, LRf->blo,
                                                                        LRf->bhi, LRf->Gcount(), midR, ctr + 6, bigR,
                                                                        ctr + 1, redoR, ctr + 4, soR);
      LAUNCH_CHECK();
      // buckets the sort gave up on get a second pass over their own key range
      // (splitter bounds can enclose a gap between key clusters); the rest go
      // to the LSD radix sort
      uint32_t* redoR2 = reinterpret_cast<uint32_t*>(ws + P.redoR2);
      k_bucket_sort_cs<BL_NT, BL_IPT, BL_M, 1, true, true><<<g_num_cus, BL_NT, 0, rst>>>(Rsrc, Rsorted, LRf->bstart, LRf->bsrc, LRf->blo, LRf->bhi,
                                                                        LRf->Gcount(), redoR, ctr + 4, bigR, ctr + 1,
                                                                        redoR2, ctr + 5, soR);
      LAUNCH_CHECK();
      k_bucket_sort_lsd<<<g_num_cus, LSD_NT, 0, rst>>>(Rsrc, Rsorted, LRf->bstart, LRf->bsrc, redoR2, ctr + 5, bigR, ctr + 1, soR);
      LAUNCH_CHECK();
      mkR.mark(MK_R_SORT);
      k_big_sort<<<g_num_cus, BIG_NT, 0, rst>>>(Rsrc, Rsorted, LRf->bstart, LRf->bsrc, bigR, ctr + 1, soR);
      LAUNCH_CHECK();
      mkR.mark(MK_R_BIG);
      if (r_side && !P.hostS) {   // the rest needs R's partitions
        HIP_TRY(hipEventRecord(side->done, rst));
        HIP_TRY(hipStreamWaitEvent(st, side->done, 0));
      }
      // the partition table: on this stream after R's sort, or with S in
      // host memory on R's stream, which S's chunks wait for
      const hipStream_t pst = P.hostS ? rst : st;
      uint32_t* const pbsum = P.hostS ? rbsum : bsum;
      uint32_t* Pc = reinterpret_cast<uint32_t*>(ws + P.Pc);
      uint32_t* pstart = reinterpret_cast<uint32_t*>(ws + P.pstart);
      uint32_t* plen = reinterpret_cast<uint32_t*>(ws + P.plen);
      uint64_t* pkey = reinterpret_cast<uint64_t*>(ws + P.pkey);
      uint8_t* const pterm = bmpsm ? reinterpret_cast<uint8_t*>(ws + P.pterm) : nullptr;
      if (bmpsm) {
        k_partitions_runs<<<1, 1024, 0, pst>>>(LRf->bstart, soR.bkey, LRf->Gcount(), P.NB1, Pc, pstart, plen, pkey,
                                              pterm, stats ? res : nullptr);
        LAUNCH_CHECK();
      } else {
        // flags in items, their scan in item_pre (both free until the join's items are counted)
        uint32_t* flags = reinterpret_cast<uint32_t*>(ws + P.items);
        uint32_t* pre = reinterpret_cast<uint32_t*>(ws + P.item_pre);
        const uint32_t nb = (uint32_t)cdiv(LRf->Gmax, 256);
        k_partition_flags<<<nb, 256, 0, pst>>>(LRf->bstart, LRf->Gcount(), LRf->Gmax, flags);
        LAUNCH_CHECK();
        rc = scan_u32(flags, pre, LRf->Gmax, pbsum, pst);
        if (rc != MPSM_OK) return rc;
        k_partition_write<<<nb, 256, 0, pst>>>(LRf->bstart, soR.bkey, LRf->Gmax, flags, pre, Pc, pstart, plen, pkey,
                                              stats ? res : nullptr);
        LAUNCH_CHECK();
      }
      uint8_t* span = reinterpret_cast<uint8_t*>(ws + P.span);
      k_join_units<<<(uint32_t)cdiv(P.Pmax, 256), 256, 0, pst>>>(Pc, plen, P.Pmax, span, pterm);
      LAUNCH_CHECK();
      mk.mark(MK_PART);

      // ---- phase 4: merge starts of every partition in every run, then the join
      uint32_t* o = reinterpret_cast<uint32_t*>(ws + P.o);
      float2* qe = reinterpret_cast<float2*>(ws + P.qe);
      if (learn_s) {
        k_search_model<<<(uint32_t)cdiv(P.Pmax, 256), 256, 0, pst>>>(modelS, pkey, Pc, P.Pmax, qe);
        LAUNCH_CHECK();
      }
      // the search and the join over Qn runs of S in Ub (run_start / run_len
      // relative to Ub; run_idx: their index entries)
      auto search_join = [&](const tup_t* Ub, const uint32_t* run_start, const uint32_t* run_len, uint32_t Qn,
                             const uint64_t* run_idx) -> mpsm_status {
        const uint64_t nsearch = cdiv((uint64_t)P.Pmax + 1, 64) * cdiv(Qn, SEARCH_RUNS);
        k_search<<<(uint32_t)nsearch, SEARCH_NT, 0, st>>>(Ub, run_start, run_len, Qn, run_idx, IDX_STRIDE,
                                                              P.idx_per_run, Pc, pkey, P.Pmax, o,
                                                              learn_s ? MPSM_SEARCH_LEARNED
                                                                      : (P.search == MPSM_SEARCH_LEARNED ? MPSM_SEARCH_INDEX
                                                                                                         : P.search),
                                                              modelS, qe, stats ? res : nullptr, span, pterm);
        LAUNCH_CHECK();
        mk.mark(MK_SEARCH);
        uint32_t* items = reinterpret_cast<uint32_t*>(ws + P.items);
        uint32_t* item_pre = reinterpret_cast<uint32_t*>(ws + P.item_pre);
        k_join_items<<<(uint32_t)cdiv(((uint64_t)P.Pmax + 2) * 64, 256), 256, 0, st>>>(Pc, o, Qn, run_len, P.Pmax,
                                                                                       P.JCH, span, items);
        LAUNCH_CHECK();
        rc = scan_u32(items, item_pre, (uint64_t)P.Pmax + 2, bsum, st);
        if (rc != MPSM_OK) return rc;
        mk.mark(MK_ITEMS);

        JoinArgs A;
        A.Rs = Rsorted;
        A.U = Ub;
        A.run_start = run_start;
        A.run_len = run_len;
        A.Q = Qn;
        A.Pcount = Pc;
        A.pstart = pstart;
        A.plen = plen;
        A.o = o;
        A.item_pre = item_pre;
        A.Pmax = P.Pmax;
        A.JCH = P.JCH;
        A.res = res;
        A.J = nullptr;
        A.pjoin = nullptr;
        A.span = span;
        A.pairs = reinterpret_cast<uint64_t*>(d_pairs);
        A.pairs_cap = d_pairs ? pairs_capacity : 0;
        A.item_cnt = reinterpret_cast<uint32_t*>(ws + P.item_cnt);
        A.item_cap = (uint32_t)P.item_cap;
        A.swapped = P.swapped;
        const bool raw = P.swapped || P.want_max || d_pairs;
        if (raw) k_join<0, VAL_RAW><<<g_num_cus, JOIN_NT, 0, st>>>(A);
        else k_join<0, VAL_HR><<<g_num_cus, JOIN_NT, 0, st>>>(A);
        LAUNCH_CHECK();
        if (d_pairs) {
          k_join<1, VAL_RAW><<<g_num_cus, JOIN_NT, 0, st>>>(A);
          LAUNCH_CHECK();
          rc = scan_u32(A.item_cnt, A.item_cnt, P.item_cap, bsum, st);
          if (rc != MPSM_OK) return rc;
          k_join<2, VAL_RAW><<<g_num_cus, JOIN_NT, 0, st>>>(A);
          LAUNCH_CHECK();
        }
        return MPSM_OK;
      };
      if (!P.hostS) {
        rc = search_join(U, LS.seg.start, LS.seg.len, P.Q, ridx);
        if (rc != MPSM_OK) return rc;
      } else if (hs->spilled) {
        // S's runs in host memory from an earlier call: their run table and
        // run index (every stride-th key, read from the runs), then the
        // search and the join, which move through the key domain partition
        // by partition and read every run's slice of it over the host link
        uint32_t* rt = reinterpret_cast<uint32_t*>(ws + P.runtab);
        k_run_table<<<(uint32_t)cdiv((uint64_t)P.Q + 1, 256), 256, 0, st>>>(rt, rt + P.Q + 1, P.Q, P.L, (uint32_t)P.nS);
        LAUNCH_CHECK();
        k_run_index<<<(uint32_t)cdiv((uint64_t)P.Q * P.idx_per_run, 256), 256, 0, st>>>(
            hs->runs_dev, rt, rt + P.Q + 1, P.Q, P.idx_per_run, IDX_STRIDE, ridx);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(side->done, rst));   // R's partitions are ready
        HIP_TRY(hipStreamWaitEvent(st, side->done, 0));
        rc = search_join(hs->runs_dev, rt, rt + P.Q + 1, P.Q, ridx);
        if (rc != MPSM_OK) return rc;
      } else {
        HIP_TRY(hipEventRecord(side->done, rst));   // R's partitions are ready
        // S in host memory: the tuples of whole runs at a time are copied
        // into a buffer of U, bucketed into T, sorted back into the buffer,
        // joined there with every R partition (the join is a sum over runs)
        // and copied out to the host runs, if the caller keeps them.  Two buffers, so that the next
        // chunk comes in and the previous chunk's runs go out (one copy
        // stream per direction) while a chunk is sorted and joined.  The
        // counters of S's passes (words 0, 2, 3 and 7 of ctr) start at zero
        // in every chunk.
        SideStream& cs = *side;
        const uint32_t nbuf = P.nSc < P.nS ? 2u : 1u;
        const uint64_t nk = cdiv(P.nS, P.nSc);
        auto ubuf = [&](uint64_t k) { return U + (k % nbuf) * P.nSc; };
        auto clen = [&](uint64_t k) { return P.nS - k * P.nSc < P.nSc ? P.nS - k * P.nSc : P.nSc; };
        HIP_TRY(hipEventRecord(cs.c_start, st));
        HIP_TRY(hipStreamWaitEvent(cs.cin, cs.c_start, 0));
        HIP_TRY(hipStreamWaitEvent(cs.cout, cs.c_start, 0));
        copies_forked = true;
        HIP_TRY(hipMemcpyAsync(ubuf(0), hs->S_host, clen(0) * sizeof(tup_t), hipMemcpyHostToDevice, cs.cin));
        HIP_TRY(hipEventRecord(cs.c_in, cs.cin));
        for (uint64_t k = 0; k < nk; k++) {
          const uint64_t c = k * P.nSc, n = clen(k);
          const uint32_t q0 = (uint32_t)(c / P.L), qn = (uint32_t)cdiv(n, P.L);
          HIP_TRY(hipStreamWaitEvent(st, cs.c_in, 0));   // chunk k is in
          if (k + 1 < nk) {
            // chunk k + 1's buffer held chunk k - 1, which must be joined and out
            if (k >= 1) {
              HIP_TRY(hipStreamWaitEvent(cs.cin, cs.c_joined, 0));
              if (hs->runs_host) HIP_TRY(hipStreamWaitEvent(cs.cin, cs.c_out, 0));
            }
            HIP_TRY(hipMemcpyAsync(ubuf(k + 1), hs->S_host + c + P.nSc, clen(k + 1) * sizeof(tup_t),
                                   hipMemcpyHostToDevice, cs.cin));
            HIP_TRY(hipEventRecord(cs.c_in, cs.cin));
          }
          if (k) {
            k_clear_words<<<1, 64, 0, st>>>(ctr, (1u << 0) | (1u << 2) | (1u << 3) | (1u << 7));
            LAUNCH_CHECK();
          }
          Level LC = make_level(ws, P.segS, qn, P.NBs, 0, P.OSs, P.tilesS, P.seed ^ TAG_S, P.splS, P.cS, P.cntS,
                                P.bstS, P.bndS, qn * P.NBs);
          LC.run_len = P.L;
          if (P.padS) regions(LC, P.capS, P.rstS, P.fillS, P.dirtyS, P.bsrcS, 7);
          rc = bucket_pass(ubuf(k), T, (uint32_t)n, LC, bsum, st, mk, MK_S_SPL);
          if (rc != MPSM_OK) return rc;
          rc = sort_runs(LC, ubuf(k), ridx + (uint64_t)q0 * P.idx_per_run);
          if (rc != MPSM_OK) return rc;
          if (hs->runs_host) {
            HIP_TRY(hipEventRecord(cs.c_sorted, st));
            HIP_TRY(hipStreamWaitEvent(cs.cout, cs.c_sorted, 0));
            HIP_TRY(hipMemcpyAsync(hs->runs_host + c, ubuf(k), n * sizeof(tup_t), hipMemcpyDeviceToHost, cs.cout));
            HIP_TRY(hipEventRecord(cs.c_out, cs.cout));
          }
          if (k == 0) HIP_TRY(hipStreamWaitEvent(st, side->done, 0));
          rc = search_join(ubuf(k), LC.seg.start, LC.seg.len, qn, ridx + (uint64_t)q0 * P.idx_per_run);
          if (rc != MPSM_OK) return rc;
          HIP_TRY(hipEventRecord(cs.c_joined, st));
        }
        if (hs->runs_host) HIP_TRY(hipStreamWaitEvent(st, cs.c_out, 0));   // every run is in host memory
      }
      mk.mark(MK_JOIN);
      k_finalize<<<1, 64, 0, st>>>(res, d_out_count, d_out_checksum, d_pairs ? pairs_capacity : 0);
      LAUNCH_CHECK();
      mk.mark(MK_FIN);
    }
    return mk.ok ? MPSM_OK : MPSM_EHIP;
  };
  const mpsm_status erc = enqueue();
  if (erc != MPSM_OK) {
    if (forked) {
      (void)hipEventRecord(side->done, side->st);
      (void)hipStreamWaitEvent(st, side->done, 0);
    }
    if (copies_forked) {
      (void)hipEventRecord(side->c_in, side->cin);
      (void)hipStreamWaitEvent(st, side->c_in, 0);
      (void)hipEventRecord(side->c_out, side->cout);
      (void)hipStreamWaitEvent(st, side->c_out, 0);
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    return erc;
  }
  if (stats) {
    HIP_TRY(hipEventRecord(ev1, st));
    HIP_TRY(hipEventSynchronize(ev1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    Result r;
    HIP_TRY(hipMemcpy(&r, res, sizeof(r), hipMemcpyDeviceToHost));
    unsigned long long c[6];
    HIP_TRY(hipMemcpy(c, ctr, sizeof(c), hipMemcpyDeviceToHost));
    uint32_t pc = 0;
    if (P.nR && P.nS) HIP_TRY(hipMemcpy(&pc, ws + P.Pc, 4, hipMemcpyDeviceToHost));
    memset(stats, 0, sizeof(*stats));
    stats->max_payload_sum = r.maxsum;
    stats->nonempty = r.count > 0 ? 1 : 0;
    stats->partitions = pc;
    stats->runs = P.Q;
    stats->oversize_buckets = c[0] + c[1];
    stats->resorted_buckets = c[3] + c[5];
    stats->retried_buckets = c[4];
    stats->search_probes = r.search_probes;
    stats->search_fallbacks = r.fallbacks;
    stats->max_partition = r.spare;
    float eps_r = -1.f, eps_s = -1.f;
    if (learn_r) HIP_TRY(hipMemcpy(&eps_r, &modelR->eps, sizeof(float), hipMemcpyDeviceToHost));
    if (learn_s) HIP_TRY(hipMemcpy(&eps_s, &modelS->eps, sizeof(float), hipMemcpyDeviceToHost));
    stats->cdf_eps_r = eps_r;
    stats->cdf_eps_s = eps_s;
    stats->swapped = (uint64_t)P.swapped;
    stats->ms_total = ms;
    stats->pairs_truncated = r.truncated;
    // segments the exact path redid, from the dirty flags of each pass without a histogram
    auto redone = [&](bool on, uint64_t off, uint32_t nseg, uint64_t* out) -> mpsm_status {
      if (!on || !P.nR || !P.nS) return MPSM_OK;
      std::vector<uint32_t> dirty(nseg);
      HIP_TRY(hipMemcpy(dirty.data(), ws + off, (size_t)nseg * 4, hipMemcpyDeviceToHost));
      for (uint32_t d : dirty) *out += d ? 1 : 0;
      return MPSM_OK;
    };
    mpsm_status rr = redone(P.padS, P.dirtyS, P.Qc, &stats->redone_runs);
    if (rr == MPSM_OK) rr = redone(P.padR1, P.dirtyR1, P.QR, &stats->redone_r_segments);
    if (rr == MPSM_OK) rr = redone(P.padR2, P.dirtyR2, P.NB1, &stats->redone_r_segments);
    if (rr != MPSM_OK) return rr;
    if (r.truncated) return MPSM_ECAPACITY;
  }
  return MPSM_OK;
}

}  // namespace

extern "C" {

mpsm_status mpsm_join(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS, uint64_t* d_out_count,
                      uint64_t* d_out_checksum, mpsm_pair* d_pairs, uint64_t pairs_capacity, const mpsm_config* cfg,
                      void* d_workspace, uint64_t workspace_bytes, void* stream, mpsm_stats* stats) {
  return join_impl(d_R, nR, d_S, nS, d_out_count, d_out_checksum, d_pairs, pairs_capacity, cfg, d_workspace,
                   workspace_bytes, stream, stats, nullptr, 0);
}

mpsm_status mpsm_join_events(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS,
                             uint64_t* d_out_count, uint64_t* d_out_checksum, mpsm_pair* d_pairs,
                             uint64_t pairs_capacity, const mpsm_config* cfg, void* d_workspace,
                             uint64_t workspace_bytes, void* stream, void** events, uint32_t n_events) {
  if (n_events && !events) return MPSM_EINVAL;
  return join_impl(d_R, nR, d_S, nS, d_out_count, d_out_checksum, d_pairs, pairs_capacity, cfg, d_workspace,
                   workspace_bytes, stream, nullptr, events, n_events);
}

}  // extern "C"

namespace {

// Options the join with S in host memory supports: S keeps its role (it is
// the relation outside device memory) and R's splitters need no S runs.
bool host_runs_config_ok(const mpsm_config* cfg) {
  return config_valid(cfg) && cfg->role != MPSM_ROLE_SWAP &&
         (cfg->splitter == MPSM_SPLIT_SAMPLED || cfg->splitter == MPSM_SPLIT_LEARNED);
}

}  // namespace

extern "C" {

uint64_t mpsm_join_host_runs_workspace_bytes(uint64_t nR, uint64_t nS, const mpsm_config* cfg, uint64_t chunk_tuples) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!host_runs_config_ok(cfg) || chunk_tuples == 0) return 0;
  Plan P;
  if (!make_plan(nR, nS, cfg, &P, chunk_tuples)) return 0;
  return P.total;
}

mpsm_status mpsm_join_host_runs(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* h_S, uint64_t nS,
                                mpsm_tuple* h_runs, uint64_t* d_out_count, uint64_t* d_out_checksum,
                                const mpsm_config* cfg, uint64_t chunk_tuples, void* d_workspace,
                                uint64_t workspace_bytes, void* stream) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!host_runs_config_ok(cfg) || chunk_tuples == 0) return MPSM_EINVAL;
  if (nS && !h_S) return MPSM_EINVAL;
  if (((uintptr_t)h_S & 15) || ((uintptr_t)h_runs & 15)) return MPSM_EINVAL;
  HostS hs;
  hs.S_host = reinterpret_cast<const tup_t*>(h_S);
  hs.runs_host = reinterpret_cast<tup_t*>(h_runs);
  hs.S_dev = nullptr;
  hs.chunk = chunk_tuples;
  hs.spilled = false;
  hs.runs_dev = nullptr;
  if (nS) {
    // both buffers must be pinned host memory the device can address
    void* p = nullptr;
    void* q = nullptr;
    if (hipHostGetDevicePointer(&p, const_cast<mpsm_tuple*>(h_S), 0) != hipSuccess || !p ||
        (h_runs && (hipHostGetDevicePointer(&q, h_runs, 0) != hipSuccess || !q))) {
      (void)hipGetLastError();   // the failed lookup is the caller's error, not a later call's
      return MPSM_EINVAL;
    }
    hs.S_dev = static_cast<const tup_t*>(p);
  }
  return join_impl(d_R, nR, h_S, nS, d_out_count, d_out_checksum, nullptr, 0, cfg, d_workspace, workspace_bytes,
                   stream, nullptr, nullptr, 0, false, &hs);
}

uint64_t mpsm_join_spilled_runs_workspace_bytes(uint64_t nR, uint64_t nS, const mpsm_config* cfg) {
  // the plan of the host-memory join with the smallest chunk (one run)
  return mpsm_join_host_runs_workspace_bytes(nR, nS, cfg, 1);
}

mpsm_status mpsm_join_spilled_runs(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* h_runs, uint64_t nS,
                                   uint64_t* d_out_count, uint64_t* d_out_checksum, const mpsm_config* cfg,
                                   void* d_workspace, uint64_t workspace_bytes, void* stream) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!host_runs_config_ok(cfg)) return MPSM_EINVAL;
  if ((nS && !h_runs) || ((uintptr_t)h_runs & 15)) return MPSM_EINVAL;
  HostS hs;
  hs.S_host = nullptr;
  hs.runs_host = nullptr;
  hs.chunk = 1;
  hs.spilled = true;
  hs.S_dev = nullptr;
  hs.runs_dev = nullptr;
  if (nS) {
    void* p = nullptr;
    if (hipHostGetDevicePointer(&p, const_cast<mpsm_tuple*>(h_runs), 0) != hipSuccess || !p) {
      (void)hipGetLastError();   // the failed lookup is the caller's error, not a later call's
      return MPSM_EINVAL;
    }
    hs.runs_dev = static_cast<const tup_t*>(p);
    hs.S_dev = hs.runs_dev;   // the learned search's sample: any positions of S's tuples
  }
  return join_impl(d_R, nR, h_runs, nS, d_out_count, d_out_checksum, nullptr, 0, cfg, d_workspace, workspace_bytes,
                   stream, nullptr, nullptr, 0, false, &hs);
}

}  // extern "C"

namespace {

// Workspace of mpsm_join_noalloc: a fixed array in the library's own device
// memory, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in for the symbol): the device address of each GPU's copy is looked
// up once, with that GPU current, and kept here.
static __device__ __align__(256) unsigned char scratch[MPSM_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[SIDE_MAX_DEVICES];

mpsm_status scratch_for_current_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SIDE_MAX_DEVICES) return MPSM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPSM_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MPSM_OK;
}

}  // namespace

extern "C" {

mpsm_status mpsm_join_noalloc(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS,
                              uint64_t* d_out_count, uint64_t* d_out_checksum, mpsm_pair* d_pairs,
                              uint64_t pairs_capacity, const mpsm_config* cfg, void* stream) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!config_valid(cfg)) return MPSM_EINVAL;
  Plan P;
  if (!make_plan(nR, nS, cfg, &P)) return MPSM_EINVAL;
  // sizes beyond the array are refused before any device call
  if (P.total > (uint64_t)MPSM_NOALLOC_SCRATCH_BYTES) return MPSM_ENOMEM;
  void* ws = nullptr;
  const mpsm_status rs = scratch_for_current_device(&ws);
  if (rs != MPSM_OK) return rs;
  // one stream (no side stream of the library's own) and no statistics
  // (which would create events): nothing here allocates
  return join_impl(d_R, nR, d_S, nS, d_out_count, d_out_checksum, d_pairs, pairs_capacity, cfg, ws,
                   (uint64_t)MPSM_NOALLOC_SCRATCH_BYTES, stream, nullptr, nullptr, 0, true);
}

uint32_t mpsm_marker_count(void) { return kNumMarkers; }

const char* mpsm_marker_name(uint32_t i) { return i < kNumMarkers ? kMarkers[i] : nullptr; }

mpsm_status mpsm_events_create(void** events, uint32_t n) {
  if (n && !events) return MPSM_EINVAL;
  for (uint32_t i = 0; i < n; i++) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return MPSM_EHIP;
    events[i] = e;
  }
  return MPSM_OK;
}

void mpsm_events_destroy(void** events, uint32_t n) {
  for (uint32_t i = 0; events && i < n; i++)
    if (events[i]) { (void)hipEventDestroy((hipEvent_t)events[i]); events[i] = nullptr; }
}

mpsm_status mpsm_events_elapsed(void* start, void* stop, float* ms) {
  if (!start || !stop || !ms) return MPSM_EINVAL;
  return hipEventElapsedTime(ms, (hipEvent_t)start, (hipEvent_t)stop) == hipSuccess ? MPSM_OK : MPSM_EHIP;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

// Host layer over mpsm_join_batch: a copy of the descriptors (uploaded into
// the workspace), the current tuning and, once used, a captured hipGraph.
struct mpsm_batch {
  std::vector<mpsm_join_desc> d;
  mpsm_config cfg;
  mpsm_batch_shape shape;                // the batch's own sums
  uint32_t L = 0, BT = 0, JCH = 0;       // current tuning
  uint64_t ws_max = 0;                   // workspace serving every candidate tuning
  void* host = nullptr;                  // pinned staging of the descriptors
  void* uploaded_to = nullptr;           // workspace that holds them
  hipGraphExec_t graph = nullptr;
  void* graph_ws = nullptr;
  hipStream_t capture = nullptr;         // private stream the graph is captured on
};

namespace {

constexpr uint32_t kBatchL[] = {1u << 16, 1u << 18, 1u << 20};
constexpr uint32_t kBatchBT[] = {2048u, 4096u};
constexpr uint32_t kBatchJCH[] = {16384u, 65536u};
constexpr uint32_t BATCH_N_MAX = 1u << 20;        // joins per batch
constexpr uint32_t BATCH_SORT_GRID = 1u << 16;    // workgroups of the batch's bucket sorts (they loop)

// Sizes of a batch launch, from the number of joins and bounds on their
// sizes only (the descriptors are in device memory): every launch grid and
// every table is sized for the largest batch of this shape class.
struct BatchPlan {
  uint32_t n, L, BT, JCH, W;
  uint64_t maxR, maxS, maxNS;
  uint32_t NBs, OSs, OSr, Qmax, Gs, Gr, nbRmax;
  uint32_t tilesS, tilesR, Pmax;
  uint64_t cntS, cntR, ocap, item_cap;
  // workspace offsets
  uint64_t status, descs, T, U, Rp, Rs, cS, cR, bsum, bsumR, segS, segR, srcS, srcR, J, wave, splS, splR, bstS, bstR;
  uint64_t bndS, bndR, bigS, midS, redoS, midR, redoR, redoR2, bigR, ctr, bkey, Pc, pstart, plen, pkey, pjoin, ridx;
  uint64_t o, items, item_pre, tstart, ototal, span;
  // passes without a histogram (as for one join): S's runs, R's segments
  int padS, padR;
  uint64_t capS, rstS, fillS, bsrcS, dirtyS, capR, rstR, fillR, bsrcR, dirtyR;
  uint64_t total;
};

bool batch_tuning_valid(uint32_t L, uint32_t BT, uint32_t JCH) {
  return L >= (1u << 16) && L <= (1u << 22) && (L & (L - 1)) == 0 && BT >= 1024 && BT <= 4096 && JCH >= 4096 &&
         JCH <= (uint32_t)JOIN_CHUNK_MAX;
}

bool batch_cfg_supported(const mpsm_config* cfg) {
  return cfg->splitter == MPSM_SPLIT_SAMPLED && cfg->search != MPSM_SEARCH_LEARNED && !cfg->want_max &&
         cfg->role != MPSM_ROLE_SWAP;
}

// Waves: as configured, else 4 for 32 joins or more, 2 for 8 or more;
// never more than the joins, and one when there are too many joins to rank.
uint32_t batch_waves(uint32_t n, const mpsm_config& cfg) {
  uint32_t W = cfg.waves ? cfg.waves : (n >= 32 ? 4u : (n >= 8 ? 2u : 1u));
  if (W > n) W = n;
  if (n > BATCH_RANK_MAX || W < 1) W = 1;
  return W;
}

// Default run length: the shortest of 2^16 .. 2^22 that keeps every join
// within the run limit.
uint32_t batch_default_L(uint64_t maxNS) {
  uint32_t L = 1u << 16;
  while (L < (1u << 22) && cdiv(maxNS, L) > (uint64_t)JOIN_QMAX) L <<= 1;
  return L;
}

bool make_batch_plan(uint32_t n, const mpsm_batch_shape& sh, const mpsm_config& cfg, uint32_t L, uint32_t BT,
                     uint32_t JCH, BatchPlan* P) {
  memset(P, 0, sizeof(*P));
  if (n == 0 || n > BATCH_N_MAX || !batch_tuning_valid(L, BT, JCH)) return false;
  P->n = n; P->L = L; P->BT = BT; P->JCH = JCH;
  P->maxR = sh.max_sum_nR; P->maxS = sh.max_sum_nS;
  P->maxNS = sh.max_nS && sh.max_nS < sh.max_sum_nS ? sh.max_nS : sh.max_sum_nS;
  if (P->maxR >= (1ull << 32) || P->maxS >= (1ull << 32)) return false;
  if (cdiv(P->maxNS, L) > (uint64_t)JOIN_QMAX) return false;
  P->W = batch_waves(n, cfg);
  const uint32_t BTs = BT < S_BUCKET_MEAN ? BT : S_BUCKET_MEAN;
  P->NBs = (uint32_t)cdiv(L, BTs);
  if (P->NBs > (uint32_t)MAX_NB) P->NBs = MAX_NB;
  const uint32_t OSreq = cfg.oversample ? cfg.oversample : 32u;
  auto os_for = [&](uint32_t NB) { return NB > 1 ? (SMP_CAP / NB < OSreq ? SMP_CAP / NB : OSreq) : 1u; };
  P->OSs = os_for(P->NBs);
  P->OSr = os_for(MAX_NB);
  // S: every join adds at most one partial run, every run one partial tile
  uint64_t Q = P->maxS / L + n;
  if (Q > P->maxS) Q = P->maxS;
  if (Q < 1) Q = 1;
  P->Qmax = (uint32_t)Q;
  P->Gs = P->Qmax * P->NBs;
  P->tilesS = (uint32_t)(P->maxS / HIST_TILE + P->Qmax);
  P->cntS = (uint64_t)P->tilesS * P->NBs;
  // R: one segment per join, ceil(nR / BT) buckets (1 for an empty segment)
  uint64_t Gr = P->maxR / BT + n;
  if (Gr > (uint64_t)n * MAX_NB) Gr = (uint64_t)n * MAX_NB;
  P->Gr = (uint32_t)Gr;
  P->nbRmax = (uint32_t)(P->maxR / BT + 1 < (uint64_t)MAX_NB ? P->maxR / BT + 1 : MAX_NB);
  P->tilesR = (uint32_t)(P->maxR / HIST_TILE + n);
  P->cntR = (uint64_t)P->nbRmax * P->tilesR;
  if (P->cntR < 1) P->cntR = 1;
  P->Pmax = P->Gr;
  P->ocap = ((uint64_t)P->nbRmax + 1) * P->Qmax;
  P->item_cap = P->maxS / JCH + P->Pmax + 2;
  const uint32_t ipr = (uint32_t)cdiv(L, IDX_STRIDE);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) { uint64_t o = off; off += (bytes + 255) & ~255ull; return o; };
  const uint64_t ts = sizeof(tup_t);
  // every join's runs and R segment are segments of the batch's passes, so
  // the claims spread over many counters
  P->padS = P->maxS >= (1u << 22) && pad_area(P->maxS) < (1ull << 32);
  P->padR = P->maxR >= (1u << 22) && pad_area(P->maxR) < (1ull << 32);
  P->status = take(8);   // offset 0: the batch status word
  P->descs = take((uint64_t)n * sizeof(mpsm_join_desc));
  P->T = take((P->padS ? pad_area(P->maxS) : P->maxS) * ts);
  P->U = take(P->maxS * ts);
  P->Rp = take((P->padR ? pad_area(P->maxR) : P->maxR) * ts);
  P->Rs = take(P->maxR * ts);
  P->cS = take(P->cntS * 4 + 4);
  P->cR = take(P->cntR * 4);
  uint64_t maxscan = P->cntS > P->cntR ? P->cntS : P->cntR;
  if (P->item_cap > maxscan) maxscan = P->item_cap;
  P->bsum = take((cdiv(maxscan, SCAN_BLOCK) + 1) * 4);
  P->bsumR = take((cdiv(P->cntR, SCAN_BLOCK) + 1) * 4);   // R's scan, beside S's phase
  P->segS = take(6ull * (P->Qmax + 1) * 4);
  P->segR = take(6ull * (n + 1) * 4);
  P->srcS = take((uint64_t)P->Qmax * 8);
  P->srcR = take((uint64_t)n * 8);
  P->J = take((uint64_t)n * sizeof(BatchJoin));
  P->wave = take((uint64_t)n * 4);
  P->splS = take((uint64_t)P->Qmax * P->NBs * 8);
  P->splR = take((uint64_t)n * MAX_NB * 8);
  P->bstS = take(((uint64_t)P->Gs + 1) * 4);
  P->bstR = take(((uint64_t)P->Gr + 1) * 4);
  P->bndS = take((uint64_t)P->Gs * 16);
  P->bndR = take((uint64_t)P->Gr * 16);
  P->bigS = take((uint64_t)P->Gs * 4);
  P->midS = take((uint64_t)P->Gs * 4);
  P->redoS = take((uint64_t)P->Gs * 4);
  P->midR = take((uint64_t)P->Gr * 4);
  P->redoR = take((uint64_t)P->Gr * 4);
  P->redoR2 = take((uint64_t)P->Gr * 4);
  P->bigR = take((uint64_t)P->Gr * 4);
  P->ctr = take(16 * 8);
  P->bkey = take((uint64_t)P->Gr * 8);
  P->Pc = take(4);
  P->pstart = take((uint64_t)P->Pmax * 4);
  P->plen = take((uint64_t)P->Pmax * 4);
  P->pkey = take((uint64_t)P->Pmax * 8);
  P->pjoin = take((uint64_t)P->Pmax * 4);
  P->ridx = take((uint64_t)P->Qmax * ipr * 8);
  P->o = take(P->ocap * 4);
  P->items = take(((uint64_t)P->Pmax + 2) * 4);
  P->item_pre = take(((uint64_t)P->Pmax + 2) * 4);
  P->tstart = take(8);
  P->ototal = take(8);
  P->span = take((uint64_t)P->Pmax + 2);
  if (P->padS) {
    P->capS = take((uint64_t)P->Gs * 4);
    P->rstS = take((uint64_t)P->Gs * 4);
    P->fillS = take((uint64_t)P->Gs * 4);
    P->bsrcS = take(((uint64_t)P->Gs + 1) * 4);
    P->dirtyS = take((uint64_t)P->Qmax * 4);
  }
  if (P->padR) {
    P->capR = take((uint64_t)P->Gr * 4);
    P->rstR = take((uint64_t)P->Gr * 4);
    P->fillR = take((uint64_t)P->Gr * 4);
    P->bsrcR = take(((uint64_t)P->Gr + 1) * 4);
    P->dirtyR = take((uint64_t)n * 4);
  }
  P->total = off;
  return true;
}

// The run-length, bucket and work-item tuning of a config (0: defaults).
void batch_tuning_of(const mpsm_config& cfg, uint64_t maxNS, uint32_t* L, uint32_t* BT, uint32_t* JCH) {
  *L = cfg.log2_run_len ? (1u << cfg.log2_run_len) : batch_default_L(maxNS);
  *BT = cfg.bucket_target ? cfg.bucket_target : 4096u;
  *JCH = cfg.join_chunk ? cfg.join_chunk : 65536u;
}

// The launch sequence of a batch whose descriptors are at d_descs (device):
// the descriptor check and wave assignment, then per wave its tables and
// every phase of the method for the wave's joins.
mpsm_status batch_enqueue(const mpsm_join_desc* d_descs, const BatchPlan& P, uint64_t seed, int search, char* ws,
                          hipStream_t st) {
  tup_t* T = reinterpret_cast<tup_t*>(ws + P.T);
  tup_t* U = reinterpret_cast<tup_t*>(ws + P.U);
  tup_t* Rp = reinterpret_cast<tup_t*>(ws + P.Rp);
  tup_t* Rs = reinterpret_cast<tup_t*>(ws + P.Rs);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(ws + P.bsum);
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(ws + P.ctr);
  BatchJoin* J = reinterpret_cast<BatchJoin*>(ws + P.J);
  uint32_t* wave = reinterpret_cast<uint32_t*>(ws + P.wave);
  unsigned long long* tstart = reinterpret_cast<unsigned long long*>(ws + P.tstart);
  unsigned long long* ototal = reinterpret_cast<unsigned long long*>(ws + P.ototal);
  // R's phase runs on the side stream beside S's run sort, from the point
  // where S's tuples are scattered (as for a single join); under capture
  // the fork and join make them two branches of the graph
  SideStream* side = nullptr;
  mpsm_status rc = side_stream(&side);
  if (rc != MPSM_OK) return rc;
  Marker mk{nullptr, 0, st};
  k_batch_check<<<1, BPLAN_NT, 0, st>>>(d_descs, P.n, P.W, P.maxR, P.maxS, P.maxNS, wave,
                                        reinterpret_cast<uint32_t*>(ws + P.status), tstart);
  LAUNCH_CHECK();
  const Seg sgS = seg_at(ws, P.segS, P.Qmax);
  const Seg sgR = seg_at(ws, P.segR, P.n);
  const tup_t** srcS = reinterpret_cast<const tup_t**>(ws + P.srcS);
  const tup_t** srcR = reinterpret_cast<const tup_t**>(ws + P.srcR);
  const uint32_t sort_grid_s = P.Gs < BATCH_SORT_GRID ? P.Gs : BATCH_SORT_GRID;
  const uint32_t sort_grid_r = P.Gr < BATCH_SORT_GRID ? P.Gr : BATCH_SORT_GRID;
  for (uint32_t w = 0; w < P.W; w++) {
    k_batch_plan<<<1, BPLAN_NT, 0, st>>>(d_descs, P.n, wave, w, P.L, P.BT, P.Qmax, J, sgS.start, sgS.len, srcS,
                                         sgR.start, sgR.len, srcR, reinterpret_cast<uint32_t*>(ctr), 32);
    LAUNCH_CHECK();
    // phase 1: S runs of the wave's joins
    Level LS = make_level(ws, P.segS, P.Qmax, P.NBs, 0, P.OSs, P.tilesS, seed ^ TAG_S, P.splS, P.cS, P.cntS, P.bstS,
                          P.bndS, P.Gs);
    // regions of a pass without a histogram; `any` is a word of ctr, which
    // k_batch_plan zeroes for every wave
    auto regions = [&](Level& Lv, uint64_t cap, uint64_t rst, uint64_t fill, uint64_t dirty, uint64_t bsrc,
                       uint32_t any_word) {
      Lv.rg.cap = reinterpret_cast<uint32_t*>(ws + cap);
      Lv.rg.start = reinterpret_cast<uint32_t*>(ws + rst);
      Lv.rg.fill = reinterpret_cast<uint32_t*>(ws + fill);
      Lv.rg.dirty = reinterpret_cast<uint32_t*>(ws + dirty);
      Lv.rg.any = reinterpret_cast<uint32_t*>(ctr + any_word);
      Lv.bsrc = reinterpret_cast<uint32_t*>(ws + bsrc);
    };
    if (P.padS) regions(LS, P.capS, P.rstS, P.fillS, P.dirtyS, P.bsrcS, 7);
    rc = bucket_pass(nullptr, T, 0, LS, bsum, st, mk, 0, srcS);
    if (rc != MPSM_OK) return rc;
    HIP_TRY(hipEventRecord(side->fork, st));
    HIP_TRY(hipStreamWaitEvent(side->st, side->fork, 0));
    SortOut soS;
    soS.run_idx = reinterpret_cast<uint64_t*>(ws + P.ridx);
    soS.run_start = LS.seg.start;
    soS.idx_stride = IDX_STRIDE;
    soS.idx_shift = __builtin_ctz(IDX_STRIDE);
    soS.idx_per_run = (uint32_t)cdiv(P.L, IDX_STRIDE);
    soS.NB = P.NBs;
    soS.bkey = nullptr;
    uint32_t* midS = reinterpret_cast<uint32_t*>(ws + P.midS);
    uint32_t* bigS = reinterpret_cast<uint32_t*>(ws + P.bigS);
    uint32_t* redoS = reinterpret_cast<uint32_t*>(ws + P.redoS);
    k_bucket_sort_cs<BS_NT, BS_IPT, BS_M, 8, false, false><<<sort_grid_s, BS_NT, 0, st>>>(
        T, U, LS.bstart, LS.bsrc, LS.blo, LS.bhi, LS.Gcount(), nullptr, nullptr, midS, ctr + 2, redoS, ctr + 3, soS);
    LAUNCH_CHECK();
    k_bucket_sort_cs<BL_NT, BL_IPT, BL_M, 1, true, false><<<g_num_cus, BL_NT, 0, st>>>(
        T, U, LS.bstart, LS.bsrc, LS.blo, LS.bhi, LS.Gcount(), midS, ctr + 2, bigS, ctr + 0, redoS, ctr + 3, soS);
    LAUNCH_CHECK();
    k_bucket_sort_lsd<<<g_num_cus, LSD_NT, 0, st>>>(T, U, LS.bstart, LS.bsrc, redoS, ctr + 3, bigS, ctr + 0, soS);
    LAUNCH_CHECK();
    k_big_sort<<<g_num_cus, BIG_NT, 0, st>>>(T, U, LS.bstart, LS.bsrc, bigS, ctr + 0, soS);
    LAUNCH_CHECK();
    // phases 2 and 3: one R segment per join, bucket counts from its size
    Level LR = make_level(ws, P.segR, P.n, MAX_NB, P.BT, P.OSr, P.tilesR, seed ^ TAG_R1, P.splR, P.cR, P.cntR,
                          P.bstR, P.bndR, P.Gr);
    const hipStream_t rst = side->st;
    Marker mkR{nullptr, 0, rst};
    if (P.padR) regions(LR, P.capR, P.rstR, P.fillR, P.dirtyR, P.bsrcR, 8);
    rc = bucket_pass(nullptr, Rp, 0, LR, reinterpret_cast<uint32_t*>(ws + P.bsumR), rst, mkR, 0, srcR);
    if (rc != MPSM_OK) return rc;
    SortOut soR;
    soR.run_idx = nullptr;
    soR.run_start = nullptr;
    soR.idx_stride = 1;
    soR.idx_shift = 0;
    soR.idx_per_run = 0;
    soR.NB = 1;
    soR.bkey = reinterpret_cast<uint64_t*>(ws + P.bkey);
    uint32_t* midR = reinterpret_cast<uint32_t*>(ws + P.midR);
    uint32_t* redoR = reinterpret_cast<uint32_t*>(ws + P.redoR);
    uint32_t* redoR2 = reinterpret_cast<uint32_t*>(ws + P.redoR2);
    uint32_t* bigR = reinterpret_cast<uint32_t*>(ws + P.bigR);
    k_bucket_sort_cs<BS_NT, BS_IPT, BS_M, 8, false, false><<<sort_grid_r, BS_NT, 0, rst>>>(
        Rp, Rs, LR.bstart, LR.bsrc, LR.blo, LR.bhi, LR.Gcount(), nullptr, nullptr, midR, ctr + 6, redoR, ctr + 4, soR);
    LAUNCH_CHECK();
    k_bucket_sort_cs<BL_NT, BL_IPT, BL_M, 1, true, false><<<g_num_cus, BL_NT, 0, rst>>>(
        Rp, Rs, LR.bstart, LR.bsrc, LR.blo, LR.bhi, LR.Gcount(), midR, ctr + 6, bigR, ctr + 1, redoR, ctr + 4, soR);
    LAUNCH_CHECK();
    k_bucket_sort_cs<BL_NT, BL_IPT, BL_M, 1, true, true><<<g_num_cus, BL_NT, 0, rst>>>(
        Rp, Rs, LR.bstart, LR.bsrc, LR.blo, LR.bhi, LR.Gcount(), redoR, ctr + 4, bigR, ctr + 1, redoR2, ctr + 5, soR);
    LAUNCH_CHECK();
    k_bucket_sort_lsd<<<g_num_cus, LSD_NT, 0, rst>>>(Rp, Rs, LR.bstart, LR.bsrc, redoR2, ctr + 5, bigR, ctr + 1, soR);
    LAUNCH_CHECK();
    k_big_sort<<<g_num_cus, BIG_NT, 0, rst>>>(Rp, Rs, LR.bstart, LR.bsrc, bigR, ctr + 1, soR);
    LAUNCH_CHECK();
    // the rest needs R's partitions
    HIP_TRY(hipEventRecord(side->done, rst));
    HIP_TRY(hipStreamWaitEvent(st, side->done, 0));
    uint32_t* Pc = reinterpret_cast<uint32_t*>(ws + P.Pc);
    uint32_t* pstart = reinterpret_cast<uint32_t*>(ws + P.pstart);
    uint32_t* plen = reinterpret_cast<uint32_t*>(ws + P.plen);
    uint64_t* pkey = reinterpret_cast<uint64_t*>(ws + P.pkey);
    uint32_t* pjoin = reinterpret_cast<uint32_t*>(ws + P.pjoin);
    k_partitions_batch<<<1, 1024, 0, st>>>(LR.bstart, soR.bkey, LR.Gcount(), J, P.n, Pc, pstart, plen, pkey, pjoin);
    LAUNCH_CHECK();
    k_batch_blocks<<<1, 64, 0, st>>>(J, P.n, ototal);
    LAUNCH_CHECK();
    uint8_t* span = reinterpret_cast<uint8_t*>(ws + P.span);
    k_join_units_batch<<<(uint32_t)cdiv(P.Pmax, 256), 256, 0, st>>>(Pc, plen, pjoin, P.Pmax, span);
    LAUNCH_CHECK();
    // phase 4
    uint32_t* o = reinterpret_cast<uint32_t*>(ws + P.o);
    const int mode = search == MPSM_SEARCH_BINARY ? SEARCH_BINARY
                   : search == MPSM_SEARCH_INTERP ? SEARCH_INTERP : SEARCH_INDEX;
    k_search_batch<<<(uint32_t)cdiv(P.ocap, 256), 256, 0, st>>>(U, LS.seg.start, LS.seg.len,
                                                               reinterpret_cast<uint64_t*>(ws + P.ridx), IDX_STRIDE,
                                                               soS.idx_per_run, J, P.n, pkey, o, ototal, mode, span);
    LAUNCH_CHECK();
    uint32_t* items = reinterpret_cast<uint32_t*>(ws + P.items);
    uint32_t* item_pre = reinterpret_cast<uint32_t*>(ws + P.item_pre);
    k_join_items_batch<<<(uint32_t)cdiv(P.Pmax + 2, 256), 256, 0, st>>>(Pc, pjoin, J, o, LS.seg.len, P.Pmax, P.JCH,
                                                                        span, items);
    LAUNCH_CHECK();
    rc = scan_u32(items, item_pre, (uint64_t)P.Pmax + 2, bsum, st);
    if (rc != MPSM_OK) return rc;
    JoinArgs A;
    memset(&A, 0, sizeof(A));
    A.Rs = Rs;
    A.U = U;
    A.run_start = LS.seg.start;
    A.run_len = LS.seg.len;
    A.Q = 0;
    A.Pcount = Pc;
    A.pstart = pstart;
    A.plen = plen;
    A.o = o;
    A.item_pre = item_pre;
    A.Pmax = P.Pmax;
    A.JCH = P.JCH;
    A.res = nullptr;
    A.J = J;
    A.pjoin = pjoin;
    A.span = span;
    k_join<0, VAL_HR, true><<<g_num_cus, JOIN_NT, 0, st>>>(A);
    LAUNCH_CHECK();
    k_finalize_batch<<<(uint32_t)cdiv(P.n, 256), 256, 0, st>>>(J, P.n, tstart);
    LAUNCH_CHECK();
  }
  return MPSM_OK;
}

void ensure_num_cus() {
  if (g_num_cus) return;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) ==
                                              hipSuccess)
    g_num_cus = ncu > 0 ? ncu : 256;
  else
    g_num_cus = 256;
}

bool batch_shape_valid(const mpsm_batch_shape* sh) {
  return sh && sh->max_sum_nR < (1ull << 32) && sh->max_sum_nS < (1ull << 32);
}

void batch_drop_graph(mpsm_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_ws = nullptr;
}

mpsm_status batch_set(mpsm_batch* b, uint32_t L, uint32_t BT, uint32_t JCH) {
  BatchPlan P;
  if (!make_batch_plan((uint32_t)b->d.size(), b->shape, b->cfg, L, BT, JCH, &P)) return MPSM_EUNSUPPORTED;
  b->L = L; b->BT = BT; b->JCH = JCH;
  batch_drop_graph(b);
  return MPSM_OK;
}

mpsm_status batch_run(mpsm_batch* b, void* d_ws, uint64_t bytes, void* stream, int use_graph) {
  if (!b || !d_ws || ((uintptr_t)d_ws & 255)) return MPSM_EINVAL;
  BatchPlan P;
  if (!make_batch_plan((uint32_t)b->d.size(), b->shape, b->cfg, b->L, b->BT, b->JCH, &P)) return MPSM_EUNSUPPORTED;
  if (bytes < P.total) return MPSM_ENOMEM;
  ensure_num_cus();
  hipStream_t st = (hipStream_t)stream;
  char* ws = static_cast<char*>(d_ws);
  // the descriptors sit at the same workspace offset under every tuning
  const uint64_t dbytes = b->d.size() * sizeof(mpsm_join_desc);
  if (b->uploaded_to != d_ws) {
    if (!b->host) HIP_TRY(hipHostMalloc(&b->host, dbytes, hipHostMallocDefault));
    memcpy(b->host, b->d.data(), dbytes);
    HIP_TRY(hipMemcpyAsync(ws + P.descs, b->host, dbytes, hipMemcpyHostToDevice, st));
    b->uploaded_to = d_ws;
  }
  const mpsm_join_desc* d_descs = reinterpret_cast<const mpsm_join_desc*>(ws + P.descs);
  if (!use_graph) return batch_enqueue(d_descs, P, b->cfg.seed, b->cfg.search, ws, st);
  if (!b->graph || b->graph_ws != d_ws) {
    // captured on a stream of the batch's own (the caller's may be the
    // legacy default stream, which cannot be captured), launched on the
    // caller's; the descriptors reach the workspace first
    batch_drop_graph(b);
    if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamSynchronize(st));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    const mpsm_status rc = batch_enqueue(d_descs, P, b->cfg.seed, b->cfg.search, ws, b->capture);
    const hipError_t ec = hipStreamEndCapture(b->capture, &g);
    if (rc != MPSM_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (ec != hipSuccess || !g) return MPSM_EHIP;
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return MPSM_EHIP;
    b->graph = ex;
    b->graph_ws = d_ws;
  }
  HIP_TRY(hipGraphLaunch(b->graph, st));
  return MPSM_OK;
}

// Cache key: the batch's shape in coarse (log2) terms.
std::string batch_signature(const mpsm_batch* b) {
  uint64_t sR = 0, sS = 0, mR = 0, mS = 0;
  for (const mpsm_join_desc& j : b->d) {
    sR += j.nR; sS += j.nS;
    if (j.nR > mR) mR = j.nR;
    if (j.nS > mS) mS = j.nS;
  }
  auto lg = [](uint64_t x) { int k = 0; while (x > 1) { x >>= 1; k++; } return k; };
  char buf[160];
  snprintf(buf, sizeof(buf), "gfx950:n%u:R%d:S%d:maxR%d:maxS%d:search%d:w%u", (unsigned)b->d.size(), lg(sR),
           lg(sS), lg(mR), lg(mS), (int)b->cfg.search, batch_waves((uint32_t)b->d.size(), b->cfg));
  return buf;
}

bool cache_lookup(const char* path, const std::string& sig, uint32_t* L, uint32_t* BT, uint32_t* JCH) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char key[256];
    unsigned lg = 0, bt = 0, jc = 0;
    float ms = 0.f;
    if (sscanf(line, "%255s %u %u %u %f", key, &lg, &bt, &jc, &ms) != 5) continue;
    if (sig != key || lg > 31) continue;
    const uint32_t l = 1u << lg;
    if (!batch_tuning_valid(l, bt, jc)) continue;
    *L = l; *BT = bt; *JCH = jc;
    found = true;   // the last valid entry wins
  }
  fclose(f);
  return found;
}

}  // namespace

extern "C" {

uint64_t mpsm_join_batch_workspace_bytes(uint32_t n, const mpsm_batch_shape* shape, const mpsm_config* cfg) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!config_valid(cfg) || !batch_cfg_supported(cfg) || !batch_shape_valid(shape)) return 0;
  uint32_t L, BT, JCH;
  batch_tuning_of(*cfg, shape->max_nS ? shape->max_nS : shape->max_sum_nS, &L, &BT, &JCH);
  BatchPlan P;
  if (!make_batch_plan(n, *shape, *cfg, L, BT, JCH, &P)) return 0;
  return P.total;
}

mpsm_status mpsm_join_batch(const mpsm_join_desc* d_descs, uint32_t n, const mpsm_batch_shape* shape,
                            const mpsm_config* cfg, void* d_workspace, uint64_t workspace_bytes, void* stream) {
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!config_valid(cfg) || !batch_shape_valid(shape)) return MPSM_EINVAL;
  if (!batch_cfg_supported(cfg)) return MPSM_EUNSUPPORTED;
  if (!d_descs || ((uintptr_t)d_descs & 7) || !d_workspace || ((uintptr_t)d_workspace & 255)) return MPSM_EINVAL;
  uint32_t L, BT, JCH;
  batch_tuning_of(*cfg, shape->max_nS ? shape->max_nS : shape->max_sum_nS, &L, &BT, &JCH);
  BatchPlan P;
  if (!make_batch_plan(n, *shape, *cfg, L, BT, JCH, &P)) return MPSM_EINVAL;
  if (workspace_bytes < P.total) return MPSM_ENOMEM;
  ensure_num_cus();
  return batch_enqueue(d_descs, P, cfg->seed, cfg->search, static_cast<char*>(d_workspace), (hipStream_t)stream);
}

mpsm_status mpsm_batch_create(const mpsm_join_desc* descs, uint32_t n, const mpsm_config* cfg, mpsm_batch** out) {
  if (!out) return MPSM_EINVAL;
  *out = nullptr;
  if (!descs || n == 0 || n > BATCH_N_MAX) return MPSM_EINVAL;
  mpsm_config def;
  if (!cfg) { mpsm_config_default(&def); cfg = &def; }
  if (!config_valid(cfg)) return MPSM_EINVAL;
  if (!batch_cfg_supported(cfg)) return MPSM_EUNSUPPORTED;
  mpsm_batch_shape sh;
  memset(&sh, 0, sizeof(sh));
  for (uint32_t i = 0; i < n; i++) {
    const mpsm_join_desc& j = descs[i];
    if ((j.nR && !j.d_R) || (j.nS && !j.d_S) || !j.d_out_count || !j.d_out_checksum) return MPSM_EINVAL;
    if (((uintptr_t)j.d_R & 15) || ((uintptr_t)j.d_S & 15) || ((uintptr_t)j.d_out_count & 7) ||
        ((uintptr_t)j.d_out_checksum & 7) || ((uintptr_t)j.d_out_times & 7))
      return MPSM_EINVAL;
    if (j.nR >= (1ull << 32) || j.nS >= (1ull << 32)) return MPSM_EINVAL;
    if (j.nR && j.nS) {
      sh.max_sum_nR += j.nR;
      sh.max_sum_nS += j.nS;
      if (j.nS > sh.max_nS) sh.max_nS = j.nS;
    }
  }
  if (!batch_shape_valid(&sh)) return MPSM_EINVAL;
  mpsm_batch* b = new mpsm_batch();
  b->d.assign(descs, descs + n);
  b->cfg = *cfg;
  b->shape = sh;
  // initial tuning: the config's values, else a run length that keeps every
  // join within the run limit, 4096-tuple buckets and 64 K-tuple work items
  uint32_t L, BT, JCH;
  batch_tuning_of(*cfg, sh.max_nS, &L, &BT, &JCH);
  if (!cfg->log2_run_len && L < (1u << 18)) L = 1u << 18;
  // workspace for every candidate tuning (and the initial one)
  BatchPlan P;
  uint64_t ws = 0;
  for (uint32_t l : kBatchL)
    for (uint32_t bt : kBatchBT)
      for (uint32_t jc : kBatchJCH)
        if (make_batch_plan(n, sh, b->cfg, l, bt, jc, &P) && P.total > ws) ws = P.total;
  if (!make_batch_plan(n, sh, b->cfg, L, BT, JCH, &P)) { delete b; return MPSM_EUNSUPPORTED; }
  b->ws_max = P.total > ws ? P.total : ws;
  const mpsm_status rc = batch_set(b, L, BT, JCH);
  if (rc != MPSM_OK) { mpsm_batch_destroy(b); return rc; }
  *out = b;
  return MPSM_OK;
}

void mpsm_batch_destroy(mpsm_batch* b) {
  if (!b) return;
  batch_drop_graph(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->host) (void)hipHostFree(b->host);
  delete b;
}

uint64_t mpsm_batch_workspace_bytes(const mpsm_batch* b) { return b ? b->ws_max : 0; }

mpsm_status mpsm_batch_run(mpsm_batch* b, void* d_workspace, uint64_t workspace_bytes, void* stream, int use_graph) {
  return batch_run(b, d_workspace, workspace_bytes, stream, use_graph);
}

mpsm_status mpsm_batch_get_tuning(const mpsm_batch* b, mpsm_batch_tuning* t) {
  if (!b || !t) return MPSM_EINVAL;
  memset(t, 0, sizeof(*t));
  t->log2_run_len = (uint32_t)__builtin_ctz(b->L);
  t->bucket_target = b->BT;
  t->join_chunk = b->JCH;
  return MPSM_OK;
}

mpsm_status mpsm_batch_set_tuning(mpsm_batch* b, const mpsm_batch_tuning* t) {
  if (!b || !t || t->log2_run_len > 31) return MPSM_EINVAL;
  return batch_set(b, 1u << t->log2_run_len, t->bucket_target, t->join_chunk);
}

mpsm_status mpsm_batch_autotune(mpsm_batch* b, void* d_workspace, uint64_t workspace_bytes, void* stream,
                                const char* cache_path, mpsm_batch_tuning* chosen) {
  if (!b) return MPSM_EINVAL;
  const uint32_t n = (uint32_t)b->d.size();
  const std::string sig = batch_signature(b);
  uint32_t L = 0, BT = 0, JCH = 0;
  if (cache_lookup(cache_path, sig, &L, &BT, &JCH)) {
    BatchPlan P;
    if (make_batch_plan(n, b->shape, b->cfg, L, BT, JCH, &P) && (!d_workspace || P.total <= workspace_bytes)) {
      const mpsm_status rc = batch_set(b, L, BT, JCH);
      if (rc != MPSM_OK) return rc;
      if (chosen) { mpsm_batch_get_tuning(b, chosen); chosen->from_cache = 1; }
      return MPSM_OK;
    }
  }
  if (!d_workspace) return MPSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = -1.f;
  uint32_t bL = b->L, bBT = b->BT, bJ = b->JCH;
  mpsm_status rc = MPSM_OK;
  for (uint32_t l : kBatchL)
    for (uint32_t bt : kBatchBT)
      for (uint32_t jc : kBatchJCH) {
        BatchPlan P;
        if (!make_batch_plan(n, b->shape, b->cfg, l, bt, jc, &P) || P.total > workspace_bytes) continue;
        if ((rc = batch_set(b, l, bt, jc)) != MPSM_OK) break;
        if ((rc = batch_run(b, d_workspace, workspace_bytes, stream, 0)) != MPSM_OK) break;   // warm-up
        float t[3];
        for (int r = 0; r < 3 && rc == MPSM_OK; r++) {
          if (hipEventRecord(e0, st) != hipSuccess) { rc = MPSM_EHIP; break; }
          rc = batch_run(b, d_workspace, workspace_bytes, stream, 0);
          if (rc != MPSM_OK) break;
          if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
            rc = MPSM_EHIP;
        }
        if (rc != MPSM_OK) break;
        const float med = t[0] < t[1] ? (t[1] < t[2] ? t[1] : (t[0] < t[2] ? t[2] : t[0]))
                                       : (t[0] < t[2] ? t[0] : (t[1] < t[2] ? t[2] : t[1]));
        if (best < 0.f || med < best) { best = med; bL = l; bBT = bt; bJ = jc; }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != MPSM_OK) return rc;
  if (best < 0.f) return MPSM_ENOMEM;
  rc = batch_set(b, bL, bBT, bJ);
  if (rc != MPSM_OK) return rc;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s %u %u %u %.4f\n", sig.c_str(), (unsigned)__builtin_ctz(bL), bBT, bJ, best);
      fclose(f);
    }
  }
  if (chosen) { mpsm_batch_get_tuning(b, chosen); chosen->from_cache = 0; chosen->ms = best; }
  return MPSM_OK;
}

uint64_t mpsm_clock_hz(void) { return 100000000ull; }

mpsm_status mpsm_join_slices_host(const uint32_t* oa, const uint32_t* ob, const uint32_t* run_start,
                                  const uint32_t* run_len, uint32_t Q, uint32_t* cum, uint32_t* sbase) {
  if (Q && (!oa || !ob || !run_start || !run_len || !cum || !sbase)) return MPSM_EINVAL;
  uint32_t c = 0;
  for (uint32_t j = 0; j < Q; j++) {
    cum[j] = c;
    sbase[j] = slice_base(run_start[j], oa[j], run_len[j], c);
    c += slice_len(oa[j], ob[j], run_len[j]);
  }
  if (cum) cum[Q] = c;
  return MPSM_OK;
}

mpsm_status mpsm_lower_bound_window_host(const uint64_t* keys, uint32_t a, uint32_t b, uint64_t klo, uint64_t khi,
                                         uint64_t key, uint32_t* out, uint32_t* probes) {
  if (!out || (a < b && !keys)) return MPSM_EINVAL;
  uint32_t pr = 0;
  *out = lb_window_at([keys](uint32_t i) { return keys[i]; }, a, b, klo, khi, key, &pr);
  if (probes) *probes = pr;
  return MPSM_OK;
}

}  // extern "C"
