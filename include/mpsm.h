/*
 * mpsm.h -- C ABI of the range-partitioned massively parallel sort-merge
 * (P-MPSM) equi-join on one AMD Instinct MI355X (gfx950).
 *
 * Method: Albutiu, Kemper, Neumann, "Massively Parallel Sort-Merge Joins in
 * Main Memory Multi-Core Database Systems", PVLDB 5(10), 2012.
 *   Problem statement (Section 5.1): relations of {joinkey: 64-bit,
 *   payload: 64-bit} tuples, equi-join on joinkey, no foreign-key or index
 *   assumptions.
 *   Method (Section 3.2, Fig. 5): phase 1 sorts chunks of the public input S
 *   into runs; phase 2 range-partitions the private input R with histograms,
 *   prefix sums and a synchronisation-free scatter (Section 3.2.1, Figs. 6
 *   and 10); phase 3 sorts every R partition; phase 4 merge-joins every R
 *   partition with every S run from a searched start position (Section
 *   3.2.2, Fig. 7).  Role choice: the smaller input is the private one
 *   (Section 3.2).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HIP global memory of the
 *     current device); everything else is host memory.
 *   - Calls only enqueue work on `stream` (a hipStream_t, may be NULL for the
 *     default stream) and return; results are valid once the stream has
 *     completed, unless the call documents that it synchronises.
 *   - The library never allocates device memory on these paths and keeps no
 *     pointer after returning.  The caller owns all buffers.
 *   - Inputs are never modified.
 *   - Arguments are validated on the host before anything is enqueued; a
 *     rejected call enqueues nothing.  Only a failing HIP runtime call
 *     (MPSM_EHIP) can end a call after part of its work was enqueued.
 */
#ifndef MPSM_H
#define MPSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One tuple: 16 bytes, 16-byte aligned arrays (Section 5.1 schema). */
typedef struct mpsm_tuple {
  uint64_t key;
  uint64_t payload;
} mpsm_tuple;

/* One join result pair, always in the caller's orientation. 24 bytes. */
typedef struct mpsm_pair {
  uint64_t key;
  uint64_t r_payload;
  uint64_t s_payload;
} mpsm_pair;

typedef enum mpsm_status {
  MPSM_OK = 0,
  MPSM_EINVAL = 1,        /* bad argument (NULL with n > 0, misalignment, size limits, bad config) */
  MPSM_ECAPACITY = 2,     /* more pairs than pairs_capacity (only reported by synchronising calls) */
  MPSM_ENOMEM = 3,        /* workspace smaller than mpsm_workspace_bytes() */
  MPSM_EHIP = 4,          /* a HIP runtime call failed */
  MPSM_EUNSUPPORTED = 5   /* option not available */
} mpsm_status;

enum { MPSM_ROLE_AUTO = 0, MPSM_ROLE_AS_GIVEN = 1, MPSM_ROLE_SWAP = 2 };
/* Splitters of the range partitioning of R:
 *   SAMPLED  equi-depth quantiles of a seeded sample, per segment;
 *   LEARNED  first level from the inverse of a learned CDF of R (a
 *            piecewise-linear CDF over 4096 sample quantiles plus a small
 *            residual network, trained on the GPU from 2^16 keys the call
 *            draws); a second level, when R needs one, stays sampled (its
 *            buckets are finer than the model's knots).
 * The learned CDFs are built on a stream of the library's own (one per
 * calling thread) while S is sorted, and joined before R is partitioned.
 * S runs are always split by sampled splitters.
 *   COST     first level balanced by the paper's cost model (Section 4.3):
 *            the largest partition cost |R_i| log2 |R_i| + Q |R_i| + |S_i|
 *            (Q = S runs; |S_i| from the S runs' equi-height bounds merged
 *            into a global S distribution, Section 4.1; |R_i| from a sorted
 *            R sample) is minimised over contiguous groups of sample cells.
 *            A second level, when R needs one, stays sampled.
 *   NONE     B-MPSM (Section 2.1, Fig. 3): no range partitioning.  R is
 *            sorted into runs of the S run length exactly as S is, and every
 *            R run is merge-joined with every S run (each partition of an R
 *            run is one of its sort buckets, a key range inside that run).
 *            Its join work grows with the number of R runs, and it is
 *            immune to skew by construction. */
enum { MPSM_SPLIT_SAMPLED = 0, MPSM_SPLIT_LEARNED = 1, MPSM_SPLIT_COST = 2, MPSM_SPLIT_NONE = 3 };
/* Start search of every R partition in every S run (Section 3.2.2):
 *   BINARY   bisection of the run;  INTERP  the paper's interpolation search;
 *   INDEX    bisection of the run's equi-height index, then of one window;
 *   LEARNED  INDEX narrowed to an error-bounded window around the slot the
 *            learned CDF of S predicts, with the full index bisection as the
 *            fallback when the window does not bracket the answer. */
enum { MPSM_SEARCH_BINARY = 0, MPSM_SEARCH_INTERP = 1, MPSM_SEARCH_LEARNED = 2, MPSM_SEARCH_INDEX = 3 };

/* Tuning and variant choices.  Zero in a numeric field means "automatic".
 * No choice changes the join result (count, checksum, pair multiset). */
typedef struct mpsm_config {
  uint32_t struct_size;    /* sizeof(mpsm_config) */
  int32_t role;            /* MPSM_ROLE_*: which input is private (R) */
  int32_t splitter;        /* MPSM_SPLIT_*: how R's range partitions are chosen */
  int32_t search;          /* MPSM_SEARCH_*: how merge starts in S runs are found */
  uint32_t log2_run_len;   /* S run length 2^k, 12 <= k <= 24 */
  uint32_t bucket_target;  /* mean tuples per sort bucket / R partition, 256..4096 */
  uint32_t join_chunk;     /* S tuples per join work item, 1024..261888 */
  uint32_t want_max;       /* 1: also compute max(R.payload + S.payload) (Section 5.1 query) */
  uint32_t oversample;     /* sample keys drawn per bucket for the splitters of every level, 1..64
                              (0: 32 for S's runs and R's first level, 16 for R's second) */
  uint32_t waves;          /* batches only: waves the joins are taken in, 1..64 (see mpsm_join_batch) */
  uint64_t seed;           /* seed of the splitter samples */
} mpsm_config;

/* Optional host-side statistics (filled by synchronising calls). */
typedef struct mpsm_stats {
  uint64_t max_payload_sum;   /* wrapping u64 max of R.payload + S.payload over pairs */
  uint64_t nonempty;          /* 1 if the join has at least one pair */
  uint64_t partitions;        /* non-empty R partitions */
  uint64_t runs;              /* S runs */
  uint64_t oversize_buckets;  /* buckets sorted by the multi-pass fallback */
  uint64_t search_probes;     /* key reads made by the start search */
  uint64_t swapped;           /* 1 if the caller's S was used as the private input */
  double ms_total;            /* device time of the whole call */
  uint64_t search_fallbacks;  /* learned search: predictions whose window failed the bracket check */
  uint64_t max_partition;     /* tuples in the largest R partition */
  double cdf_eps_r;           /* learned CDF of R: largest error on its sample (-1 if not trained) */
  double cdf_eps_s;           /* learned CDF of S: same */
  uint64_t resorted_buckets;  /* buckets whose one-pass sort gave up, re-sorted by LSD radix passes */
  uint64_t retried_buckets;   /* R buckets the one-pass sort gave up on and sorted again over their own key range */
  uint64_t pairs_truncated;   /* 1 if pairs were requested and the join has more than pairs_capacity */
  uint64_t redone_runs;       /* S runs whose bucket regions overflowed and were scattered again exactly
                                 (large S only: smaller S takes the exact path directly) */
  uint64_t redone_r_segments; /* the same for R: first-level buckets redone at the second level (large R with
                                 two levels), or R runs (large R, MPSM_SPLIT_NONE) */
} mpsm_stats;

/* Fill *cfg with defaults (all automatic, role AUTO, sampled splitters,
 * index-assisted binary search, seed 0x1207014500000000). */
void mpsm_config_default(mpsm_config* cfg);

/* Bytes of device workspace mpsm_join needs for these sizes and options.
 * cfg may be NULL (defaults).  Returns 0 if the sizes are not supported. */
uint64_t mpsm_workspace_bytes(uint64_t nR, uint64_t nS, const mpsm_config* cfg);

/* The equi-join of R and S (paper Section 3.2):
 *   d_R, d_S        device arrays of nR / nS tuples, 16-byte aligned; may be
 *                   NULL when the count is 0.  nR, nS < 2^32.
 *   d_out_count     device u64: number of pairs (r, s) with r.key == s.key.
 *   d_out_checksum  device u64: sum over all pairs, mod 2^64, of
 *                   H = m(m(m(key + 0x9E3779B97F4A7C15) + r.payload) + s.payload),
 *                   m = the SplitMix64 output function.  Order independent.
 *   d_pairs         optional device array of pairs_capacity pairs; when
 *                   non-NULL the first min(count, pairs_capacity) pairs are
 *                   written in unspecified order.  The count is always
 *                   exact, so a caller can size the buffer with a first call.
 *   cfg             optional (NULL = defaults).
 *   d_workspace     device buffer of at least mpsm_workspace_bytes(nR, nS,
 *                   cfg) bytes, 256-byte aligned; its contents on entry do
 *                   not matter and on return hold intermediate results.
 *   stream          hipStream_t (void* here so the header needs no HIP).
 *   stats           optional; when non-NULL the call synchronises the
 *                   stream and fills *stats, and returns MPSM_ECAPACITY if
 *                   pairs were truncated (the device status word the call
 *                   keeps in its workspace; without stats the caller can
 *                   test *d_out_count > pairs_capacity itself).
 * Returns MPSM_OK; argument errors (MPSM_EINVAL, MPSM_ENOMEM) are returned
 * before anything is enqueued.  A HIP failure (MPSM_EHIP) can happen after
 * part of the launch sequence was enqueued; the caller's stream is then made
 * to wait for the library's side stream before the call returns. */
mpsm_status mpsm_join(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS,
                      uint64_t* d_out_count, uint64_t* d_out_checksum, mpsm_pair* d_pairs, uint64_t pairs_capacity,
                      const mpsm_config* cfg, void* d_workspace, uint64_t workspace_bytes, void* stream,
                      mpsm_stats* stats);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mpsm_join
 * with the workspace taken from a fixed array inside the library, one copy
 * per GPU, MPSM_NOALLOC_SCRATCH_BYTES bytes, held until the process ends.
 * Same arguments, results and errors as mpsm_join, without the caller's
 * workspace and without stats; the call uses the caller's stream only (no
 * second stream) and calls no allocating routine.  Joins whose workspace
 * (mpsm_workspace_bytes) exceeds MPSM_NOALLOC_SCRATCH_BYTES return
 * MPSM_ENOMEM before any device call (about 1.5 M tuples in all fit).  The
 * array's address on a GPU is looked up on the first call with that GPU
 * current.  Every call on one GPU shares its array and leaves its
 * intermediate results there; each call initialises what it needs, so the
 * previous contents never matter, but calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race. */
#define MPSM_NOALLOC_SCRATCH_BYTES (64ull << 20)
mpsm_status mpsm_join_noalloc(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS,
                              uint64_t* d_out_count, uint64_t* d_out_checksum, mpsm_pair* d_pairs,
                              uint64_t pairs_capacity, const mpsm_config* cfg, void* stream);

/* Human-readable name of a status code (static string). */
const char* mpsm_status_string(mpsm_status s);

/* Where mpsm_join leaves its intermediate results inside the workspace,
 * for inspection by tests.  All offsets are byte offsets into the workspace;
 * counts that depend on the data are stored in the workspace at the given
 * offsets (u32).  Fills *out and returns MPSM_OK, or MPSM_EINVAL. */
typedef struct mpsm_layout {
  uint32_t swapped;          /* private input is the caller's S */
  uint32_t levels;           /* R partitioning levels (1 or 2) */
  uint64_t run_len;          /* S run length */
  uint32_t runs;             /* Q = number of S runs */
  uint32_t s_buckets;        /* buckets per S run */
  uint32_t r_buckets1;       /* level-1 R buckets */
  uint32_t r_buckets2;       /* level-2 R buckets per level-1 bucket (1 if one level) */
  uint32_t s_oversample, r_oversample1, r_oversample2;
  uint64_t s_level_seed, r_level_seed1, r_level_seed2;  /* segment s samples with splitmix(level_seed, s) */
  uint64_t off_s_sorted;     /* nS' tuples: the S runs, each sorted */
  uint64_t off_r_sorted;     /* nR' tuples: R sorted, partitions contiguous */
  uint64_t off_s_splitters;  /* runs * (s_buckets-1) u64 */
  uint64_t off_r_splitters1; /* r_buckets1-1 u64 */
  uint64_t off_r_splitters2; /* r_buckets1 * (r_buckets2-1) u64 */
  uint64_t off_s_bucket_start; /* runs*s_buckets+1 u32 */
  uint64_t off_r_bucket_start1;/* r_buckets1+1 u32 */
  uint64_t off_r_bucket_start; /* final R buckets + 1 u32 (positions in the sorted R) */
  uint64_t off_partitions;   /* u32 count P of non-empty R partitions */
  uint64_t off_part_start;   /* P u32 */
  uint64_t off_part_len;     /* P u32 */
  uint64_t off_part_key;     /* P u64: first key of each partition */
  uint64_t off_offsets;      /* (P_max+1) x runs u32: start of partition p in run j; written for the
                                partitions that start a join unit (span > 0) and for row P */
  uint32_t p_max;            /* capacity of the partition arrays */
  uint32_t idx_stride;       /* equi-height index: every idx_stride-th key of a run */
  uint64_t off_run_index;    /* runs * idx_per_run u64 */
  uint32_t idx_per_run;
  uint32_t padded_passes;    /* bucket passes without a histogram (sample-sized regions, exact redo on
                                overflow): bit 0 S's runs, bit 1 R's runs (MPSM_SPLIT_NONE), bit 2 R's
                                second level */
  uint64_t off_join_span;    /* P u8: partitions joined together starting at p (2: p and p+1 share an LDS
                                tile; 1: p alone; 0: p is the second of a pair) */
  /* splitter COST only: */
  uint64_t off_cost_sample;  /* cost_cells u64: the sorted R sample (cell i starts at its key i) */
  uint64_t off_cost_s_below; /* cost_cells+1 u64: estimated S tuples below each sample key; last = |S| */
  uint64_t off_cost_best;    /* f64: the largest group cost of the chosen split */
  uint32_t cost_cells;
  uint32_t reserved2;
  /* learned CDF models (R's with splitter LEARNED, S's with search LEARNED):
     each starts with cdf_knots u64 knot keys, the sorted keys of ranks
     floor(i (cdf_sample - 1) / (cdf_knots - 1)) of a sample of cdf_sample
     keys of the relation drawn at positions floor(x_t n / 2^64), x_t the
     SplitMix64 stream cdf_seed_r / cdf_seed_s (t = 0 .. cdf_sample - 1) */
  uint64_t off_cdf_model_r, off_cdf_model_s;
  uint64_t cdf_seed_r, cdf_seed_s;
  uint32_t cdf_sample, cdf_knots;
} mpsm_layout;

mpsm_status mpsm_workspace_layout(uint64_t nR, uint64_t nS, const mpsm_config* cfg, mpsm_layout* out);

/* Measurement: mpsm_join that also records events[i] (hipEvent_t handles,
 * created with mpsm_events_create) on `stream` at marker i of the launch
 * sequence, for i < n_events.  Marker i is placed after the step named by
 * mpsm_marker_name(i); marker 0 is the start.  Steps that a call does not
 * run still record their marker, so the elapsed time between consecutive
 * markers is the device time of that step.  R's partitioning and sort
 * (markers r1_splitters .. r_oversize_sort) run on a second stream of the
 * library, beside S's bucket sort (from the end of S's scatter on), unless
 * splitters are cost-balanced; their markers are then recorded on that
 * stream, R's first step counts from s_scatter, and the partition step from
 * the later of s_oversize_sort and r_oversize_sort.  Same arguments, results and errors
 * as mpsm_join otherwise. */
mpsm_status mpsm_join_events(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* d_S, uint64_t nS,
                             uint64_t* d_out_count, uint64_t* d_out_checksum, mpsm_pair* d_pairs,
                             uint64_t pairs_capacity, const mpsm_config* cfg, void* d_workspace,
                             uint64_t workspace_bytes, void* stream, void** events, uint32_t n_events);

/* The equi-join with S outside device memory (the memory-constrained
 * variant of Section 3.1 and its Figure 4, which spills the sorted runs to
 * disk and reads them back in key order during the join).  Here S and its
 * runs live in host memory; R, the private input, is partitioned and sorted
 * on the device first, and S then passes through the device once, in
 * chunks of whole runs: each chunk is sorted into runs, joined with every R
 * partition while it is on the device (the join is a sum over runs), and
 * its runs are written back to host memory.
 *   h_S       pinned host array (hipHostMalloc, or a pinned torch tensor) of
 *             nS tuples, 16-byte aligned; read only.
 *   h_runs    pinned host array of nS tuples, 16-byte aligned, written: on
 *             completion it holds S's Q = ceil(nS / L) runs in place (run q
 *             is S[q*L, min((q+1)*L, nS)) sorted by key; L is the run
 *             length of the plan: 2^cfg->log2_run_len, or chosen from nS
 *             when that is 0, as the run_len of mpsm_workspace_layout for
 *             the same sizes and cfg->role = MPSM_ROLE_AS_GIVEN reports).
 *             May be NULL: the runs are then not kept, and S crosses the
 *             host link once, inwards.  With nR = 0 nothing is joined and
 *             no runs are written.
 *   chunk_tuples  tuples copied in, sorted and joined at a time (rounded
 *             down to a multiple of L, at least L): the device holds two
 *             chunks of S (one is copied while the other is sorted), so the
 *             workspace grows with the chunk, not with nS.
 * d_R, nR, d_out_count, d_out_checksum, d_workspace (at least
 * mpsm_join_host_runs_workspace_bytes() bytes) and stream as for mpsm_join;
 * R stays the private input and S the public one (cfg->role SWAP, and the
 * splitter kinds that need S's runs before R's partitioning, COST and NONE,
 * return MPSM_EINVAL), no pairs are written and no statistics kept.  A host
 * buffer that the device cannot address returns MPSM_EINVAL before anything
 * is enqueued.  The call returns once the work is enqueued on `stream`;
 * h_S must stay unchanged and h_runs unread until the stream completes. */
uint64_t mpsm_join_host_runs_workspace_bytes(uint64_t nR, uint64_t nS, const mpsm_config* cfg,
                                             uint64_t chunk_tuples);
mpsm_status mpsm_join_host_runs(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* h_S, uint64_t nS,
                                mpsm_tuple* h_runs, uint64_t* d_out_count, uint64_t* d_out_checksum,
                                const mpsm_config* cfg, uint64_t chunk_tuples, void* d_workspace,
                                uint64_t workspace_bytes, void* stream);

/* The join phase of the memory-constrained variant on its own (Section 3.1,
 * Fig. 4): S's sorted runs are already in host memory, as
 * mpsm_join_host_runs leaves them in h_runs, and a private input R is
 * joined with them without sorting S again.  R is partitioned and sorted on
 * the device; the run index (every 256th key of each run, the page index of
 * Fig. 4) is read from the runs; the start search and the join then move
 * through the key domain partition by partition and read each run's slice
 * of it over the host link, each slice once.
 *   h_runs  pinned host array of nS tuples, 16-byte aligned, read only:
 *           Q = ceil(nS / L) runs in place, run q = positions [q*L,
 *           min((q+1)*L, nS)) sorted by key, where L is the run length
 *           mpsm_join_host_runs chooses for the same nS and cfg (it depends
 *           on nS and cfg->log2_run_len only).  Runs that are not sorted
 *           give undefined results, never an access outside h_runs.
 * The other arguments, the workspace (mpsm_join_spilled_runs_workspace_bytes)
 * and the errors are those of mpsm_join_host_runs. */
uint64_t mpsm_join_spilled_runs_workspace_bytes(uint64_t nR, uint64_t nS, const mpsm_config* cfg);
mpsm_status mpsm_join_spilled_runs(const mpsm_tuple* d_R, uint64_t nR, const mpsm_tuple* h_runs, uint64_t nS,
                                   uint64_t* d_out_count, uint64_t* d_out_checksum, const mpsm_config* cfg,
                                   void* d_workspace, uint64_t workspace_bytes, void* stream);

/* Number of markers and the name of the step that ends at marker i
 * (static string; NULL for i out of range). */
uint32_t mpsm_marker_count(void);
const char* mpsm_marker_name(uint32_t i);

/* Create / destroy n timing events; elapsed milliseconds between two
 * completed events (host calls; they synchronise on nothing else). */
mpsm_status mpsm_events_create(void** events, uint32_t n);
void mpsm_events_destroy(void** events, uint32_t n);
mpsm_status mpsm_events_elapsed(void* start, void* stop, float* ms);


/* ---- Batched joins --------------------------------------------------------
 * Many independent equi-joins of uneven sizes as one launch sequence: every
 * phase of the method is a single kernel launch over all joins being joined
 * (segment tables span the joins; each join's inputs are read in place), so
 * the per-launch cost is paid once per group of joins instead of once per
 * join, and the whole sequence can be captured once into a hipGraph and
 * replayed.  Each join's result is the one mpsm_join gives (count and
 * checksum as documented there).  In a batch R is always the private input
 * (no role swap), splitters are sampled and the start search is BINARY,
 * INTERP or INDEX; pairs and the max aggregate are not produced. */
typedef struct mpsm_join_desc {
  const mpsm_tuple* d_R;   /* device, nR tuples, 16-byte aligned (NULL if nR == 0) */
  uint64_t nR;
  const mpsm_tuple* d_S;   /* device, nS tuples, 16-byte aligned (NULL if nS == 0) */
  uint64_t nS;
  uint64_t* d_out_count;   /* device u64 */
  uint64_t* d_out_checksum;/* device u64 */
  uint64_t* d_out_times;   /* device u64[3] or NULL: batch start, start of the join's first work item,
                              end of its last work item (GPU wall clock, mpsm_clock_hz() ticks per second;
                              a join without work items reports the batch start three times) */
} mpsm_join_desc;

/* Bounds of a batch's shape class: the sums of nR and of nS over the joins
 * whose sides are both non-empty, and the largest nS of one join (0: the
 * sum).  Each sum must stay below 2^32.  A launch sized for a shape serves
 * every batch of at most that many joins within its bounds. */
typedef struct mpsm_batch_shape {
  uint64_t max_sum_nR;
  uint64_t max_sum_nS;
  uint64_t max_nS;
} mpsm_batch_shape;

/* Workspace bytes of mpsm_join_batch for n joins of this shape class and
 * config (NULL: defaults); 0 if not supported. */
uint64_t mpsm_join_batch_workspace_bytes(uint32_t n, const mpsm_batch_shape* shape, const mpsm_config* cfg);

/* n independent joins whose descriptors are in DEVICE memory (d_descs: n
 * mpsm_join_desc, 8-byte aligned), as one stream-ordered launch sequence.
 * The host reads neither the descriptors nor any size: launches are sized
 * by n and *shape, and the descriptors are read and checked on the GPU, so
 * the call can be captured into a hipGraph once and the graph replayed for
 * any new batch written into the same descriptor array (same n, within the
 * shape's bounds).  Joins are taken in waves (cfg->waves, 0: 4 for 32 joins
 * or more, 2 for 8 or more, else 1; one wave beyond 4096 joins): ordered
 * by nR + nS (ties by index), cut into groups of equal count, smallest
 * first, so that small joins finish without waiting for the large ones;
 * a join with an empty side is in the first wave.  cfg's log2_run_len (16..22),
 * bucket_target (1024..4096) and join_chunk (4096..261888) set the tuning
 * (0: the shortest run length that keeps every join within 2048 runs,
 * 4096, 65536).  The workspace (mpsm_join_batch_workspace_bytes, 256-byte
 * aligned) needs no initialisation; its first 4 bytes receive the batch
 * status once the stream completes: MPSM_OK, or MPSM_EINVAL when a
 * descriptor is malformed (NULL or misaligned pointers, a size of 2^32 or
 * more, nS above max_nS) or the joins exceed the shape's sums; then no
 * output is written.  Host-side checks (config, shape, alignment, workspace
 * size) return before anything is enqueued.  Calls on one workspace must
 * not overlap.  Nothing is allocated. */
mpsm_status mpsm_join_batch(const mpsm_join_desc* d_descs, uint32_t n, const mpsm_batch_shape* shape,
                            const mpsm_config* cfg, void* d_workspace, uint64_t workspace_bytes, void* stream);

/* Host-side layer over mpsm_join_batch (opaque): keeps a host copy of the
 * descriptors, uploads them into its workspace, picks the tuning (autotuner)
 * and captures the launch into a hipGraph on first use. */
typedef struct mpsm_batch mpsm_batch;

/* Tuning of a batch: the S run length, the mean bucket / partition size
 * (which fixes the number of buckets, i.e. the radix fan-out of every
 * pass) and the S tuples per join work item (the join's work split). */
typedef struct mpsm_batch_tuning {
  uint32_t log2_run_len;   /* 16..22 */
  uint32_t bucket_target;  /* 1024..4096 */
  uint32_t join_chunk;     /* 4096..261888 */
  uint32_t from_cache;     /* set by mpsm_batch_autotune: 1 if read from the cache file */
  float ms;                /* set by mpsm_batch_autotune: measured batch time of the choice (0 if cached) */
} mpsm_batch_tuning;

/* Plan a batch of n >= 1 joins (descs: host array, copied).  Sums of nR and
 * of nS must each stay below 2^32.  cfg may be NULL; its log2_run_len,
 * bucket_target and join_chunk, when non-zero, are the initial tuning.
 * Touches no device.  Returns MPSM_EINVAL / MPSM_EUNSUPPORTED on bad input. */
mpsm_status mpsm_batch_create(const mpsm_join_desc* descs, uint32_t n, const mpsm_config* cfg, mpsm_batch** out);
void mpsm_batch_destroy(mpsm_batch* b);

/* Workspace bytes that serve every tuning the autotuner may pick. */
uint64_t mpsm_batch_workspace_bytes(const mpsm_batch* b);

/* Enqueue the batch on `stream` (mpsm_join_batch with the batch's own sums
 * as its shape).  The first call with a workspace copies the descriptors
 * into it (from pinned memory the batch keeps); with use_graph != 0 the
 * launch sequence is captured into a hipGraph on first use (on a stream the
 * batch owns, after synchronising `stream`) and replayed on `stream`
 * afterwards (the graph is bound to that workspace).  Calls on one workspace
 * must not overlap. */
mpsm_status mpsm_batch_run(mpsm_batch* b, void* d_workspace, uint64_t workspace_bytes, void* stream, int use_graph);

/* Pick the tuning of this batch: from cache_path (a text file, may be NULL)
 * when it holds an entry for a batch of this shape, else by timing every
 * candidate tuning that fits the workspace on `stream` (synchronising) and
 * appending the fastest to the cache.  Unreadable or malformed cache entries
 * are ignored.  Sets the batch's tuning and fills *chosen (may be NULL). */
mpsm_status mpsm_batch_autotune(mpsm_batch* b, void* d_workspace, uint64_t workspace_bytes, void* stream,
                                const char* cache_path, mpsm_batch_tuning* chosen);

/* Current tuning; set a tuning explicitly (validated; drops the graph). */
mpsm_status mpsm_batch_get_tuning(const mpsm_batch* b, mpsm_batch_tuning* t);
mpsm_status mpsm_batch_set_tuning(mpsm_batch* b, const mpsm_batch_tuning* t);

/* Ticks per second of the GPU wall clock used by d_out_times. */
uint64_t mpsm_clock_hz(void);

/* Host copy of the join kernel's slice plan (Section 3.2.2), for tests that
 * run without a GPU.  A join unit reads slice j = [oa[j], ob[j]) of each of
 * the Q sorted S runs (run j at S positions [run_start[j], run_start[j] +
 * run_len[j])); the offsets come from the start search.  The kernel clamps
 * both offsets to the run and treats a reversed pair as empty, so its reads
 * stay inside the runs whatever the offsets hold; this function runs the
 * same per-run code.  Host arrays: oa, ob, run_start, run_len (Q each) in;
 * cum (Q + 1: exclusive prefix of the clamped slice lengths, cum[Q] their
 * sum) and sbase (Q: concatenated index x with cum[j] <= x < cum[j+1] reads
 * S position sbase[j] + x, mod 2^32) out.  Returns MPSM_EINVAL on NULL
 * arrays with Q > 0. */
mpsm_status mpsm_join_slices_host(const uint32_t* oa, const uint32_t* ob, const uint32_t* run_start,
                                  const uint32_t* run_len, uint32_t Q, uint32_t* cum, uint32_t* sbase);

/* The last step of the start search (Section 3.2.2: where a private
 * partition starts in a public run), run on the CPU with the device code, for
 * tests (no GPU needed): the lower bound of key in keys[a, b) (sorted), given
 * that every key before a is smaller and keys[b], if inside the run, is not;
 * klo and khi (the index keys around the window) only choose the first
 * 8-key line it probes.  keys: host array of at least b keys.  *out: the
 * lower bound; *probes (may be NULL): lines probed.  MPSM_EINVAL on NULL
 * out, or NULL keys with a < b. */
mpsm_status mpsm_lower_bound_window_host(const uint64_t* keys, uint32_t a, uint32_t b, uint64_t klo, uint64_t khi,
                                         uint64_t key, uint32_t* out, uint32_t* probes);

#ifdef __cplusplus
}
#endif

#endif /* MPSM_H */
