/*
 * hoph.h -- C ABI of libhoph, the MI355X (gfx950) library for one-permutation
 * hashing (OPH) and its grouped (GOPH) and hierarchical (HOPH) early-stop
 * comparison, after Zhang, Lin, Zhu, Yuan, Long and Huang, "Hierarchical One
 * Permutation Hashing: Efficient Multimedia Near Duplicate Detection"
 * (arXiv 1805.11254).
 *
 * Conventions for every entry point:
 *  - Every call returns hoph_status; nothing is thrown across the ABI and
 *    nothing aborts.  hoph_last_error() holds a message for the calling thread.
 *  - d_* arguments are device pointers (HIP device memory of the current
 *    device); h_* and plain struct pointers are host memory.  The caller owns
 *    every buffer it passes; the library owns hoph_index objects.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Work is queued
 *    on that stream in order.  Calls that must read a device count
 *    (query_*, minwise_query, hoph_sync) synchronise that stream once.
 *  - A set is a CSR segment: ids d_ids[d_offsets[i] .. d_offsets[i+1]), ids in
 *    [0, universe).  Duplicate ids are allowed (the minimum is idempotent).
 *  - A signature is k uint32 words.  Word b is the smallest permuted value that
 *    fell in bin b minus the first value of bin b (Sec. 3.2, "smallest possible
 *    representation"), or HOPH_EMPTY when no value fell in the bin.
 *  - Limits: 1 <= k_group <= 64, k % k_group == 0, k / k_group <= 64.
 */
#ifndef HOPH_H
#define HOPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HOPH_OK = 0,
    HOPH_E_INVAL = -1,       /* invalid argument, checked on the host before any launch      */
    HOPH_E_RANGE = -2,       /* an id >= universe was seen by the device (reported at a sync) */
    HOPH_E_CAPACITY = -3,    /* an output or the index is too small; see hoph_results.needed  */
    HOPH_E_NOMEM = -4,       /* device or pinned host allocation failed                       */
    HOPH_E_UNSUPPORTED = -5, /* exact 64-bit decision state would overflow for these params   */
    HOPH_E_DEVICE = -6       /* a HIP runtime call failed                                     */
} hoph_status;

#define HOPH_EMPTY 0xFFFFFFFFu
#define HOPH_MAX_KGROUP 64u
#define HOPH_MAX_GROUPS 64u

/* An exact rational num/den (den > 0).  T = 0.8 is {4, 5}; eps = 1e-4 is {1, 10000}. */
typedef struct { uint32_t num, den; } hoph_ratio;

/* The one shared permutation psi (Sec. 3.2). */
enum {
    HOPH_HASH_TABLE = 0,      /* psi(x) = d_perm[x]; d_perm is a bijection of [0, universe); R = universe   */
    HOPH_HASH_MODP31 = 1,     /* psi(x) = (a x + b) mod (2^31 - 1); universe <= 2^31 - 1; R = 2^31 - 1       */
    HOPH_HASH_MODP32P15 = 2   /* psi(x) = (a x + b) mod (2^32 + 15); universe <= 2^32; R = 2^32 + 15        */
};

/* How the permuted range [0, R) is cut into k bins. */
enum {
    HOPH_LAYOUT_OPH = 0,      /* Sec. 3.2: k equal contiguous bins, bin(v) = floor(v k / R); GOPH groups are
                                 the contiguous runs of k_group bins                                     */
    HOPH_LAYOUT_HIER = 1      /* Sec. 4.1: split a:b (floor), the first part is a group of k_group equal
                                 bins, the second part is split again; L = k / k_group groups; every split
                                 must leave both parts larger than k_group (the paper's stop rule)         */
};

/* Which bins count as "empty" in N_eb (Eqs. 2 and 4). */
enum {
    HOPH_EMPTY_JOINT = 0,     /* Eq. 4: empty in both signatures (default)                              */
    HOPH_EMPTY_LITERAL = 1,   /* no correction: rate = matched / k_group (Alg. 1 and 2 as printed)      */
    HOPH_EMPTY_EITHER = 2     /* empty in either signature (reproduces the worked examples' estimates)  */
};

typedef struct {
    uint32_t layout;          /* HOPH_LAYOUT_*                                           */
    uint32_t k;               /* bins per signature                                      */
    uint32_t k_group;         /* k': bins per group                                      */
    uint32_t ratio_a;         /* HIER: the a of a:b (>= 1); ignored for OPH              */
    uint32_t ratio_b;         /* HIER: the b of a:b (>= 1)                               */
    uint32_t hash;            /* HOPH_HASH_*                                             */
    uint64_t universe;        /* D: every id must be < universe                          */
    uint64_t hash_a;          /* MODP*: 1 <= a < p                                       */
    uint64_t hash_b;          /* MODP*: 0 <= b < p                                       */
    const uint32_t *d_perm;   /* TABLE: device array of universe entries, a bijection    */
} hoph_sketch_params;

/* How the coarse pass compares the first coarse_depth groups of every pair.
   Results are identical either way; only the work differs. */
enum {
    HOPH_COARSE_CODES = 0,    /* an 8-bit code per bin, EMPTY kept distinct (the "smallest
                                 possible representation" of Sec. 3.2 narrowed further):
                                 codes never under-count matched bins, so a pair is dropped
                                 only where the full comparison rejects it too; every other
                                 pair is re-checked on the 32-bit words (default)          */
    HOPH_COARSE_WORDS = 1     /* the full 32-bit words, accepting and rejecting            */
};

typedef struct {
    hoph_ratio T;             /* similarity threshold, 0 < T <= 1                        */
    hoph_ratio eps;           /* error tolerance of the small-probability event, 0 <= eps < 1 */
    uint32_t empty_policy;    /* HOPH_EMPTY_*                                            */
    uint32_t coarse_depth;    /* 0 = let the library choose (the first group alone when it
                                 rejects at least 1/8 of its match counts, else one group
                                 past the first step that has a reject cutoff, in whole code
                                 units; a batch whose survivors overflow at that depth is
                                 re-run at the deepest available); else the most groups
                                 scanned for a pair before it moves to the per-pair pass (a tuning knob: results do
                                 not depend on it).  Clamped to the groups available: with
                                 codes, the groups that carry codes (whole code units of
                                 pk groups, pk = min(floor(32 / k'), L) for k' <= 16, else 1:
                                 at least 4 units, about 128 bins for HOPH and 256 for GOPH,
                                 at most 24 units, 12 when k' > 32); on words, 4 groups of
                                 at most 128 bins */
    uint32_t coarse_filter;   /* HOPH_COARSE_*                                           */
    uint32_t reserved;        /* set to 0                                                */
} hoph_query_params;

/* Accepted pairs as CSR: for query i, set ids d_set_ids[d_offsets[i] .. d_offsets[i+1]),
   ascending.  needed is written on return: the total number of accepted pairs. */
typedef struct {
    uint64_t *d_offsets;      /* device, n_q + 1 entries                                 */
    uint32_t *d_set_ids;      /* device, capacity entries                                */
    uint64_t capacity;
    uint64_t needed;          /* out                                                     */
} hoph_results;

typedef struct hoph_index hoph_index;   /* opaque, owned by the library */

/*
 * sketch_oph -- OPH / HOPH signatures of n_sets sets (Sec. 3.2, Sec. 4.1).
 * d_sigs: n_sets * k uint32, row-major (set i at d_sigs + i * k).
 * Asynchronous.  An id >= universe (or, for HOPH_HASH_TABLE, a table value >= the
 * universe) raises HOPH_E_RANGE at the next hoph_sync on the device, and the
 * signature of its set is then unspecified; an empty set gets an all-EMPTY
 * signature and raises HOPH_E_INVAL there (Jaccard similarity is undefined for it),
 * and so does a set whose end offset is below its start (none of its ids is read).
 * Offsets must stay within d_ids: the device cannot check that bound.
 * Host errors: HOPH_E_INVAL (bad params, null pointers with n_sets > 0).
 */
hoph_status sketch_oph(const hoph_sketch_params *params, const uint32_t *d_ids,
                       const uint64_t *d_offsets, uint64_t n_sets, uint32_t *d_sigs,
                       void *hip_stream);

/*
 * build_index -- a resident index of signatures: the signature words in
 * row-major rows (one set's k words contiguous, so the per-pair pass of
 * Sec. 3.3 / Sec. 4.1 reads one group of one set as one run) plus, for the
 * first groups, 8-bit bin codes stored as bit planes in tiles of 64 sets (the
 * coarse pass's input; hoph_index_code_planes gives their layout).
 * capacity >= n_sets is the number of sets the index can hold (index_append
 * grows it up to capacity).
 * d_sigs: n_sets * k uint32 row-major, as written by sketch_oph.  Allocates device
 * memory (the only allocation point besides first-use workspace growth).
 * Asynchronous on hip_stream; *out is valid on return.
 */
hoph_status build_index(const hoph_sketch_params *params, const uint32_t *d_sigs,
                        uint64_t n_sets, uint64_t capacity, hoph_index **out, void *hip_stream);

/* index_append -- append n_new signatures (ids continue from the current size).
   HOPH_E_CAPACITY if size + n_new > capacity.  Asynchronous. */
hoph_status index_append(hoph_index *index, const uint32_t *d_sigs, uint64_t n_new,
                         void *hip_stream);

/*
 * index_append_sets -- sketch n_sets sets (Sec. 3.2, Sec. 4.1, with the index's
 * own sketch parameters, as sketch_oph) straight into the index: each
 * signature is written into its index row (and the narrowed code planes of
 * the first groups) without an intermediate copy; ids continue from the
 * current size.  d_ids / d_offsets as for sketch_oph (device, CSR).  Results
 * are identical to sketch_oph followed by index_append.  HOPH_E_CAPACITY if
 * size + n_sets > capacity.  Asynchronous; ids out of range and empty sets are
 * reported as by sketch_oph, at the next hoph_sync on the device.  The
 * permutation table of a HOPH_HASH_TABLE index must stay valid.
 */
hoph_status index_append_sets(hoph_index *index, const uint32_t *d_ids, const uint64_t *d_offsets,
                              uint64_t n_sets, void *hip_stream);

/* hoph_index_reset -- forget every stored set (size 0, capacity kept) so the
   index can be refilled with index_append without a new allocation. */
hoph_status hoph_index_reset(hoph_index *index);

/* hoph_query_timing -- device time of the last query_* call on this index, in
   milliseconds, measured with HIP events on the query's stream:
   ms[0] coarse pass, ms[1] per-survivor pass, ms[2] sort and CSR output.
   (query_oph_full reports its scan in ms[0].) */
hoph_status hoph_query_timing(const hoph_index *index, float ms[3]);

/* hoph_query_counts -- pair counts of the last query_goph / query_hoph call on
   this index (host array): counts[0] the pairs the coarse pass kept for the
   per-survivor pass (all of them, when the batch was redone in parts),
   counts[1] the accepted pairs (Alg. 1 / Alg. 2 outcomes).  Zeros before any
   query and after a query with no queries or no sets. */
hoph_status hoph_query_counts(const hoph_index *index, uint64_t counts[2]);

/* Coarse-pass kernels, as hoph_coarse_plan reports them. */
enum {
    HOPH_PLAN_NONE = 0,               /* no query yet, or nothing to compare                          */
    HOPH_PLAN_WORDS = 1,              /* the 32-bit words of the first groups (HOPH_COARSE_WORDS)      */
    HOPH_PLAN_CODES = 2,              /* the codes of one or more groups, the general form            */
    HOPH_PLAN_FIRST_GROUP = 3,        /* the first group's codes, every plane held in registers       */
    HOPH_PLAN_FIRST_GROUP_LIGHT = 4,  /* the first group's codes, only the first-phase planes held     */
    HOPH_PLAN_LINEAR = 5,             /* two to four groups' codes under the linear bound              */
    HOPH_PLAN_LINEAR_LIGHT = 6,       /* the same, only the first-phase planes held                    */
    HOPH_PLAN_OPH_FULL = 7            /* the plain OPH comparator's full-signature pass                */
};

/* hoph_coarse_plan -- how the last query_*, self_join or hoph_scan_timing call
   on this index ran its coarse pass (host array; a report, the results do not
   depend on it):
   plan[0] the groups it walked (its depth; 0 for HOPH_PLAN_OPH_FULL),
   plan[1] the kernel (HOPH_PLAN_*), plan[2] the code planes compared before
   the rest (0: one phase), plan[3] tiles of 64 indexed sets per wavefront.
   The first-group kernels and their plane count follow an expected-cost model;
   a self-join feeds it keep rates measured on sampled pairs of index rows
   (taken on the first self-join with given parameters, and again when the
   index size has changed twofold; kept across hoph_index_reset). */
hoph_status hoph_coarse_plan(const hoph_index *index, uint32_t plan[4]);

/* hoph_scan_timing -- a measurement hook: the coarse pass of query_goph /
   query_hoph (by the index layout; Alg. 1 / Alg. 2 up to the coarse depth) for
   the n_q query signatures d_qsigs, timed alone.  The per-query records are
   built once, the pass runs once untimed and then reps times back to back
   between two HIP events on hip_stream; the mean duration of one pass in
   milliseconds is written to *ms_per_launch.  With flush_bytes > 0 (at least
   4 MiB; pick it larger than the device's last-level cache), d_flush (device,
   caller-owned, 16-byte aligned, flush_bytes long) is read before every timed
   pass, so that each pass reads the index from HBM into caches that hold only
   clean lines, and the time of those reads alone (timed the same way right
   after) is subtracted; its first 4 MiB may be overwritten.  No results are
   produced.  Synchronises hip_stream. */
hoph_status hoph_scan_timing(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                             const hoph_query_params *qp, uint32_t reps, void *d_flush, uint64_t flush_bytes,
                             float *ms_per_launch, void *hip_stream);

/* hoph_stream_timing -- a measurement hook for the HBM ceilings the kernels are
   compared with: mean device ms of one pass, over reps passes back to back, of
   ms[0] reading d_a (bytes, 16-byte aligned; its first 4 MiB may be
   overwritten), ms[1] writing d_b (bytes, 8-byte aligned), ms[2] copying d_a to
   d_b (device to device).  bytes >= 4 MiB.  Synchronises hip_stream. */
hoph_status hoph_stream_timing(void *d_a, void *d_b, uint64_t bytes, uint32_t reps, float ms[3], void *hip_stream);

/* hoph_append_timing -- device time of the last index_append_sets call on this
   index, in ms: ms[0] the sketch into the index rows, ms[1] the code planes of
   the new rows (0 where the sketch writes them itself: an odd code-unit width
   or odd k) (zeros before any call).  Waits for that call to finish. */
hoph_status hoph_append_timing(const hoph_index *index, float ms[2]);

/* hoph_index_code_planes -- copies the index's narrowed code planes (a test
   hook, for comparing how they were written): dims[0] = code units that carry
   codes (a unit is pk whole consecutive groups, pk = min(floor(32 / k'), L)
   when k' <= 16, else one group), dims[1] = rows (the capacity), dims[2] =
   words per (row, unit) (PW = 8 W, W = 1 plane word, 2 when k' > 32; word
   p W + w holds bit p of the 8-bit codes of the unit's bins 32 w .. 32 w + 31);
   word w of (unit u, row s) is at ((u * dims[1] / 64 + s / 64) * 64 + s % 64) *
   dims[2] + w, and only rows below the index size are defined.  d_out: device,
   out_words >= dims[0] * dims[1] * dims[2], else HOPH_E_CAPACITY (dims are
   written either way).  Asynchronous on hip_stream. */
hoph_status hoph_index_code_planes(const hoph_index *index, uint32_t *d_out, uint64_t out_words, uint64_t dims[3],
                                   void *hip_stream);

/* hoph_index_rows -- copies the signatures of index rows first .. first + n - 1
   (uint32[n][k], row-major, the layout sketch_oph writes: the OPH bins of
   Sec. 3.2 or the hierarchical bins of Sec. 4.1) into d_out (device, caller-owned,
   n * k words).  HOPH_E_RANGE when first + n exceeds the index size.
   Asynchronous on hip_stream. */
hoph_status hoph_index_rows(const hoph_index *index, uint64_t first, uint64_t n, uint32_t *d_out,
                            void *hip_stream);

/* hoph_index_size -- number of sets in the index (0 for NULL). */
uint64_t hoph_index_size(const hoph_index *index);

/* hoph_index_free -- release the index and its device memory (NULL is a no-op). */
void hoph_index_free(hoph_index *index);

/*
 * query_goph -- Alg. 1 (GOPH): for each of n_q query signatures (d_qsigs,
 * n_q * k uint32 row-major, same params as the index), compare group by group
 * against every indexed set, group weights 1/L, stop under the small-probability
 * event (Def. 1) and accept iff the weighted estimate reaches T after the last
 * group.  Requires an index built with HOPH_LAYOUT_OPH.
 * Returns HOPH_E_CAPACITY (with results->needed) if capacity is too small;
 * HOPH_E_UNSUPPORTED if the exact state does not fit 64 bits.
 * Synchronises hip_stream (once in the usual case; again when the batch
 * accepted more pairs than the one-workgroup output stage sorts, or when a
 * buffer overflowed and the batch is redone); the CSR output is complete on
 * return.
 */
hoph_status query_goph(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                       const hoph_query_params *qp, hoph_results *results, void *hip_stream);

/* query_hoph -- Alg. 2 ((a:b) HOPH): as query_goph with group weights
   a b^(j-1)/(a+b)^j (last group (b/(a+b))^(L-1)).  Requires HOPH_LAYOUT_HIER. */
hoph_status query_hoph(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                       const hoph_query_params *qp, hoph_results *results, void *hip_stream);

/* query_hoph_noalloc -- query_hoph for callers that cannot allocate (code under
   HIP graph capture, tight serving loops, harnesses that forbid allocation):
   the same arguments, checks and results, but no device or pinned memory is
   allocated.  Its buffers beyond the inputs and outputs live in a 64 MiB
   device array that the library holds on each device it runs on until the
   process ends.  Limits, each refused with HOPH_E_CAPACITY and a message
   before anything runs or when reached: n_q <= 4096 queries; n_q * L <= 262,144
   per-group query masks; at most 2^20 accepted pairs per call (results->needed
   is set) and about 3.1 million first-pass survivors for any one query.  Calls
   on one device are serialised by the library (each finishes, stream
   synchronised, before the next starts); calls on different devices run
   independently.  Its pair counts and coarse-pass shape are not reported
   through hoph_query_counts or hoph_coarse_plan (they describe the index's own
   calls).  Synchronises hip_stream. */
hoph_status query_hoph_noalloc(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                               const hoph_query_params *qp, hoph_results *results, void *hip_stream);

/* query_oph_full -- plain OPH comparator (Eq. 6 over all k bins, no early stop):
   accept iff N_mb / (k - N_eb) >= T under qp->empty_policy (eps ignored). Any layout. */
hoph_status query_oph_full(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                           const hoph_query_params *qp, hoph_results *results, void *hip_stream);

/* MinWise comparator (Sec. 1-2): k independent hashes (a_i x + b_i) mod p. */
typedef struct {
    uint32_t k;               /* number of hash functions                                */
    uint32_t hash;            /* HOPH_HASH_MODP31 or HOPH_HASH_MODP32P15                 */
    uint64_t universe;
    const uint64_t *d_hash_a; /* device, k entries, 1 <= a_i < p                         */
    const uint64_t *d_hash_b; /* device, k entries, 0 <= b_i < p                         */
} hoph_minwise_params;

/* minwise_sketch -- d_sigs: n_sets * k uint64 row-major, each the minimum hash
   (UINT64_MAX for an empty set).  Asynchronous; errors as sketch_oph. */
hoph_status minwise_sketch(const hoph_minwise_params *params, const uint32_t *d_ids,
                           const uint64_t *d_offsets, uint64_t n_sets, uint64_t *d_sigs,
                           void *hip_stream);

/* minwise_query -- accept iff (#equal minima) / k >= T.  Synchronises once. */
hoph_status minwise_query(const hoph_minwise_params *params, const uint64_t *d_sigs,
                          uint64_t n_sets, const uint64_t *d_qsigs, uint32_t n_q, hoph_ratio T,
                          hoph_results *results, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Batched execution: persistent kernels, hipGraph replay, tuned tile shapes */
/* ------------------------------------------------------------------------ */

/* A plan answers batches of query *sets* against one index: sketch (chunked, so
   sets of 10 or 10,000 ids balance), per-group query masks, coarse and fine
   passes, per-query output -- every kernel reads the batch size from device
   memory, so one captured graph serves every batch up to the plan's capacities.
   Results are the same as sketch_oph followed by query_goph / query_hoph. */
typedef struct hoph_plan hoph_plan;

typedef struct {
    uint32_t kind;            /* 0: GOPH (Alg. 1, HOPH_LAYOUT_OPH index), 1: HOPH (Alg. 2)        */
    uint32_t max_queries;     /* query sets per batch (>= 1)                                      */
    uint64_t max_query_ids;   /* ids of all query sets of a batch                                 */
    uint64_t max_results;     /* accepted pairs per batch                                         */
    uint32_t use_graph;       /* 1: capture the pipeline once and replay it for every batch       */
    uint32_t tune;            /* 1: time candidate tile shapes on the first batch and keep the best */
} hoph_plan_config;

typedef struct {
    uint32_t q_per_wave;          /* queries per wavefront work item in the coarse pass      */
    uint32_t coarse_waves_per_cu; /* persistent coarse grid                                  */
    uint32_t sketch_chunk;        /* ids per sketch work item                                */
    uint32_t sketch_waves_per_cu; /* persistent sketch grid                                  */
    uint32_t depth;               /* coarse groups                                           */
    uint32_t graph;               /* 1 if batches replay a captured graph                    */
    uint32_t tuned;               /* 1 if the shapes came from timing (or the tuning cache)  */
    uint32_t fallbacks;           /* batches redone on the host-synchronised path            */
    float tune_ms;                /* the chosen shapes' time on the tuning batch             */
    uint32_t fallback_causes;     /* why, over all batches: 1 survivors past the plan's buffer,
                                     2 accepted pairs past its key buffer, 4 a query with more
                                     ids than the per-query sort takes                       */
    uint32_t reserved;
} hoph_plan_info;

/* hoph_plan_create -- allocate a plan (device buffers sized by cfg) for index
   and query parameters qp.  params must be the index's sketch parameters. */
hoph_status hoph_plan_create(hoph_index *index, const hoph_sketch_params *params,
                             const hoph_query_params *qp, const hoph_plan_config *cfg,
                             hoph_plan **out);

/* hoph_plan_run -- queue one batch of n_q query sets (device CSR; d_offsets[0] must
   be 0 and d_offsets[n_q] == n_ids) on hip_stream.  Asynchronous: no host
   synchronisation unless this is the first batch of a plan with tune = 1.
   HOPH_E_CAPACITY if n_q or n_ids exceed the plan. */
hoph_status hoph_plan_run(hoph_plan *plan, const uint32_t *d_ids, const uint64_t *d_offsets,
                          uint32_t n_q, uint64_t n_ids, void *hip_stream);

/* hoph_plan_results -- wait for the last batch and return its CSR (plan-owned device
   memory, valid until the next run): per query ascending set ids.  A batch that
   overflowed a device buffer or held a query with more than 4096 results is redone
   on the host-synchronised path, so the output is always exact.  HOPH_E_CAPACITY
   (with *n_results = pairs needed) if the batch has more than max_results pairs. */
hoph_status hoph_plan_results(hoph_plan *plan, const uint64_t **d_offsets,
                              const uint32_t **d_set_ids, uint64_t *n_results, void *hip_stream);

/* hoph_plan_query_sigs -- the OPH signatures (uint32[n_q][k], row-major, Sec. 3.2 /
   Sec. 4.1 bins) that the last batch's chunked sketch wrote: plan-owned device
   memory, valid until the next run, ordered after the batch on hip_stream (the
   caller synchronises that stream before reading it).  *n_q is the batch size.
   HOPH_E_INVAL when no batch has been run. */
hoph_status hoph_plan_query_sigs(const hoph_plan *plan, const uint32_t **d_qsigs, uint32_t *n_q);

hoph_status hoph_plan_get_info(const hoph_plan *plan, hoph_plan_info *info);
void hoph_plan_free(hoph_plan *plan);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of single-set queries                        */
/* ------------------------------------------------------------------------ */

/* A server keeps an index resident and answers single query sets submitted at
   any time.  Each of `slots` workers owns a plan and a stream: a free worker takes
   the waiting requests in arrival order while they fit its batch (queries and
   ids: the memory each slot reserves), runs them as one batch, and hands every
   request its own ascending result list; batches of different workers overlap on
   the device.  A request's result does not depend on the batch it rode in. */
typedef struct hoph_server hoph_server;

typedef struct {
    uint32_t kind;                /* 0: GOPH, 1: HOPH                                          */
    uint32_t slots;               /* concurrent batches (>= 1)                                  */
    uint32_t max_batch_queries;   /* requests per batch                                         */
    uint32_t use_graph;           /* replay a captured graph per batch                          */
    uint64_t max_batch_ids;       /* ids per batch; a request larger than this is refused       */
    uint64_t max_batch_results;   /* accepted pairs per batch                                   */
    uint64_t device_mem_budget;   /* bytes all slots may reserve (0: no limit); slots are
                                     dropped until the reservation fits, at least one stays    */
    uint32_t tune;                /* tune tile shapes at creation on one synthetic batch (up
                                     to 64 sets of up to 800 pseudo-random ids below the
                                     universe) and give them to every slot                   */
    uint32_t reserved;
} hoph_server_config;

typedef struct {
    uint64_t submitted, completed, rejected, batches, fallbacks, inserted_sets;
    double mean_ms, p50_ms, p99_ms, max_ms;   /* submit -> result ready, completed requests */
    double mean_batch_queries;
    double busy_s;                /* first submit to last completion                          */
    uint32_t slots;               /* slots that fit the memory budget                         */
    uint32_t reserved;
    uint64_t slot_bytes;          /* device bytes one slot reserves                            */
} hoph_server_stats;

/* hoph_server_create -- slots (plans, streams, pinned staging) and the insert
   staging are allocated, tuned and graph-captured here, so that no request or
   insert waits for an allocation, a tuning or a capture. */
hoph_status hoph_server_create(hoph_index *index, const hoph_sketch_params *params,
                               const hoph_query_params *qp, const hoph_server_config *cfg,
                               hoph_server **out);
/* hoph_server_submit -- enqueue one query set (host ids, copied); *ticket identifies it.
   HOPH_E_CAPACITY if the set alone exceeds a batch. */
hoph_status hoph_server_submit(hoph_server *srv, const uint32_t *h_ids, uint64_t n_ids,
                               uint64_t *ticket);
/* hoph_server_wait -- block until the request is answered; copy up to cap set ids to
   h_out (ascending) and write the count to *n_out (HOPH_E_CAPACITY if cap is too
   small; the request stays available).  Returns the request's status. */
hoph_status hoph_server_wait(hoph_server *srv, uint64_t ticket, uint32_t *h_out, uint64_t cap,
                             uint64_t *n_out);
/* hoph_server_poll -- as wait without blocking: *done = 1 when answered, else 0. */
hoph_status hoph_server_poll(hoph_server *srv, uint64_t ticket, int32_t *done, uint32_t *h_out,
                             uint64_t cap, uint64_t *n_out);
/* hoph_server_insert -- sketch n_sets host sets (CSR) and append them to the index
   (ids continue the index), in pieces of at most 65,536 sets and max(max_batch_ids,
   2^20) ids through staging allocated at creation; each piece is visible to
   batches dispatched after it is sketched, all of them when the call returns.
   HOPH_E_CAPACITY past the index capacity or for a set larger than a piece
   (nothing is inserted then); HOPH_E_INVAL for decreasing offsets. */
hoph_status hoph_server_insert(hoph_server *srv, const uint32_t *h_ids, const uint64_t *h_offsets,
                               uint64_t n_sets);
/* hoph_server_replay -- native load generator: submit request i (host CSR) at
   arrival_s[i] seconds after the call, then wait for all.  With result_offsets
   (n_requests + 1 entries) and result_ids (result_cap entries) the results are
   returned in request order (HOPH_E_CAPACITY if result_cap is too small). */
hoph_status hoph_server_replay(hoph_server *srv, const uint32_t *h_ids, const uint64_t *h_offsets,
                               uint64_t n_requests, const double *arrival_s,
                               uint64_t *result_offsets, uint32_t *result_ids, uint64_t result_cap);
hoph_status hoph_server_stats_get(hoph_server *srv, hoph_server_stats *stats);
hoph_status hoph_server_reset_stats(hoph_server *srv);
void hoph_server_destroy(hoph_server *srv);

/* hoph_sync -- synchronise hip_stream and report (then clear) the device error
   flags raised by earlier sketches on the current device. */
hoph_status hoph_sync(void *hip_stream);

const char *hoph_status_str(hoph_status status);
const char *hoph_last_error(void);    /* thread-local; "" when none */

/* ------------------------------------------------------------------------ */
/* Host-only helpers (no GPU needed)                                         */
/* ------------------------------------------------------------------------ */

/* hoph_layout_starts -- the first permuted value of each bin, starts[0..k), and
   starts[k] = R (Sec. 3.2 / Sec. 4.1).  starts: host array of k + 1 entries. */
hoph_status hoph_layout_starts(const hoph_sketch_params *params, uint64_t *starts);

/* hoph_layout_lookups -- which bin lookups the sketch kernels may use for this
   layout (a test hook, so that tests can tell which ones hoph_selftest_bins
   cross-checks): bit 0 the uniform bin estimate, bit 1 log-domain region cells,
   bit 2 power-of-two regions and bins.  The (a x + b) mod (2^31 - 1) kernels take
   the first that applies of power-of-two, estimate, cells, region search; the
   other hashes the estimate or the region search.  *mask: host. */
hoph_status hoph_layout_lookups(const hoph_sketch_params *params, uint32_t *mask);

/* hoph_tail_integers -- for X ~ Bin(n, T) (Eq. 10): *j_lo = max{j >= -1 : P(X <= j) <= eps},
   *j_hi = min{j <= n + 1 : P(X >= j) <= eps}, computed exactly.  n <= 256. */
hoph_status hoph_tail_integers(uint32_t n, hoph_ratio T, hoph_ratio eps, int32_t *j_lo,
                               int32_t *j_hi);

/* The exact decision tables the scan applies (Alg. 1/2 with Def. 1).  With
   lcm = lcm(1..k_group) and the group weights as integers W_j over wsum, the state
   after group l is S~_l = sum_{j<=l} W_j * rho_j, rho_j = lcm * rate_j; the pair is
   accepted at step l iff S~_l >= acc[l-1] and rejected iff S~_l <= rej[l-1]. */
typedef struct {
    uint32_t L, k_group, empty_policy, goph;
    int32_t j_lo, j_hi;
    int64_t lcm;              /* lcm(1..k_group)                                         */
    int64_t wsum;             /* sum of W                                                */
    int64_t W[64];
    int64_t acc[64];
    int64_t rej[64];
    int64_t dmul[65];         /* lcm / (k_group - e) for e < k_group; lcm at e = k_group */
} hoph_decision_tables;

/* hoph_build_decision_tables -- the tables for an index layout (params) and a
   query (qp); goph = 1 for GOPH weights, 0 for HOPH weights. */
hoph_status hoph_build_decision_tables(const hoph_sketch_params *params,
                                       const hoph_query_params *qp, uint32_t goph,
                                       hoph_decision_tables *out);

/* hoph_first_group_plan -- the shape the first-group code pass takes for an
   index layout (params) and a query (qp, JOINT or LITERAL; goph as for
   hoph_build_decision_tables), without a GPU: tri = 1 for a self-join,
   small_batch = 1 for a host batch of fewer than 32 queries, keep_rate (host,
   nullable; entries 2..6 read) the fraction of row pairs phase 1 keeps at 2..6
   planes as measured on the data (a self-join samples it).  out (host):
   out[0] the planes compared first (0: one phase over all 8), out[1] 1 when
   the kernel holds only those planes in registers (HOPH_PLAN_FIRST_GROUP_LIGHT),
   out[2] tiles of 64 sets per wavefront.  A test hook for the expected-cost
   choice; a query uses it when its coarse pass stops after the first group. */
hoph_status hoph_first_group_plan(const hoph_sketch_params *params, const hoph_query_params *qp,
                                  uint32_t goph, uint32_t tri, uint32_t small_batch,
                                  const double *keep_rate, uint32_t out[3]);

/* hoph_selftest_bins -- runs the library's own hash-and-bin arithmetic (the code
   the sketch kernel inlines) on the host for n ids: out_bin[i], out_off[i].  Both
   bin lookups are run where the layout admits the uniform estimate, and a
   disagreement is HOPH_E_UNSUPPORTED.  A test hook for checking that arithmetic
   without a GPU. */
hoph_status hoph_selftest_bins(const hoph_sketch_params *params, const uint32_t *h_perm,
                               const uint32_t *h_ids, uint64_t n, uint32_t *out_bin,
                               uint32_t *out_off);

/*
 * hoph_self_join -- near-duplicate detection inside the collection (the query of
 * Sec. 3.3 with q taken from the collection itself): every pair of index rows
 * i < j that the grouped (OPH-layout index, Alg. 1) or hierarchical (HIER index,
 * Alg. 2) comparison accepts, as CSR over the rows: for row i, the ascending j > i
 * in d_set_ids[d_offsets[i] .. d_offsets[i+1]); d_offsets has size + 1 entries.
 * The decision is symmetric, so the pair (j, i) is not repeated.  Errors and
 * capacity reporting as for query_hoph.  Synchronises the stream (on the first
 * call with given parameters, and after the index size changes twofold, also
 * once to read 512 rows' first code planes back, whose pair agreement picks the
 * coarse kernel; hoph_coarse_plan reports the choice).
 */
hoph_status hoph_self_join(const hoph_index *index, const hoph_query_params *qp,
                           hoph_results *results, void *hip_stream);

/*
 * hoph_pair_estimates -- the similarity estimate of n_pairs pairs over their
 * whole signatures, to report with accepted pairs (d_pairs[2i] = query row < n_q
 * of d_qsigs, d_pairs[2i+1] = set id < index size; device, uint32):
 *  - d_est[i] (int64): the weighted sum of group rates, Lemma 3 for an a:b HOPH
 *    index and the mean of the group rates for a GOPH (OPH layout) index, exactly,
 *    as an integer over *denominator (written on return, host);
 *  - d_mb[i], d_eb[i] (uint32): matched and empty bins over all k bins (Eq. 1-4
 *    under empty_policy), so that Eq. 6 is d_mb / (k - d_eb);
 *  - d_var[i] (double): Eq. 8 with the observed 1/(k - N_eb) in place of its
 *    expectation, R = the Eq. 6 estimate and g = d_unions[i] = |D1 u D2| (device,
 *    nullable: then the large-g limit R (1 - R) / (k - N_eb)).
 * A pair out of range gets d_est = -1, d_mb = d_eb = 0xFFFFFFFF and a NaN variance.
 * HOPH_E_UNSUPPORTED where the exact state does not fit (as for queries).
 * Asynchronous on hip_stream.
 */
hoph_status hoph_pair_estimates(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                                const uint32_t *d_pairs, uint64_t n_pairs, uint32_t empty_policy,
                                const double *d_unions, int64_t *d_est, uint32_t *d_mb, uint32_t *d_eb,
                                double *d_var, int64_t *denominator, void *hip_stream);

/* hoph_pair_counts -- per-group counts (m_j, e_j) under policy for n_pairs pairs
   (d_pairs[2i] = query row < n_q, d_pairs[2i+1] = set id < index size) against the
   index: d_m and d_e are n_pairs * L uint32, device; a pair out of range gets
   0xFFFFFFFF in every group.  A test hook for the device counting.  Synchronises. */
hoph_status hoph_pair_counts(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                             const uint32_t *d_pairs, uint64_t n_pairs, uint32_t policy,
                             uint32_t *d_m, uint32_t *d_e, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HOPH_H */
