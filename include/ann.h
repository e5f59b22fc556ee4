/*
 * ann.h - C ABI of the MI355X (gfx950) library for search over an augmented
 * neighborhood graph: an exact kNN graph over the reference vectors plus a
 * bridge graph from Cartesian-concatenated codebook vectors
 * (Wang et al., "Fast Neighborhood Graph Search using Cartesian
 * Concatenation", arXiv:1312.3062).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Every call declared to return int returns a value of ann_status:
 *    ANN_OK (0) or a negative error code (int rather than the enum type, so
 *    that the return width is fixed for foreign-function callers).  No
 *    exception crosses the ABI.  ann_last_error() returns a thread-local
 *    message describing the last failure of the calling thread.
 *  - On error the index passed in is unchanged and output buffers hold
 *    undefined contents.
 *  - "host" pointers point to CPU memory, "device" pointers (d_ prefix) to
 *    memory on the GPU that holds the index.  All pointers are borrowed for
 *    the duration of the call only.
 *  - Distances are SQUARED Euclidean distances (the paper stores the square
 *    of the distance, Sec. 3.2 and Sec. 4.2).  For ANN_U8 data they are
 *    exact int32 values; for ANN_F32 data they are float.
 *  - Result rows hold `k` entries ascending by (distance, id).  When fewer
 *    than k vectors were evaluated the row is padded with id -1 and
 *    distance INT32_MAX (u8) or +infinity (f32).
 *  - Every order and every tie is resolved by the total order on
 *    (distance, node id).  A bridge vector with linear id lid has node id
 *    n + lid, so at equal distance a reference vector comes first.
 *  - The index is read-only after it is built; searches on different
 *    streams may run concurrently on one index.
 *  - Results depend only on (index, query, k, budget, queue_len,
 *    precision): never on batch composition, launch shape or tuning.
 */
#ifndef ANN_H
#define ANN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ann_index ann_index; /* opaque; owned by the library */

typedef enum { ANN_U8 = 0, ANN_F32 = 1 } ann_dtype;

typedef enum {
    ANN_OK = 0,
    ANN_EINVAL = -1,       /* invalid argument (null pointer, bad size, dtype mismatch) */
    ANN_ENOMEM = -2,       /* device or host allocation failed */
    ANN_EDEVICE = -3,      /* a HIP call failed */
    ANN_ESTATE = -4,       /* object in the wrong state */
    ANN_EUNSUPPORTED = -5, /* valid request outside what the library implements */
    ANN_EIO = -6,          /* file could not be read or written */
    ANN_ERESOURCE = -7     /* a per-query structure outgrew its capacity */
} ann_status;

/* Search precision for ANN_F32 indexes.  u8 indexes are always exact. */
typedef enum {
    ANN_PRECISION_EXACT = 0,      /* fp32 distances from the fp32 rows */
    ANN_PRECISION_BF16_RERANK = 1 /* bf16 copies drive the search; final top
                                     rerank_k re-ranked from the fp32 rows */
} ann_precision;

/*
 * Index build parameters (Sec. 4.1 "Data structure").
 *  graph_k      R, out-degree of the exact kNN graph (row i = the R nearest
 *               j != i, ascending by (distance, j)).  0 builds no graph.
 *  P, K         P subspaces of d/P contiguous dims (P divides d); K codewords
 *               per subspace; K^P bridge vectors.  1 <= P <= 4, 1 <= K <= 256,
 *               n + K^P < 2^32.
 *  kmeans_iters Lloyd iterations per subspace (assign, then update).  The K
 *               initial rows are the first K entries of a Fisher-Yates
 *               shuffle of [0, n) driven by SplitMix64(seed); ties in
 *               assignment go to the smaller codeword; u8 centroids are the
 *               member mean rounded half up; empty clusters keep their
 *               centroid.
 *  bridge_t     each reference vector is linked from its bridge_t nearest
 *               bridge vectors (by (distance, lid)).
 *  bridge_b     each bridge vector keeps its bridge_b nearest linked
 *               references (by (distance, id)); 0 keeps all.
 */
typedef struct {
    uint32_t struct_size; /* sizeof(ann_build_params) */
    int32_t graph_k;
    int32_t P;
    int32_t K;
    int32_t kmeans_iters;
    int32_t bridge_t;
    int32_t bridge_b;
    int32_t reserved; /* must be 0 */
    uint64_t seed;
} ann_build_params;

/*
 * Search parameters (Alg. 1).
 *  queue_len  L, capacity of the main queue of reference vectors
 *             (1 <= L <= 64).  When the queue is full a new candidate
 *             evicts the worst entry if it is better, else it is dropped
 *             (it stays visited and in the result set).  The single bridge
 *             vector of the paper's main queue is held in its own slot.
 *  precision  ann_precision (ignored for u8).
 *  rerank_k   ANN_PRECISION_BF16_RERANK only: how many of the best bf16
 *             candidates are re-ranked in fp32 (0 means k).
 * Launch tuning (results never depend on these; 0 = library default):
 *  lookahead     queue entries whose kNN rows are loaded and whose
 *                neighbours are measured together, 1..8 (default: as many
 *                as 64 lanes hold, 64 / graph_k).
 *  persistent    1: a grid of resident wavefronts drains a device work
 *                counter instead of one workgroup per query.
 *  waves_per_cu  persistent only: resident wavefronts per compute unit
 *                (default: as many as fit).
 *  order         persistent with per-query budgets: 1 serves the queries
 *                in descending budget (powers of two), longest first.
 * A caller built against the first version (struct_size 16, no tuning
 * fields) is accepted and gets the defaults.
 */
typedef struct {
    uint32_t struct_size; /* sizeof(ann_search_params) */
    int32_t queue_len;
    int32_t precision;
    int32_t rerank_k;
    int32_t lookahead;
    int32_t persistent;
    int32_t waves_per_cu;
    int32_t order;
} ann_search_params;

typedef struct {
    int64_t n;                /* reference vectors */
    int32_t d;                /* dimension */
    int32_t dtype;            /* ann_dtype */
    int32_t P, K;             /* subspaces, codewords per subspace */
    int32_t graph_k;          /* R */
    int32_t reserved;
    int64_t n_bridges;        /* K^P */
    int64_t n_bridge_entries; /* E, total length of all bridge lists */
    int64_t device_bytes;     /* device memory owned by the index */
} ann_index_info;

/* Per-query counters written by ann_search_device when d_stats is given
 * (nq x ANN_NSTATS int32, row-major). */
enum {
    ANN_STAT_EVALS = 0,        /* distance evaluations t (<= budget) */
    ANN_STAT_REF_POPS = 1,     /* reference vectors expanded (kNN rows read) */
    ANN_STAT_BRIDGE_POPS = 2,  /* non-empty bridge vectors expanded */
    ANN_STAT_BRIDGE_IDS = 3,   /* bridge-list entries read */
    ANN_STAT_BRIDGES_GEN = 4,  /* bridges extracted by the multi-sequence,
                                  empty ones and look-ahead included */
    ANN_STAT_HEAP_MAX = 5,     /* largest multi-sequence frontier */
    ANN_STAT_FLAGS = 6,        /* 0, or ANN_ERESOURCE if a structure overflowed */
    ANN_STAT_ROWS = 7,         /* vector rows gathered, look-ahead included */
    ANN_STAT_LOOKAHEADS = 8,   /* batches of kNN rows loaded ahead */
    ANN_STAT_RERUN = 9,        /* 1 if the query was searched again by the re-run kernel
                                  (its multi-sequence outgrew LDS and no global slot was
                                  free) */
    ANN_STAT_MOVED = 10,       /* 1 if the multi-sequence outgrew LDS and carried on in a
                                  global slot of the workspace */
    ANN_NSTATS = 12            /* 11 reserved, written as 0 */
};

/* ------------------------------------------------------------------ */
/* Index construction                                                  */
/* ------------------------------------------------------------------ */

/*
 * Build the index on the current HIP device (Sec. 4.1): copy X to the
 * device, train the codebooks (k-means per subspace), build the exact kNN
 * graph and the bridge graph.
 *  data       host, n x d row-major, uint8 (ANN_U8) or float (ANN_F32).
 *  codebooks  host, optional: P x K x (d/P) of the data dtype.  When given
 *             no k-means runs and these codewords are used as they are.
 *  graph      host, optional: n x graph_k uint32 kNN rows to use instead of
 *             building them (each row: ids in [0, n), no repeats).
 *  out        receives the new index; free it with ann_index_free.
 * Errors: ANN_EINVAL (null data/out/params, n < 1, d < 1, P does not divide
 * d, K out of range, K > n when training, n + K^P >= 2^32, bridge_t < 1,
 * bridge_b < 0, graph_k < 0 or >= n, u8 rows not a multiple of 16 bytes,
 * f32 d not a multiple of 4), ANN_ENOMEM, ANN_EDEVICE.
 */
int ann_build_index(const void* data, int64_t n, int32_t d, int32_t dtype, const ann_build_params* params,
                    const void* codebooks, const uint32_t* graph, ann_index** out);

/*
 * Assemble an index from given parts (host arrays) without building any of
 * them; used to search an index built elsewhere.
 *  data        n x d (dtype); codebooks P x K x (d/P) (dtype);
 *  graph       n x graph_k uint32 (may be null when graph_k == 0);
 *  bridge_off  K^P + 1 uint32 offsets, bridge_off[0] = 0, non-decreasing;
 *  bridge_ids  bridge_off[K^P] uint32 reference ids; list lid is
 *              bridge_ids[bridge_off[lid] .. bridge_off[lid+1]).
 * Lists and graph rows must not repeat an id.
 * Errors: ANN_EINVAL on inconsistent sizes or ids out of range.
 */
int ann_index_import(const void* data, int64_t n, int32_t d, int32_t dtype, int32_t P, int32_t K,
                     const void* codebooks, int32_t graph_k, const uint32_t* graph, const uint32_t* bridge_off,
                     const uint32_t* bridge_ids, ann_index** out);

int ann_index_get_info(const ann_index* idx, ann_index_info* info);

/*
 * Copy index parts to host buffers sized from ann_index_get_info; each
 * pointer may be null to skip that part.  codebooks P x K x (d/P) (dtype),
 * graph n x graph_k, bridge_off K^P + 1, bridge_ids n_bridge_entries.
 */
int ann_index_export(const ann_index* idx, void* codebooks, uint32_t* graph, uint32_t* bridge_off,
                     uint32_t* bridge_ids);

/* Write / read a versioned binary file holding the whole index. */
int ann_index_save(const ann_index* idx, const char* path);
int ann_index_load(const char* path, ann_index** out);

void ann_index_free(ann_index* idx);

/* ------------------------------------------------------------------ */
/* Search (Sec. 4.2, Alg. 1)                                           */
/* ------------------------------------------------------------------ */

/*
 * Best-first search over the augmented graph for nq queries.
 * For each query: subspace distance tables and their sort, multi-sequence
 * extraction of bridge vectors in increasing distance, then Alg. 1 with a
 * strict budget of `budget` distance evaluations.
 *  queries  host, nq x d (index dtype).
 *  k        1..1024 results per query; budget >= 0.
 *  ids      host, nq x k int32.  dists host, nq x k (int32 for u8, float
 *           for f32).
 * Synchronous.  Errors: ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE, ANN_ERESOURCE.
 */
int ann_search(const ann_index* idx, const void* queries, int64_t nq, int32_t k, int32_t budget,
               const ann_search_params* params, int32_t* ids, void* dists);

/*
 * Device form of ann_search, asynchronous on `stream` (a hipStream_t, may
 * be null for the default stream).  All buffers are device memory.
 *  d_k, d_budget  optional per-query k and budget (int32, nq each); when
 *                 given, each entry must lie in [1, k] and [0, budget].
 *                 k and budget are then the maxima: row stride of the
 *                 outputs and the size of per-query structures.
 *  d_ids, d_dists nq x k outputs (row stride k).
 *  d_stats        optional nq x ANN_NSTATS int32 counters.
 *  d_trace        optional nq x budget int32: the ids in evaluation order,
 *                 padded with -1.
 * A query whose multi-sequence frontier outgrows its capacity gets flag
 * ANN_ERESOURCE in d_stats and a row of -1; ann_search reports it as an
 * error.
 */
int ann_search_device(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                      const int32_t* d_k, const int32_t* d_budget, const ann_search_params* params,
                      int32_t* d_ids, void* d_dists, int32_t* d_stats, int32_t* d_trace, void* stream);

/*
 * Device workspace for ann_search_device_ws and this request (bytes): the
 * per-query lists, global slots for multi-sequence state that outgrows LDS
 * (one per query that can be resident, never more than the batch's queries
 * or 512 MB) and, for a budget whose visited set does not fit a
 * workgroup's LDS (beyond about 31,000 evaluations), one visited bitmap of
 * n bits per workgroup of that budget class (at most 1 GB of them).
 */
int ann_search_workspace_size(const ann_index* idx, int64_t nq, int32_t k, int32_t budget,
                              const ann_search_params* params, int64_t* bytes);

/*
 * ann_search_device with a caller-provided device workspace (16-byte aligned):
 * the call allocates nothing, so it can be captured into a graph and
 * replayed.  The workspace is owned by the caller and must not be shared by
 * launches that overlap in time.  A workspace smaller than
 * ann_search_workspace_size holds fewer global slots (at least one must
 * fit, else ANN_EINVAL); queries that find no free slot are searched again
 * by a second kernel, with the same results.
 */
int ann_search_device_ws(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                         const int32_t* d_k, const int32_t* d_budget, const ann_search_params* params,
                         int32_t* d_ids, void* d_dists, int32_t* d_stats, int32_t* d_trace, void* workspace,
                         int64_t workspace_bytes, void* stream);

/*
 * Neighborhood-graph search without the bridge graph (Sec. 2.2, the
 * iterative search that Sec. 5.3 compares against): the seed vectors are
 * measured first, in the given order (a repeated seed is measured once),
 * then the main queue is expanded best first over the kNN graph exactly as
 * in Alg. 1, with no bridge vector ever in the queue.  The budget counts
 * the seeds' distance evaluations too.
 *  d_seeds  device, n_seeds int32 reference ids in [0, n), the same for every
 *           query (an id outside [0, n) is skipped); 0 <= n_seeds <= 2^20.
 * Other arguments as ann_search_device (one k and budget for the batch;
 * exact precision only).  In d_stats the seed list counts as one bridge pop
 * of n_seeds entries.  Asynchronous on `stream`.
 * Errors: ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE.
 */
int ann_search_graph_device(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                            const int32_t* d_seeds, int32_t n_seeds, const ann_search_params* params,
                            int32_t* d_ids, void* d_dists, int32_t* d_stats, int32_t* d_trace, void* stream);

/*
 * ann_search_device that allocates nothing, for callers that cannot call
 * hipMalloc: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Its workspace is a buffer of
 * ANN_NOALLOC_SCRATCH_BYTES compiled into the library: one copy on each GPU
 * the library runs on, held until the process ends.  Same arguments, results
 * and asynchrony as ann_search_device.
 * Errors: as ann_search_device; ANN_EINVAL when the request's smallest
 * workspace (per-query lists of about 8 bytes a query, one multi-sequence
 * slot and, for budgets beyond LDS, one visited bitmap of n bits) exceeds
 * the buffer: search fewer queries per call.
 * Every call on a GPU uses that GPU's one buffer: calls that overlap in time
 * on one GPU (other streams, other threads) race and must not be made.
 */
#define ANN_NOALLOC_SCRATCH_BYTES (64u << 20)
int ann_search_device_noalloc(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                              const int32_t* d_k, const int32_t* d_budget, const ann_search_params* params,
                              int32_t* d_ids, void* d_dists, int32_t* d_stats, int32_t* d_trace, void* stream);

/*
 * Launch autotuner: times the launch-tuning choices of ann_search_params
 * (lookahead, persistent, waves_per_cu, order) on the given device batch
 * and writes the fastest into *params; the other fields are kept.  Every
 * candidate runs twice; the three fastest and the default are then timed
 * five more times each, in turn, and the lowest median wins.  Every
 * candidate must return the same ids; a difference is reported as
 * ANN_ESTATE.  Allocates two nq x k output buffers for the duration of the
 * call.  Synchronous on `stream`.
 */
int ann_autotune(const ann_index* idx, const void* d_queries, int64_t nq, int32_t k, int32_t budget,
                 const int32_t* d_k, const int32_t* d_budget, ann_search_params* params, void* stream);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching over a device-resident index           */
/* ------------------------------------------------------------------ */

/*
 * A request server: requests (a batch of query vectors with their own k and
 * budget, each query searched by Alg. 1 as in ann_search) are queued by
 * ann_server_submit and served by micro-batch launches on `slots` streams.
 * Whenever a slot is free, pending requests are taken in arrival order into
 * one micro-batch while its footprint fits:
 *  - device memory: the micro-batch's query rows, k and budget per query,
 *    result rows and search workspace are one chunk of a device arena of
 *    `device_bytes`, beside the chunks of the micro-batches in flight;
 *  - LDS: each query, while resident on a compute unit, occupies the LDS
 *    layout of its budget class (ann_server_footprint); the queries in
 *    flight hold at most `lds_rounds` times the chip's LDS.
 * Requests arriving while others run are admitted as slots and memory free
 * up; their launches overlap on the device.  Results are those of
 * ann_search for each query: independent of the mix.
 * A server is driven by one thread; it switches to the index's device
 * inside each call and back.
 */
typedef struct ann_server ann_server;

typedef struct {
    uint32_t struct_size;     /* sizeof(ann_server_params) */
    int32_t slots;            /* micro-batches in flight at once, 1..16 */
    int32_t slot_queries;     /* most queries in one micro-batch (and in one request) */
    int32_t kmax;             /* largest k of a request, 1..1024 */
    int32_t max_budget;       /* largest budget of a request */
    int32_t lds_rounds;       /* LDS in flight, in multiples of the chip's LDS (0: 2) */
    int64_t device_bytes;     /* device arena (0: `slots` full micro-batches) */
    ann_search_params search; /* queue length, precision, launch tuning */
} ann_server_params;

typedef struct {
    int64_t pending;          /* requests waiting for admission */
    int64_t busy_slots;       /* micro-batches in flight */
    int64_t launches;         /* micro-batches launched so far */
    int64_t lds_in_flight, lds_limit;          /* bytes */
    int64_t device_in_flight, device_bytes;    /* bytes of the arena */
} ann_server_info;

/*
 * Create a server over idx (which must outlive it).  Allocates the device
 * arena and pinned host staging for each slot.
 * Errors: ANN_EINVAL (bad parameters, an arena smaller than one full
 * micro-batch, one query at max_budget needing more LDS than the chip),
 * ANN_ENOMEM, ANN_EDEVICE.
 */
int ann_server_create(const ann_index* idx, const ann_server_params* params, ann_server** out);

/* LDS (while resident) and device bytes of a request of nq queries. */
int ann_server_footprint(const ann_server* server, int32_t nq, int32_t k, int32_t budget, int64_t* lds_bytes,
                         int64_t* device_bytes);

/*
 * Queue a request: queries host, nq x d (index dtype), copied before the
 * call returns.  *ticket identifies it.  Pending requests are admitted
 * here and in ann_server_progress.
 * Errors: ANN_EINVAL (nq outside 1..slot_queries, k above kmax, budget
 * above max_budget, an LDS footprint the server can never admit),
 * ANN_EDEVICE.
 */
int ann_server_submit(ann_server* server, const void* queries, int32_t nq, int32_t k, int32_t budget,
                      int64_t* ticket);

/*
 * Retire finished micro-batches and admit pending requests; never blocks.
 * Writes up to `cap` tickets of requests completed since the last call to
 * done[] and their count to *n_done.
 */
int ann_server_progress(ann_server* server, int64_t* done, int32_t cap, int32_t* n_done);

/*
 * Results of a completed request: ids host nq x k int32, dists host nq x k
 * (int32 for u8, float for f32), as ann_search writes them.  The ticket is
 * released.  Errors: ANN_EINVAL (unknown ticket), ANN_ESTATE (not done).
 */
int ann_server_result(ann_server* server, int64_t ticket, int32_t* ids, void* dists);

/* Block until every submitted request has completed. */
int ann_server_drain(ann_server* server);

int ann_server_get_info(const ann_server* server, ann_server_info* info);

/* Wait for the micro-batches in flight, then free everything. */
void ann_server_destroy(ann_server* server);

/* ------------------------------------------------------------------ */
/* Graph-D-ADC: the search as the inverted-list lookup of IVFADC       */
/* ------------------------------------------------------------------ */

/*
 * The paper's billion-scale system (Sec. 5): a vocabulary of coarse centres
 * indexed by the augmented neighborhood graph; each vector belongs to the
 * inverted list of the centre the graph search returns for it (k = 1), and
 * its residual to that centre is encoded by product quantisation (pq_m
 * subspaces of d / pq_m dims, 256 codewords each, one byte per subspace).
 * A query searches the centres for its nearest lists and re-ranks their
 * vectors by the asymmetric distance |q - c - r|^2, r the residual's
 * codewords concatenated.
 */
typedef struct ann_ivf ann_ivf;

typedef struct {
    uint32_t struct_size;       /* sizeof(ann_ivf_params) */
    int32_t lists;              /* C coarse centres: a seeded sample of the vectors (the first C of a
                                   SplitMix64-driven Fisher-Yates shuffle of [0, n) from `seed`) */
    int32_t pq_m;               /* bytes per vector: 8 or 16, dividing d */
    int32_t pq_iters;           /* k-means iterations of the residual codebooks (initial codewords: the
                                   residuals of 256 rows drawn the same way from seed + 1) */
    int32_t assign_budget;      /* budget of the search assigning each vector to its list */
    int32_t reserved;           /* must be 0 */
    uint64_t seed;
    ann_build_params centres;   /* the augmented index over the centres */
} ann_ivf_params;

typedef struct {
    int64_t n;
    int32_t d, lists, pq_m, reserved;
    int64_t device_bytes;       /* lists, codes, the per-vector constants and codebooks (the centres'
                                   index excluded) */
} ann_ivf_info;

/*
 * Build from host data (n x d uint8, 256 <= n < 2^31) on the current device.
 * Errors: ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE, ANN_ERESOURCE (a vector found
 * no list within assign_budget).
 */
int ann_ivf_build(const void* data, int64_t n, int32_t d, const ann_ivf_params* params, ann_ivf** out);

int ann_ivf_get_info(const ann_ivf* ivf, ann_ivf_info* info);

/* The augmented index over the centres (owned by the ivf). */
const ann_index* ann_ivf_centres(const ann_ivf* ivf);

/*
 * Host copies (each pointer may be null): centres lists x d; list_off
 * lists + 1 (list j holds positions list_off[j] .. list_off[j+1]); list_ids
 * n vector ids in list order (a list in increasing id); codes n x pq_m in
 * list order; pq_codebooks pq_m x 256 x (d / pq_m) float.
 */
int ann_ivf_export(const ann_ivf* ivf, uint8_t* centres, uint32_t* list_off, uint32_t* list_ids, uint8_t* codes,
                   float* pq_codebooks);

/*
 * For each query: the `lists` nearest centres by the graph search (budget
 * centre_budget, queue length 64), then the vectors of those lists, lists by
 * increasing centre distance and each list in its order, up to `candidates`
 * of them (the scan stops mid-list when they are reached), ranked by the
 * asymmetric distance (fp32).  d_ids nq x k int32, d_dists nq x k float,
 * ascending by (distance, id), padded with -1 / +infinity.  1 <= k <= 1024,
 * 1 <= lists <= 1024.  Asynchronous on `stream`; the lists of the batch
 * (nq x lists ids and distances) live in a stream-ordered allocation freed
 * on the same stream.  Errors: ANN_EINVAL, ANN_EUNSUPPORTED (the distance
 * tables of this d and pq_m exceed a workgroup's LDS), ANN_EDEVICE.
 */
int ann_ivf_search_device(const ann_ivf* ivf, const void* d_queries, int64_t nq, int32_t k, int32_t lists,
                          int32_t centre_budget, int32_t candidates, int32_t* d_ids, float* d_dists, void* stream);

void ann_ivf_free(ann_ivf* ivf);

/*
 * Query preprocessing alone (Sec. 4.2): for each query the P x K squared
 * distances to the codewords, each subspace sorted ascending by
 * (value, codeword index).  d_sorted nq x P x K (int32 for u8, float for
 * f32); d_perm nq x P x K int32 codeword of each rank.  Asynchronous.
 */
int ann_query_tables_device(const ann_index* idx, const void* d_queries, int64_t nq, void* d_sorted,
                            int32_t* d_perm, void* stream);

/*
 * Exact k nearest neighbours by linear scan (the ground truth of Sec. 5.1).
 *  d_x n x d, d_q nq x d (dtype); exclude_self != 0 means query i is row i
 *  of d_x and is left out of its own list (the kNN graph).  Outputs nq x k
 *  ascending by (distance, id).  Asynchronous.
 */
int ann_knn_device(const void* d_x, int64_t n, int32_t d, int32_t dtype, const void* d_q, int64_t nq, int32_t k,
                   int32_t exclude_self, int32_t* d_ids, void* d_dists, void* stream);

/* Thread-local message of the last error; never null. */
const char* ann_last_error(void);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int ann_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ANN_H */
