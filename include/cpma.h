/*
 * cpma.h -- C ABI of the MI355X (gfx950) compressed packed memory array.
 *
 * A CPMA is a pointer-free sorted set of 64-bit keys (Wheatman, Burns, Bulu\c{c},
 * Xu, "CPMA: An Efficient Batch-Parallel Compressed Set Without Pointers",
 * PPoPP'24).  Keys live in fixed-size leaves of an implicit binary tree; a leaf
 * stores its first key (the head) uncompressed and the following keys as
 * delta-encoded byte codes packed to the left (Section "Compressed Packed
 * Memory Array", "CPMA structure").  Every node of the implicit tree keeps its
 * byte density between height-dependent bounds (Section "Packed Memory
 * Array", "Design and operations"); batch updates merge into leaves, count
 * densities level by level and redistribute the violating regions (Section
 * "Parallel Batch Updates in a PMA").
 *
 * All state lives in device memory of the GPU that is current when the set is
 * built.  Every call takes a HIP stream (hipStream_t passed as void*, NULL =
 * the null stream) and enqueues its work there.
 *
 * Conventions shared by every entry point:
 *   - Key domain: [0, 2^64 - 2].  UINT64_MAX is reserved and a key equal to it
 *     is rejected with CPMA_ERR_RESERVED_KEY before anything is modified.
 *   - Memory spaces: `mem` says whether the key / query / output pointers of a
 *     call are host memory (CPMA_MEM_HOST) or device memory of the set's GPU
 *     (CPMA_MEM_DEVICE).  Inputs are only read during the call.  Outputs
 *     written to host memory, and the host out-parameters n_added / n_removed,
 *     are complete when the call returns (the call synchronises the stream);
 *     outputs written to device memory are complete when the stream reaches
 *     the point after the call.
 *   - Ownership: the handle owns all device memory it allocates (leaves,
 *     heads, used counts, scratch), through cpma_config's allocator hooks when
 *     they are set; cpma_destroy frees it.  Caller buffers are never retained.
 *     cpma_build also reserves what the next growth steps need (spare leaf
 *     arrays for one growing factor with room for another, resize scratch for
 *     three), so that a resize soon after a build allocates nothing; scratch
 *     buffers grow with room and are kept for reuse.
 *   - Concurrency: one writer per handle (the paper phases updates and queries,
 *     Section "Evaluation on graph workloads", F-Graph description).  Queries
 *     may run concurrently with each other on one stream, never with an
 *     update.
 *   - Errors: argument errors (CPMA_ERR_INVALID, CPMA_ERR_RESERVED_KEY) are
 *     detected before any mutation and leave the set unchanged.  An update
 *     takes every device allocation it can need before it writes the
 *     structure: its batch buffers, the overflow arena, and what a resize of
 *     the worst case can need (the root is within its bound before the batch
 *     and each new key adds at most 10 code bytes); a window redistribution
 *     that cannot get its staging memory spreads the whole structure over its
 *     own leaves instead, with the memory already taken.  So CPMA_ERR_NOMEM
 *     from an update leaves the set unchanged and the handle usable.  A device
 *     failure (CPMA_ERR_DEVICE: a failed launch or copy, an internal limit)
 *     leaves the handle unusable except for cpma_destroy.
 */
#ifndef CPMA_H
#define CPMA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpma cpma; /* opaque handle */

typedef enum {
  CPMA_OK = 0,
  CPMA_ERR_INVALID = 1,      /* bad argument (NULL pointer, bad config, ...) */
  CPMA_ERR_NOMEM = 2,        /* device allocation failed */
  CPMA_ERR_DEVICE = 3,       /* HIP runtime error or internal limit reached */
  CPMA_ERR_RESERVED_KEY = 4  /* a key equal to UINT64_MAX was passed */
} cpma_status;

typedef enum { CPMA_MEM_HOST = 0, CPMA_MEM_DEVICE = 1 } cpma_mem;

/*
 * Structure parameters.  A zero field takes the default.
 *   leaf_bytes     bytes per leaf S: a power of two in [64, 4096]; default 1024.
 *                  The paper sizes leaves Theta(log N) cells (Section "Packed
 *                  Memory Array"); here S is fixed per set.
 *   grow           growing factor when the root exceeds its upper bound;
 *                  default 1.2 (the factor the paper uses, appendix "Data
 *                  tables" and Section "Growing factor sensitivity").
 *   up_leaf, up_root, lo_leaf, lo_root
 *                  byte-density bounds at the leaves and at the root; bounds at
 *                  height h interpolate linearly in h/H.  Defaults 0.90, 0.70,
 *                  0.10, 0.30 (the paper's examples use 0.9 at the leaves,
 *                  Figures "pma-insert" and "cpma-update"; it gives no other
 *                  constants).  Must satisfy 0 < lo_leaf <= lo_root <
 *                  up_root <= up_leaf < 1 and lo_root * grow < up_root.
 *   build_density  target root density after a build or resize; default
 *                  up_root / grow.
 *   range_chunk    steps a wave of the range_map scan takes in a row (a range
 *                  query is a search then a scan, Section "Packed Memory
 *                  Array", "Design and operations"): the scan visits its
 *                  interior leaves 64 at a time, one per lane, and waves take
 *                  runs of this many such steps; a power of two in [1, 64];
 *                  default 2.  Layout and results do not depend on it.
 *   rebuild_frac   batch-size threshold of the full rebuild: an insert or
 *                  delete batch of k >= rebuild_frac * n keys (n the set's size
 *                  before the batch) rebuilds the whole structure -- every
 *                  leaf merged with its slice, then all of them spread over a
 *                  fresh array sized for build_density -- instead of counting
 *                  and redistributing windows (Section "Parallel Batch Updates
 *                  in a PMA" rebuilds above about n / 10, its example value).
 *                  Default 1.0: on this GPU the counted path is faster at
 *                  k = n / 10, where every leaf already takes part in the
 *                  merge (cpma_autotune measures the cut-over for a set).
 *                  Results do not depend on it.
 *   uncompressed   0 (default): the CPMA, delta-coded leaves.  1: the plain
 *                  PMA the paper measures compression against (Section
 *                  "Packed Memory Array"; Section "Evaluation on
 *                  microbenchmarks" compares the two): the same leaves, tree,
 *                  byte-density bounds and batch algorithm, but a leaf holds
 *                  its keys as raw little-endian 8-byte words packed to the
 *                  left (used = 8 x keys, zero bytes after them); a resize
 *                  restages every key.  cpma_build, the batch updates,
 *                  range_map (both forms), contains, export, sizes and trim
 *                  support it; cpma_apply_updates (and so the updates of a
 *                  server), the F-Graph calls and cpma_autotune return
 *                  CPMA_ERR_INVALID for it.
 *   values         0 (default): a set of keys.  1: a key-value CPMA (the
 *                  extension the paper names as future work for weighted
 *                  graphs, Section "Evaluation on graph workloads"): every key
 *                  carries an 8-byte value.  A leaf keeps its keys exactly as
 *                  the CPMA does (head and delta codes from byte 0) and the
 *                  values as 8-byte words in key order at the end of the leaf;
 *                  the density bounds count both (every key costs its code and
 *                  8 bytes).  Build with cpma_build_kv (cpma_build gives every
 *                  key the value 0); cpma_insert_kv inserts or overwrites;
 *                  cpma_insert_batch adds keys with value 0 and leaves present
 *                  keys' values; cpma_delete_batch, range_map (of keys),
 *                  contains, the F-Graph calls and trim work as for a set;
 *                  cpma_get and cpma_range_map_values read values;
 *                  cpma_export_code_bytes returns each leaf's code bytes.  A
 *                  resize restages every key and value.  Not with
 *                  uncompressed = 1; cpma_apply_updates and cpma_autotune
 *                  return CPMA_ERR_INVALID for it.
 *   alloc, free, ctx
 *                  device memory for everything the handle owns (leaves, heads,
 *                  used counts, counters, scratch): alloc(bytes, ctx) returns a
 *                  device pointer aligned to 256 bytes, or NULL when out of
 *                  memory (the call then fails with CPMA_ERR_NOMEM; a pointer
 *                  not so aligned fails it with CPMA_ERR_INVALID); free(ptr,
 *                  ctx) releases one.  Set both or neither (CPMA_ERR_INVALID);
 *                  NULL: hipMalloc / hipFree.  They run on the calling thread
 *                  (the worker thread for a served set); cpma_destroy frees
 *                  everything through them.  Pinned host staging is not
 *                  included.
 */
typedef struct {
  uint32_t leaf_bytes;
  double grow;
  double up_leaf, up_root, lo_leaf, lo_root;
  double build_density;
  uint32_t range_chunk;
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
  double rebuild_frac;
  int32_t uncompressed;
  int32_t values;
} cpma_config;

/* Fills *cfg with the defaults above.  Returns CPMA_ERR_INVALID if cfg is NULL. */
cpma_status cpma_config_default(cpma_config* cfg);

/*
 * Autotuner for the batching parameters: leaf size and range-scan chunk picked
 * by measurement on this GPU.  The paper sizes leaves by the structure size
 * (Theta(log N) cells; CPMA leaves grow with n, Section "Compressed Packed
 * Memory Array"); here the trade-off between bytes moved per small update and
 * decode work per scanned byte is timed instead.
 *
 * A sample of `keys` is taken as the keys below a threshold chosen so that about
 * hint->sample_keys remain, which keeps the key density (and so the codes) of
 * the full set.  For each leaf size in {256, 512, 1024, 2048, 4096} the sample
 * is built, an insert batch of hint->batch * sample / n fresh keys in the
 * sample's key range is timed, then hint->queries range queries covering about
 * hint->range_keys sample keys each; the score is
 * insert_weight * insert_ms + (1 - insert_weight) * range_ms.  At the winning
 * size, range_chunk in {1, 2, 4, 8, 16, 32} is timed on the same queries, and
 * the insert batch (with a delete of it) once with the full rebuild forced
 * and once with the counted path: rebuild_frac becomes min(base value, batch
 * / sample) when the rebuild was faster, else max(base value, 2 * batch /
 * sample).  Each time is the least of three runs after a warm-up.
 *
 * keys: n keys in `mem` (host or device), any order; UINT64_MAX is rejected.
 * hint: NULL or zero fields take defaults (batch n / 10, range_keys 1000,
 *       queries 1e5, sample_keys 2^22, insert_weight 0.5 when negative).
 * base: the other configuration fields (NULL = defaults).
 * out:  receives base with leaf_bytes, range_chunk and rebuild_frac set to the
 *       winners.
 * report: NULL or receives every measured time.
 * Synchronises `stream`; allocates and frees its own trial sets.
 */
typedef struct {
  uint64_t batch;
  uint64_t range_keys;
  uint64_t queries;
  uint64_t sample_keys;
  double insert_weight;
} cpma_tune_hint;

typedef struct {
  uint64_t sample_n;         /* keys in the tuning sample */
  uint32_t leaf_bytes[5];    /* candidates, in the order timed */
  double insert_ms[5];       /* insert batch time per candidate */
  double range_ms[5];        /* range query batch time per candidate */
  uint32_t chunk[6];
  double chunk_ms[6];        /* range query batch time per chunk at the winning size */
  uint32_t best_leaf_bytes;
  uint32_t best_chunk;
  double rebuild_ms;         /* insert + delete of the batch, full rebuild forced */
  double batch_path_ms;      /* the same with the counted batch path */
  double best_rebuild_frac;  /* rebuild_frac of the returned configuration */
} cpma_tune_report;

cpma_status cpma_autotune(const uint64_t* keys, uint64_t n, cpma_mem mem, const cpma_tune_hint* hint,
                          const cpma_config* base, void* stream, cpma_config* out,
                          cpma_tune_report* report);

/*
 * Builds a set from n keys (any order, duplicates allowed): the CPMA(start, end)
 * constructor of the paper's API (appendix "PMA/CPMA API").  keys may be NULL
 * when n == 0.  *out receives the handle (NULL on error).  cfg NULL = defaults.
 * Synchronises `stream`.
 */
cpma_status cpma_build(const uint64_t* keys, uint64_t n, cpma_mem mem,
                       const cpma_config* cfg, void* stream, cpma** out);

/*
 * insert_batch (Section "Parallel Batch Updates in a PMA"; API: returns the
 * number of keys added, not counting keys already present).  keys[0..k) in
 * any order with duplicates unless `sorted` != 0, which promises
 * non-decreasing order (checked; an unsorted batch is sorted anyway).  k == 0
 * is a no-op.  *n_added (host pointer, may be NULL) receives the count.
 * Synchronises `stream`.
 */
cpma_status cpma_insert_batch(cpma* set, const uint64_t* keys, uint64_t k,
                              cpma_mem mem, int sorted, void* stream,
                              uint64_t* n_added);

/*
 * remove_batch (deletes are symmetric to inserts, Section "Parallel Batch
 * Updates in a PMA"; API: returns the number of keys removed, not counting
 * absent keys).  Same argument rules as cpma_insert_batch.
 */
cpma_status cpma_delete_batch(cpma* set, const uint64_t* keys, uint64_t k,
                              cpma_mem mem, int sorted, void* stream,
                              uint64_t* n_removed);

/*
 * has(e) for a batch of q keys (point query: search on the leaf heads, then a
 * pass through one leaf; Section "Compressed Packed Memory Array", "Point
 * queries").  out[i] = 1 if keys[i] is in the set, else 0.  keys and out are
 * both in memory space `mem`.
 */
cpma_status cpma_contains(const cpma* set, const uint64_t* keys, uint64_t q,
                          cpma_mem mem, uint8_t* out, void* stream);

/*
 * range_map(start, end, f) for a batch of q half-open ranges [lo[i], hi[i])
 * (Section "Packed Memory Array", "Design and operations": search for the first
 * element, then scan) with f = (sum, count): sum[i] is the sum mod 2^64 of the
 * keys in the range and count[i] their number.  lo >= hi gives (0, 0).  Every
 * key of every range is decoded; no per-leaf aggregate is cached.  lo, hi, sum
 * and count are all in memory space `mem`.
 */
cpma_status cpma_range_map(const cpma* set, const uint64_t* lo, const uint64_t* hi,
                           uint64_t q, cpma_mem mem, uint64_t* sum,
                           uint64_t* count, void* stream);

/*
 * range_map for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that forbid hipMalloc): the same results as
 * cpma_range_map, with every pointer (lo, hi, sum, count) in device memory of
 * the set's GPU.  The call allocates nothing: its per-query scratch (24 bytes
 * per query, about 1.5 MiB in all) is a fixed array that each GPU the library
 * runs on holds until the process ends.  q is at most
 * CPMA_NOALLOC_MAX_QUERIES (larger: CPMA_ERR_INVALID, nothing launched).
 * Every call on one GPU shares that array: two calls whose work overlaps on
 * one GPU (different streams, or different sets on the same GPU, without
 * ordering between them) race and give wrong results.  Phase statistics are
 * not recorded.  Does not synchronise `stream`.
 */
#define CPMA_NOALLOC_MAX_QUERIES 65536u
cpma_status cpma_range_map_noalloc(const cpma* set, const uint64_t* lo, const uint64_t* hi,
                                   uint64_t q, uint64_t* sum, uint64_t* count, void* stream);

/* size(): number of keys.  0 for a NULL handle. */
uint64_t cpma_size(const cpma* set);

/*
 * get_size(): bytes of device memory held by the structure itself -- leaves
 * (num_leaves * leaf_bytes), leaf heads (8 B each) and used counts (4 B each),
 * and for a key-value set the code byte counts (4 B each).
 * Scratch buffers kept for later batches are not counted.
 */
uint64_t cpma_bytes(const cpma* set);

/*
 * Bytes of device memory the handle holds in all: the structure (cpma_bytes),
 * the spare leaf arrays a resize writes into, and every scratch buffer kept for
 * later calls, each with its allocated room.  The fixed scratch of
 * cpma_range_map_noalloc belongs to the library, not to a handle, and is not
 * counted.  0 for a NULL handle.
 */
uint64_t cpma_bytes_held(const cpma* set);

/*
 * Releases every device buffer counted by cpma_bytes_held beyond the structure
 * itself: the spare leaf arrays and the scratch kept from earlier calls (a set
 * that took one large batch otherwise keeps that batch's scratch), and moves
 * the leaf arrays into allocations that fit them.  The set is unchanged; later
 * calls allocate again what they need, and an update still takes all of it
 * before its first write.  Synchronises `stream`.
 * Errors: CPMA_ERR_INVALID for a NULL handle; CPMA_ERR_DEVICE for a broken one
 * or a failed synchronisation (nothing released).
 */
cpma_status cpma_trim(cpma* set, void* stream);

/* Number of leaves and leaf size in bytes of the current layout. */
cpma_status cpma_geometry(const cpma* set, uint64_t* num_leaves, uint32_t* leaf_bytes);

/*
 * Copies the structure to host memory for inspection: bytes[num_leaves *
 * leaf_bytes], used[num_leaves], head[num_leaves] (any pointer may be NULL to
 * skip it).  Synchronises `stream`.
 */
cpma_status cpma_export(const cpma* set, uint8_t* bytes, uint32_t* used,
                        uint64_t* head, void* stream);

/*
 * Key-value sets (cpma_config.values = 1; the key-value CPMA, Section
 * "Evaluation on graph workloads" names it as future work for weighted graphs).
 *
 * cpma_build_kv: cpma_build with a value per key; values[0..n) in the same
 * memory space as keys, values[i] belongs to keys[i]; a key given more than
 * once takes the value of its first occurrence.  cfg->values is taken as 1;
 * cfg->uncompressed must be 0 (CPMA_ERR_INVALID).  n < 2^31.
 *
 * cpma_insert_kv: inserts or overwrites (upsert): a key not in the set is added
 * with its value, a present key takes the new value.  Repeats in the batch:
 * the first occurrence's value.  *n_added = keys added (overwrites are not
 * counted).  k < 2^31.  CPMA_ERR_INVALID on a set without values.
 * Synchronises `stream`.
 *
 * cpma_get: values[i] = the value of keys[i] and found[i] = 1, or 0 and 0 when
 * it is absent; keys, values, found in memory space `mem`.
 *
 * cpma_range_map_values: range_map with f = (sum of the values mod 2^64,
 * count) over the keys in [lo[i], hi[i]); the weighted degree of a vertex u of
 * a weighted F-Graph is the range [u << 32, (u + 1) << 32).
 *
 * cpma_export_code_bytes: clen[num_leaves] (host) = each leaf's key code bytes
 * (used counts codes and values: used = clen + 8 x keys).  Synchronises.
 */
cpma_status cpma_build_kv(const uint64_t* keys, const uint64_t* values, uint64_t n, cpma_mem mem,
                          const cpma_config* cfg, void* stream, cpma** out);
cpma_status cpma_insert_kv(cpma* set, const uint64_t* keys, const uint64_t* values, uint64_t k,
                           cpma_mem mem, void* stream, uint64_t* n_added);
cpma_status cpma_get(const cpma* set, const uint64_t* keys, uint64_t q, cpma_mem mem,
                     uint64_t* values, uint8_t* found, void* stream);
cpma_status cpma_range_map_values(const cpma* set, const uint64_t* lo, const uint64_t* hi,
                                  uint64_t q, cpma_mem mem, uint64_t* vsum, uint64_t* count,
                                  void* stream);
cpma_status cpma_export_code_bytes(const cpma* set, uint32_t* clen, void* stream);

/*
 * F-Graph (Section "Evaluation on graph workloads"): the set holds a graph's
 * edges as keys u<<32 | v.  Vertex ids must be < nv; edge keys with a larger
 * source or destination are ignored.  Both calls need leaf_bytes <= 1024
 * (CPMA_ERR_INVALID otherwise) and synchronise `stream`.
 *
 * cpma_fgraph_bfs: level[v] = hop distance from `source` (UINT32_MAX when
 * unreachable), following edges u -> v.  level is nv entries in memory space
 * `mem`.  The result is unique; the traversal is level-synchronous.
 * symmetric != 0 promises that every edge u -> v has its reverse v -> u (an
 * undirected graph, as F-Graph stores); levels may then be expanded bottom-up
 * (unvisited vertices looking for a parent), whichever direction has fewer
 * vertices to expand.  With symmetric == 0 every level runs top-down; a wrong
 * promise gives the levels of the reversed edges on bottom-up levels.
 *
 * cpma_fgraph_pagerank: `iters` rounds (the paper runs 10) of
 *   p'(v) = (1 - damping) / nv + damping * sum over edges (v, u) of p(u) / deg(u)
 * from p = 1/nv, with deg(u) the number of edges leaving u and FP32 arithmetic
 * and accumulation.  The edge set must be symmetric (an undirected graph, as
 * in the paper's F-Graph); then this equals pushing p(u)/deg(u) along every
 * edge u -> v.  p is nv floats in memory space `mem`.
 */
cpma_status cpma_fgraph_bfs(const cpma* set, uint32_t nv, uint32_t source, int symmetric, cpma_mem mem,
                            uint32_t* level, void* stream);
cpma_status cpma_fgraph_pagerank(const cpma* set, uint32_t nv, int iters, double damping,
                                 cpma_mem mem, float* p, void* stream);

/*
 * The rest of F-Graph's kernels (Section "Evaluation on graph workloads":
 * PageRank, connected components and single-source betweenness centrality,
 * and the vertex array of offsets that the flat edge array has to rebuild).
 * Same edge-key and leaf-size rules as above; all three synchronise `stream`.
 *
 * cpma_fgraph_offsets: off[v] = number of edges (u, w) with u < v (both ids
 * below nv), v = 0 .. nv: the offsets array of the graph's CSR form, from one
 * degree pass and a prefix sum.  off has nv + 1 entries in memory space `mem`.
 *
 * cpma_fgraph_cc: connected components of the undirected graph the symmetric
 * edge set stores: label[v] = the smallest vertex id of v's component (so the
 * result is unique).  Label propagation over the edges, one atomic minimum per
 * run of equal source, with pointer jumping between passes, until a pass
 * changes no label.  label is nv entries in memory space `mem`.
 *
 * cpma_fgraph_bc: single-source betweenness centrality from `source` (Brandes'
 * dependency accumulation) on the symmetric edge set: sigma[v] = number of
 * shortest paths from source to v, delta[v] = sum over the vertices w whose
 * shortest paths pass through v of sigma[v] / sigma[w] * (1 + delta[w]); both
 * 0 for unreachable vertices, FP64 arithmetic (path counts are exact integers
 * while below 2^53).  Levels come from the BFS above; each level then takes
 * one pass over the leaves holding its vertices, outwards for sigma and inwards
 * for delta.  delta (and sigma unless NULL) are nv doubles in memory space
 * `mem`.
 */
cpma_status cpma_fgraph_offsets(const cpma* set, uint32_t nv, cpma_mem mem, uint64_t* off, void* stream);
cpma_status cpma_fgraph_cc(const cpma* set, uint32_t nv, cpma_mem mem, uint32_t* label, void* stream);
cpma_status cpma_fgraph_bc(const cpma* set, uint32_t nv, uint32_t source, cpma_mem mem, double* sigma,
                           double* delta, void* stream);

/*
 * Serving: continuous batching of a request stream in front of one set.
 *
 * A stager thread admits requests in arrival order while the in-flight HBM
 * footprint (admitted requests not yet done) stays under `hbm_budget` bytes and
 * at most `max_slots` requests are in flight, and uploads each admitted
 * request's data to the device on a copy stream at once: requests that arrive
 * while a step runs on the GPU join the next step, and their uploads overlap
 * that step's work.  An executor thread, the set's single writer, takes the
 * next step as soon as the current one ends: it runs every range request of the
 * step as one batched cpma_range_map launch against the state left by the
 * previous steps, then the step's insert / delete requests in arrival order
 * with one cpma_apply_updates call (the paper phases updates and queries with
 * a single writer, Section "Evaluation on graph workloads").  A request's
 * footprint and slot return to the budget when it is done.  Each request's
 * result therefore equals replaying all requests in (step, queries first,
 * updates in arrival order) order one call each.
 *
 * All request buffers are host memory and must stay valid until the request
 * is done.  `done` becomes nonzero (release store) when the outputs are
 * written; `t_admit_ns` / `t_done_ns` are the admission and completion times on
 * the steady clock that cpma_clock_ns reads, `step` the step that served it.
 * While a server runs, the set must not be used by anyone else.
 */
typedef enum { CPMA_REQ_RANGE = 0, CPMA_REQ_INSERT = 1, CPMA_REQ_DELETE = 2 } cpma_req_kind;

typedef struct {
  int32_t kind;          /* cpma_req_kind */
  uint32_t pad;
  uint64_t n;            /* number of ranges, or of keys */
  const uint64_t* keys;  /* insert / delete keys, or the ranges' lo */
  const uint64_t* hi;    /* ranges' hi (range requests only) */
  uint64_t* sum;         /* range outputs, n entries each */
  uint64_t* count;
  uint64_t result;       /* keys added / removed (insert / delete) */
  int32_t status;        /* cpma_status of the request */
  volatile int32_t done;
  uint64_t t_done_ns;
  uint64_t step;
  uint64_t t_admit_ns;
} cpma_request;

/*
 * Applies nreq insert / delete requests with the result of calling
 * cpma_insert_batch / cpma_delete_batch once per request in order (batch
 * updates of Section "Parallel Batch Updates in a PMA", phased by one writer as
 * in Section "Evaluation on graph workloads"), but with one sort of all their
 * keys and at most one delete batch and one insert batch of net changes.
 * The final set is the same; its leaf layout may differ from the one-call-per-
 * request layout (the paper fixes the set, not the placement).
 *
 * kind: nreq host entries, CPMA_REQ_INSERT or CPMA_REQ_DELETE.
 * keys, n: nreq host entries; request r's keys are keys[r][0 .. n[r]) in
 *   memory space `mem` (any order, repeats allowed; keys[r] may be NULL when
 *   n[r] == 0).  The total of n must be below 2^31.
 * result: nreq host words; result[r] = keys request r added (insert) or
 *   removed (delete), counted against the state its own call would have seen.
 * Errors: CPMA_ERR_INVALID for a bad kind, NULL pointer or total, nothing
 * changed; CPMA_ERR_RESERVED_KEY if any key is UINT64_MAX, nothing changed;
 * CPMA_ERR_DEVICE if the device failed (the set is then unusable).
 * Synchronises `stream`.
 */
cpma_status cpma_apply_updates(cpma* set, uint32_t nreq, const int32_t* kind, const uint64_t* const* keys,
                               const uint64_t* n, cpma_mem mem, uint64_t* result, void* stream);

typedef struct {
  uint64_t hbm_budget;   /* bytes of in-flight request data; 0 = 16 GiB */
  uint32_t max_slots;    /* requests in flight; 0 = 4096 */
} cpma_server_config;

typedef struct cpma_server cpma_server;

/* Starts the stager and executor threads serving `set` on the current GPU. */
cpma_status cpma_server_start(cpma* set, const cpma_server_config* cfg, cpma_server** out);
/* Queues a request (stamped with its arrival); thread safe. */
cpma_status cpma_server_submit(cpma_server* srv, cpma_request* req);
/* Serves everything queued, stops the worker and frees the server. */
cpma_status cpma_server_stop(cpma_server* srv, uint64_t* steps_run);
/* Steady-clock nanoseconds (the clock of t_done_ns). */
uint64_t cpma_clock_ns(void);

/*
 * Phase statistics (instrumentation, not part of the paper's API).  While
 * enabled, every call records HIP events around its phases on the call's stream
 * and accumulates, per phase, the number of timed launches, their total device
 * time, and the algorithmic HBM bytes the phase had to move:
 *   CPMA_PHASE_SORT        sort (MSD split + bucket sorts, or LSD passes) and
 *                          repeat removal of a batch
 *   CPMA_PHASE_LOCATE      leaf location + touched-leaf segments
 *   CPMA_PHASE_MERGE       the main per-leaf merge kernel (one wave per leaf of
 *                          narrow key span; one lane per leaf above 1024-byte
 *                          leaves); bytes = leaf bytes read and rewritten + 8 per
 *                          batch key + 20 per touched leaf
 *   CPMA_PHASE_HEAVY       the follow-up merges: leaves of wide key span, slices
 *                          longer than a wave takes, heavy slices (same bytes)
 *   CPMA_PHASE_COUNT       density counting up the implicit tree (a batch of at
 *                          most 4096 keys checks only its touched leaves' paths
 *                          when the previous count left every node within
 *                          bounds, and counts the whole tree otherwise)
 *   CPMA_PHASE_REDIST      window redistribution and resizing
 *   CPMA_PHASE_RANGE_SCAN  the range_map scan kernel; bytes = used bytes of every
 *                          visited leaf + 32 per query
 *   CPMA_PHASE_QUERY       a whole range_map or contains call
 * cpma_stats_enable(set, 1) zeroes the statistics and starts timing every
 * phase; 0 stops.  cpma_stats_select(set, mask) does the same for the phases
 * whose bit (1u << phase) is set in mask (0 stops; a bit at or above
 * CPMA_PHASE_NUM is CPMA_ERR_INVALID).  Each timed phase records two HIP events
 * on the call's stream per occurrence, and each event record leaves the GPU
 * idle for a few microseconds, so a caller that times one kernel selects its
 * phase alone.
 * cpma_stats_get copies min(n, CPMA_PHASE_NUM) entries and synchronises the
 * device.
 */
typedef enum {
  CPMA_PHASE_SORT = 0,
  CPMA_PHASE_LOCATE = 1,
  CPMA_PHASE_MERGE = 2,
  CPMA_PHASE_HEAVY = 3,
  CPMA_PHASE_COUNT = 4,
  CPMA_PHASE_REDIST = 5,
  CPMA_PHASE_RANGE_SCAN = 6,
  CPMA_PHASE_QUERY = 7,
  CPMA_PHASE_NUM = 8
} cpma_phase;

typedef struct {
  uint64_t launches;
  double ms;
  uint64_t alg_bytes;
} cpma_phase_stat;

cpma_status cpma_stats_enable(cpma* set, int on);
cpma_status cpma_stats_select(cpma* set, uint32_t phase_mask);
cpma_status cpma_stats_get(const cpma* set, cpma_phase_stat* out, int n);

/* Frees the handle and all its device memory.  NULL is a no-op. */
void cpma_destroy(cpma* set);

/* Static description of a status code. */
const char* cpma_status_str(cpma_status s);

#ifdef __cplusplus
}
#endif
#endif /* CPMA_H */
