/*
 * CPU oracle for the CPMA hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  The product path (the HIP library) never calls it, shares no
 * code with it, and must fail loudly if its own extension is missing.
 *
 * Everything here is the plain definition of what the compressed packed memory
 * array (Wheatman, Burns, Bulu\c{c}, Xu: "CPMA: An Efficient Batch-Parallel
 * Compressed Set Without Pointers", PPoPP'24) computes, written for obvious
 * correctness, not speed:
 *   - the CPMA is an exact ordered set of 64-bit keys (Section "Packed Memory
 *     Array", paragraph "Design and operations"; appendix "PMA/CPMA API"), so
 *     set results are sorted-vector set algebra;
 *   - the structure checker decodes a device image with its own byte-code
 *     codec and verifies the layout rules of Section "Compressed Packed Memory
 *     Array" (head, packed-left, byte density) and the density bounds of the
 *     implicit tree (Section "Packed Memory Array");
 *   - the F-Graph helpers (Section "Evaluation on graph workloads") build a CSR
 *     from src<<32|dst keys and run BFS and PageRank in double precision.
 *
 * Parity pins: every function is checked by tests/test_oracle_pins.py against
 * brute force, closed forms, published LEB128 byte patterns, graph special
 * cases, a hand-computed table of the density bounds and two hand-built leaf
 * images (one of five leaves with truncated windows at every height) with
 * mistakes planted in them.
 */
#ifndef CPMA_ORACLE_H
#define CPMA_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* ---- set semantics (exact) ------------------------------------------------ */
/* out (capacity n) <- sort+unique(keys); returns the unique count. */
uint64_t orc_build(const uint64_t* keys, uint64_t n, uint64_t* out);
/* out (capacity n+k) <- S u sort+unique(B); *n_added = |B' \ S|; returns |out|. */
uint64_t orc_insert(const uint64_t* S, uint64_t n, const uint64_t* B, uint64_t k,
                    uint64_t* out, uint64_t* n_added);
/* out (capacity n) <- S \ B; *n_removed = |B' n S|; returns |out|. */
uint64_t orc_delete(const uint64_t* S, uint64_t n, const uint64_t* B, uint64_t k,
                    uint64_t* out, uint64_t* n_removed);
/* out[i] = (q[i] in S) */
void orc_contains(const uint64_t* S, uint64_t n, const uint64_t* q, uint64_t nq,
                  uint8_t* out);
/* sum[i] = sum of x in S with lo[i] <= x < hi[i], wrapping mod 2^64; count[i] = #such x. */
void orc_range_map(const uint64_t* S, uint64_t n, const uint64_t* lo,
                   const uint64_t* hi, uint64_t q, uint64_t* sum, uint64_t* count);
/* orc_range_map with the queries split into contiguous blocks over `threads`
 * host threads (timing of the CPU baseline on all host cores). */
void orc_range_map_threads(const uint64_t* S, uint64_t n, const uint64_t* lo,
                           const uint64_t* hi, uint64_t q, uint64_t* sum,
                           uint64_t* count, int threads);
/* The same by a full scan with the predicate, for tiny inputs (pins orc_range_map). */
void orc_range_map_brute(const uint64_t* S, uint64_t n, const uint64_t* lo,
                         const uint64_t* hi, uint64_t q, uint64_t* sum,
                         uint64_t* count);

/* ---- byte codes ------------------------------------------------------------ */
/* Unsigned LEB128: 7-bit groups, least significant first, MSB set on every byte
 * except the last.  Returns the number of bytes written (1..10). */
int orc_varint_encode(uint64_t x, uint8_t* out);
/* Decodes one value from in[0..avail); returns bytes consumed or -1 on a
 * truncated / over-long code. */
int orc_varint_decode(const uint8_t* in, int avail, uint64_t* x);

/* ---- density bounds -------------------------------------------------------- */
/* Fixed-point bound (units of 1/65536) at height h of a tree of height H:
 * which = 0 upper, 1 lower.  params = {up_leaf, up_root, lo_leaf, lo_root}. */
int64_t orc_bound_q(const double* params, int which, int h, int H);
/* Tree height: ceil(log2 L), 0 for L <= 1. */
int orc_tree_height(uint64_t L);

/* ---- structure checker ------------------------------------------------------ */
/* Checks a read-back image (bytes[L*S], used[L], head[L]) against the expected
 * sorted unique key set expect[n].  Returns 0 if every invariant holds, else a
 * nonzero code and a message in msg. */
int orc_check_image(const uint8_t* bytes, const uint32_t* used,
                    const uint64_t* head, uint64_t L, uint32_t S,
                    const double* params, const uint64_t* expect, uint64_t n,
                    char* msg, int msglen);
/* The same checks for the uncompressed variant (the plain PMA): a leaf holds
 * its keys as 8-byte little-endian words from its start (used = 8 x keys), zero
 * bytes after them; code 15 flags a used count that is not a multiple of 8. */
int orc_check_image_pma(const uint8_t* bytes, const uint32_t* used,
                        const uint64_t* head, uint64_t L, uint32_t S,
                        const double* params, const uint64_t* expect, uint64_t n,
                        char* msg, int msglen);
/* The same checks for key-value leaves: codes in each leaf's first clen[i]
 * bytes, one 8-byte value per key at its end (used = clen + 8 x keys), zero
 * bytes between; expect_vals[n] are the values in key order.  Codes 16, 17
 * and 18 flag code bytes above used, a used count that is not the codes plus
 * 8 per key, and a wrong value. */
int orc_check_image_kv(const uint8_t* bytes, const uint32_t* used, const uint32_t* clen,
                       const uint64_t* head, uint64_t L, uint32_t S, const double* params,
                       const uint64_t* expect, const uint64_t* expect_vals, uint64_t n,
                       char* msg, int msglen);
/* Decodes an image into keys (capacity cap); returns the key count or -1. */
int64_t orc_decode_image(const uint8_t* bytes, const uint32_t* used, uint64_t L,
                         uint32_t S, uint64_t* out, uint64_t cap);

/* ---- F-Graph (edge keys src<<32|dst, sorted unique) ------------------------- */
/* level[v] = hop distance from src, UINT32_MAX if unreachable. */
void orc_bfs(const uint64_t* edges, uint64_t m, uint32_t nv, uint32_t src,
             uint32_t* level);
/* off[v] = number of edges with source < v, v = 0..nv (nv + 1 entries). */
void orc_offsets(const uint64_t* edges, uint64_t m, uint32_t nv, uint64_t* off);
/* label[v] = smallest vertex id in v's connected component (symmetric edges). */
void orc_cc(const uint64_t* edges, uint64_t m, uint32_t nv, uint32_t* label);
/* Brandes single-source betweenness: path counts sigma and dependencies delta
 * from src, double precision (symmetric edges). */
void orc_bc(const uint64_t* edges, uint64_t m, uint32_t nv, uint32_t src, double* sigma,
            double* delta);
/* iters rounds of p'(v) = (1-d)/nv + d * sum_{u in N(v)} p(u)/deg(u), p0 = 1/nv. */
void orc_pagerank(const uint64_t* edges, uint64_t m, uint32_t nv, int iters,
                  double damping, double* p);

#ifdef __cplusplus
}
#endif
#endif
