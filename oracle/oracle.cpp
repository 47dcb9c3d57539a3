// CPU oracle for the CPMA hot path -- TEST INFRASTRUCTURE ONLY (see oracle.h).
//
// Plain, slow, obviously correct.  Shares no code with the HIP library.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <queue>
#include <thread>
#include <vector>

typedef std::vector<uint64_t> Vec;

static Vec sorted_unique(const uint64_t* a, uint64_t n) {
  Vec v(a, a + n);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

// ---------------------------------------------------------------------------
// Set semantics.  The CPMA is an exact ordered set: insert_batch adds the batch
// keys not yet present and reports how many were added; remove_batch removes
// the present ones and reports how many were removed (appendix "PMA/CPMA API").
// ---------------------------------------------------------------------------
extern "C" uint64_t orc_build(const uint64_t* keys, uint64_t n, uint64_t* out) {
  Vec v = sorted_unique(keys, n);
  std::copy(v.begin(), v.end(), out);
  return v.size();
}

extern "C" uint64_t orc_insert(const uint64_t* S, uint64_t n, const uint64_t* B,
                               uint64_t k, uint64_t* out, uint64_t* n_added) {
  Vec b = sorted_unique(B, k);
  uint64_t* end = std::set_union(S, S + n, b.begin(), b.end(), out);
  uint64_t m = (uint64_t)(end - out);
  if (n_added) *n_added = m - n;
  return m;
}

extern "C" uint64_t orc_delete(const uint64_t* S, uint64_t n, const uint64_t* B,
                               uint64_t k, uint64_t* out, uint64_t* n_removed) {
  Vec b = sorted_unique(B, k);
  uint64_t* end = std::set_difference(S, S + n, b.begin(), b.end(), out);
  uint64_t m = (uint64_t)(end - out);
  if (n_removed) *n_removed = n - m;
  return m;
}

// Point query: search returns the smallest element >= x; membership is that
// element being x (Section "Packed Memory Array", "Design and operations").
extern "C" void orc_contains(const uint64_t* S, uint64_t n, const uint64_t* q,
                             uint64_t nq, uint8_t* out) {
  for (uint64_t i = 0; i < nq; i++) out[i] = std::binary_search(S, S + n, q[i]) ? 1 : 0;
}

// range_map(start, end, f) applies f to every element in [start, end): a search
// for the first element, then a scan (Section "Packed Memory Array").  Here f
// accumulates the wrapping uint64 sum and the count.
extern "C" void orc_range_map(const uint64_t* S, uint64_t n, const uint64_t* lo,
                              const uint64_t* hi, uint64_t q, uint64_t* sum,
                              uint64_t* count) {
  for (uint64_t i = 0; i < q; i++) {
    uint64_t s = 0, c = 0;
    if (lo[i] < hi[i]) {
      const uint64_t* a = std::lower_bound(S, S + n, lo[i]);
      const uint64_t* b = std::lower_bound(S, S + n, hi[i]);
      for (const uint64_t* p = a; p < b; p++) s += *p;
      c = (uint64_t)(b - a);
    }
    sum[i] = s;
    count[i] = c;
  }
}

// The same queries split into contiguous blocks over `threads` host threads
// (each block is the plain loop above); for timing the CPU baseline on all
// host cores.
extern "C" void orc_range_map_threads(const uint64_t* S, uint64_t n, const uint64_t* lo,
                                      const uint64_t* hi, uint64_t q, uint64_t* sum,
                                      uint64_t* count, int threads) {
  if (threads < 1) threads = 1;
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; t++) {
    uint64_t b = q * (uint64_t)t / (uint64_t)threads, e = q * (uint64_t)(t + 1) / (uint64_t)threads;
    pool.emplace_back([=] { orc_range_map(S, n, lo + b, hi + b, e - b, sum + b, count + b); });
  }
  for (auto& th : pool) th.join();
}

extern "C" void orc_range_map_brute(const uint64_t* S, uint64_t n, const uint64_t* lo,
                                    const uint64_t* hi, uint64_t q, uint64_t* sum,
                                    uint64_t* count) {
  for (uint64_t i = 0; i < q; i++) {
    uint64_t s = 0, c = 0;
    for (uint64_t j = 0; j < n; j++)
      if (lo[i] <= S[j] && S[j] < hi[i]) { s += S[j]; c++; }
    sum[i] = s;
    count[i] = c;
  }
}

// ---------------------------------------------------------------------------
// Byte codes (Section "Compressed Packed Memory Array", "Data compression
// techniques"): each byte carries one continue bit.  Reading adopted: unsigned
// LEB128 -- 7 payload bits per byte, least significant group first, the high
// bit set when another byte of the same value follows.
// ---------------------------------------------------------------------------
extern "C" int orc_varint_encode(uint64_t x, uint8_t* out) {
  int n = 0;
  do {
    uint8_t g = (uint8_t)(x & 0x7f);
    x >>= 7;
    if (x != 0) g |= 0x80;
    out[n++] = g;
  } while (x != 0);
  return n;
}

extern "C" int orc_varint_decode(const uint8_t* in, int avail, uint64_t* x) {
  uint64_t v = 0;
  for (int i = 0; i < avail && i < 10; i++) {
    uint64_t g = in[i] & 0x7f;
    if (i == 9 && g > 1) return -1;  // would overflow 64 bits
    v |= g << (7 * i);
    if (!(in[i] & 0x80)) {
      *x = v;
      return i + 1;
    }
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Density bounds of the implicit tree (Section "Packed Memory Array": every
// node has an upper bound, and a lower bound for deletes, that depends on its
// height).  The paper gives no constants; the reading adopted interpolates
// linearly in h/H between the leaf and root values, in fixed point with unit
// 1/65536 so that every comparison is exact integer arithmetic.
// ---------------------------------------------------------------------------
static const int64_t kQ = 65536;

extern "C" int orc_tree_height(uint64_t L) {
  int H = 0;
  while ((1ull << H) < L) H++;
  return H;
}

extern "C" int64_t orc_bound_q(const double* params, int which, int h, int H) {
  int64_t leaf = (int64_t)llround(params[which == 0 ? 0 : 2] * (double)kQ);
  int64_t root = (int64_t)llround(params[which == 0 ? 1 : 3] * (double)kQ);
  if (H == 0) return leaf;
  if (which == 0) return leaf - ((leaf - root) * h) / H;  // upper: falls with height
  return leaf + ((root - leaf) * h) / H;                  // lower: rises with height
}

// ---------------------------------------------------------------------------
// Structure checker.  Layout rules (Section "Compressed Packed Memory Array",
// "CPMA structure"): a leaf stores its head uncompressed in its first 8 bytes,
// then the deltas to the following elements as byte codes, packed to the left;
// density counts filled bytes over available bytes.
// ---------------------------------------------------------------------------
static int fail(char* msg, int msglen, int code, const char* what, uint64_t a,
                uint64_t b) {
  if (msg && msglen > 0)
    snprintf(msg, (size_t)msglen, "%s (%llu, %llu)", what, (unsigned long long)a,
             (unsigned long long)b);
  return code;
}

static uint64_t load_le64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}

// Decodes leaf i into out; returns -1 on a malformed leaf.
static int decode_leaf(const uint8_t* leaf, uint32_t used, uint32_t S, Vec& out) {
  if (used == 0) return 0;
  if (used < 8 || used > S) return -1;
  uint64_t prev = load_le64(leaf);
  out.push_back(prev);
  uint32_t pos = 8;
  while (pos < used) {
    uint64_t d;
    int len = orc_varint_decode(leaf + pos, (int)(used - pos), &d);
    if (len < 0 || d == 0) return -1;
    for (int j = 0; j < len; j++)
      if (leaf[pos + j] == 0) return -1;
    if (prev + d <= prev) return -1;  // wrapped past 2^64
    prev += d;
    out.push_back(prev);
    pos += (uint32_t)len;
  }
  return 0;
}

extern "C" int64_t orc_decode_image(const uint8_t* bytes, const uint32_t* used,
                                    uint64_t L, uint32_t S, uint64_t* out,
                                    uint64_t cap) {
  Vec all;
  for (uint64_t i = 0; i < L; i++)
    if (decode_leaf(bytes + i * (uint64_t)S, used[i], S, all) < 0) return -1;
  if (all.size() > cap) return -1;
  std::copy(all.begin(), all.end(), out);
  return (int64_t)all.size();
}

extern "C" int orc_check_image(const uint8_t* bytes, const uint32_t* used,
                               const uint64_t* head, uint64_t L, uint32_t S,
                               const double* params, const uint64_t* expect,
                               uint64_t n, char* msg, int msglen) {
  if (L == 0) return fail(msg, msglen, 1, "no leaves", 0, 0);
  Vec all;
  for (uint64_t i = 0; i < L; i++) {
    const uint8_t* leaf = bytes + i * (uint64_t)S;
    uint32_t u = used[i];
    if (u > S) return fail(msg, msglen, 2, "used exceeds leaf size", i, u);
    if (u == 0) {
      // Empty leaves only in the empty set held in a single leaf.
      if (!(L == 1 && n == 0)) return fail(msg, msglen, 3, "empty leaf", i, L);
      if (head[i] != UINT64_MAX) return fail(msg, msglen, 4, "empty leaf head", i, head[i]);
    } else {
      size_t before = all.size();
      if (decode_leaf(leaf, u, S, all) < 0)
        return fail(msg, msglen, 5, "malformed leaf", i, u);
      if (head[i] != all[before]) return fail(msg, msglen, 6, "head mismatch", i, head[i]);
      // Byte length recomputed from the decoded keys must equal used.
      uint64_t bytes_needed = 8;
      uint8_t tmp[10];
      for (size_t j = before + 1; j < all.size(); j++)
        bytes_needed += (uint64_t)orc_varint_encode(all[j] - all[j - 1], tmp);
      if (bytes_needed != u) return fail(msg, msglen, 7, "used != encoded length", i, u);
    }
    for (uint32_t b = u; b < S; b++)
      if (leaf[b] != 0) return fail(msg, msglen, 8, "nonzero byte past used", i, b);
    if (i > 0 && head[i] <= head[i - 1])
      return fail(msg, msglen, 9, "heads not increasing", i, head[i]);
  }
  for (size_t j = 1; j < all.size(); j++)
    if (all[j] <= all[j - 1]) return fail(msg, msglen, 10, "keys not increasing", j, all[j]);
  if (all.size() != n) return fail(msg, msglen, 11, "size mismatch", all.size(), n);
  for (uint64_t j = 0; j < n; j++)
    if (all[j] != expect[j]) return fail(msg, msglen, 12, "content mismatch", j, all[j]);

  // Density bounds at every node of the implicit tree: node (h, i) covers leaves
  // [i*2^h, min((i+1)*2^h, L)) and is measured against its own capacity.
  int H = orc_tree_height(L);
  for (int h = 0; h <= H; h++) {
    uint64_t width = 1ull << h;
    int64_t up = orc_bound_q(params, 0, h, H);
    int64_t lo = orc_bound_q(params, 1, h, H);
    for (uint64_t first = 0; first < L; first += width) {
      uint64_t last = std::min(L, first + width);
      uint64_t sum = 0;
      for (uint64_t j = first; j < last; j++) sum += used[j];
      __int128 cap = (__int128)(last - first) * S;
      __int128 lhs = (__int128)sum * kQ;
      if (lhs > (__int128)up * cap)
        return fail(msg, msglen, 13, "upper density bound violated at (h, first)", (uint64_t)h, first);
      bool root_single_leaf = (h == H && L == 1);
      if (!root_single_leaf && lhs < (__int128)lo * cap)
        return fail(msg, msglen, 14, "lower density bound violated at (h, first)", (uint64_t)h, first);
    }
  }
  if (msg && msglen > 0) msg[0] = 0;
  return 0;
}

// ---------------------------------------------------------------------------
// Checker of the uncompressed variant, the plain PMA (Section "Packed Memory
// Array": elements in sorted order in leaves with empty space after them).
// A leaf holds its elements as 8-byte little-endian words from its start, so
// its filled bytes are 8 per element; the head array names each leaf's first
// element; the density bounds are those of the CPMA, over filled bytes.
// ---------------------------------------------------------------------------
static int density_walk(const uint32_t* used, uint64_t L, uint32_t S, const double* params,
                        char* msg, int msglen) {
  int H = orc_tree_height(L);
  for (int h = 0; h <= H; h++) {
    uint64_t width = 1ull << h;
    int64_t up = orc_bound_q(params, 0, h, H);
    int64_t lo = orc_bound_q(params, 1, h, H);
    for (uint64_t first = 0; first < L; first += width) {
      uint64_t last = std::min(L, first + width);
      uint64_t sum = 0;
      for (uint64_t j = first; j < last; j++) sum += used[j];
      __int128 cap = (__int128)(last - first) * S;
      __int128 lhs = (__int128)sum * kQ;
      if (lhs > (__int128)up * cap)
        return fail(msg, msglen, 13, "upper density bound violated at (h, first)", (uint64_t)h, first);
      bool root_single_leaf = (h == H && L == 1);
      if (!root_single_leaf && lhs < (__int128)lo * cap)
        return fail(msg, msglen, 14, "lower density bound violated at (h, first)", (uint64_t)h, first);
    }
  }
  return 0;
}

extern "C" int orc_check_image_pma(const uint8_t* bytes, const uint32_t* used,
                                   const uint64_t* head, uint64_t L, uint32_t S,
                                   const double* params, const uint64_t* expect,
                                   uint64_t n, char* msg, int msglen) {
  if (L == 0) return fail(msg, msglen, 1, "no leaves", 0, 0);
  Vec all;
  for (uint64_t i = 0; i < L; i++) {
    const uint8_t* leaf = bytes + i * (uint64_t)S;
    uint32_t u = used[i];
    if (u > S) return fail(msg, msglen, 2, "used exceeds leaf size", i, u);
    if (u % 8 != 0) return fail(msg, msglen, 15, "used is not a whole number of elements", i, u);
    if (u == 0) {
      if (!(L == 1 && n == 0)) return fail(msg, msglen, 3, "empty leaf", i, L);
      if (head[i] != UINT64_MAX) return fail(msg, msglen, 4, "empty leaf head", i, head[i]);
    } else {
      for (uint32_t p = 0; p < u; p += 8) all.push_back(load_le64(leaf + p));
      if (head[i] != load_le64(leaf)) return fail(msg, msglen, 6, "head mismatch", i, head[i]);
    }
    for (uint32_t b = u; b < S; b++)
      if (leaf[b] != 0) return fail(msg, msglen, 8, "nonzero byte past used", i, b);
    if (i > 0 && head[i] <= head[i - 1])
      return fail(msg, msglen, 9, "heads not increasing", i, head[i]);
  }
  for (size_t j = 1; j < all.size(); j++)
    if (all[j] <= all[j - 1]) return fail(msg, msglen, 10, "keys not increasing", j, all[j]);
  if (all.size() != n) return fail(msg, msglen, 11, "size mismatch", all.size(), n);
  for (uint64_t j = 0; j < n; j++)
    if (all[j] != expect[j]) return fail(msg, msglen, 12, "content mismatch", j, all[j]);
  int code = density_walk(used, L, S, params, msg, msglen);
  if (code) return code;
  if (msg && msglen > 0) msg[0] = 0;
  return 0;
}

// ---------------------------------------------------------------------------
// Checker of key-value leaves (the key-value CPMA): a leaf holds its keys as
// the CPMA does in its first clen bytes, and one 8-byte little-endian value
// per key, in key order, in its last bytes; the bytes between are zero and its
// filled bytes are clen + 8 per key.
// ---------------------------------------------------------------------------
extern "C" int orc_check_image_kv(const uint8_t* bytes, const uint32_t* used,
                                  const uint32_t* clen, const uint64_t* head, uint64_t L,
                                  uint32_t S, const double* params, const uint64_t* expect,
                                  const uint64_t* expect_vals, uint64_t n, char* msg,
                                  int msglen) {
  if (L == 0) return fail(msg, msglen, 1, "no leaves", 0, 0);
  Vec all, vals;
  for (uint64_t i = 0; i < L; i++) {
    const uint8_t* leaf = bytes + i * (uint64_t)S;
    uint32_t u = used[i], c = clen[i];
    if (u > S) return fail(msg, msglen, 2, "used exceeds leaf size", i, u);
    if (c > u) return fail(msg, msglen, 16, "code bytes exceed used", i, c);
    if (u == 0) {
      if (!(L == 1 && n == 0)) return fail(msg, msglen, 3, "empty leaf", i, L);
      if (head[i] != UINT64_MAX) return fail(msg, msglen, 4, "empty leaf head", i, head[i]);
    } else {
      size_t before = all.size();
      if (c < 8 || decode_leaf(leaf, c, S, all) < 0) return fail(msg, msglen, 5, "malformed leaf", i, c);
      if (head[i] != all[before]) return fail(msg, msglen, 6, "head mismatch", i, head[i]);
      uint64_t bytes_needed = 8;
      uint8_t tmp[10];
      for (size_t j = before + 1; j < all.size(); j++)
        bytes_needed += (uint64_t)orc_varint_encode(all[j] - all[j - 1], tmp);
      if (bytes_needed != c) return fail(msg, msglen, 7, "code bytes != encoded length", i, c);
      uint64_t m = all.size() - before;
      if ((uint64_t)c + 8 * m != u) return fail(msg, msglen, 17, "used != code bytes + 8 per key", i, u);
      for (uint64_t j = 0; j < m; j++) vals.push_back(load_le64(leaf + S - 8 * m + 8 * j));
    }
    uint64_t m_here = u ? (u - c) / 8 : 0;
    for (uint32_t b = c; b < S - 8 * m_here; b++)
      if (leaf[b] != 0) return fail(msg, msglen, 8, "nonzero byte between codes and values", i, b);
    if (i > 0 && head[i] <= head[i - 1])
      return fail(msg, msglen, 9, "heads not increasing", i, head[i]);
  }
  for (size_t j = 1; j < all.size(); j++)
    if (all[j] <= all[j - 1]) return fail(msg, msglen, 10, "keys not increasing", j, all[j]);
  if (all.size() != n) return fail(msg, msglen, 11, "size mismatch", all.size(), n);
  for (uint64_t j = 0; j < n; j++)
    if (all[j] != expect[j]) return fail(msg, msglen, 12, "content mismatch", j, all[j]);
  for (uint64_t j = 0; j < n; j++)
    if (vals[j] != expect_vals[j]) return fail(msg, msglen, 18, "value mismatch", j, vals[j]);
  int code = density_walk(used, L, S, params, msg, msglen);
  if (code) return code;
  if (msg && msglen > 0) msg[0] = 0;
  return 0;
}

// ---------------------------------------------------------------------------
// F-Graph (Section "Evaluation on graph workloads"): an edge (u, v) is the key
// u<<32 | v; the CSR is the canonical two-array form the paper contrasts with.
// ---------------------------------------------------------------------------
static void build_csr(const uint64_t* edges, uint64_t m, uint32_t nv,
                      std::vector<uint64_t>& off, std::vector<uint32_t>& adj) {
  off.assign((size_t)nv + 1, 0);
  adj.resize(m);
  for (uint64_t e = 0; e < m; e++) off[(edges[e] >> 32) + 1]++;
  for (uint32_t v = 0; v < nv; v++) off[v + 1] += off[v];
  std::vector<uint64_t> cur(off.begin(), off.end() - 1);
  for (uint64_t e = 0; e < m; e++)
    adj[cur[edges[e] >> 32]++] = (uint32_t)(edges[e] & 0xffffffffu);
}

extern "C" void orc_bfs(const uint64_t* edges, uint64_t m, uint32_t nv, uint32_t src,
                        uint32_t* level) {
  std::vector<uint64_t> off;
  std::vector<uint32_t> adj;
  build_csr(edges, m, nv, off, adj);
  for (uint32_t v = 0; v < nv; v++) level[v] = UINT32_MAX;
  if (src >= nv) return;
  std::queue<uint32_t> q;
  level[src] = 0;
  q.push(src);
  while (!q.empty()) {
    uint32_t u = q.front();
    q.pop();
    for (uint64_t e = off[u]; e < off[u + 1]; e++) {
      uint32_t v = adj[e];
      if (level[v] == UINT32_MAX) {
        level[v] = level[u] + 1;
        q.push(v);
      }
    }
  }
}

// The vertex array of offsets that a CSR keeps and the flat edge array lacks
// (Section "Evaluation on graph workloads": the reconstruction cost of the
// vertex array): off[v] = number of edges whose source is below v.
extern "C" void orc_offsets(const uint64_t* edges, uint64_t m, uint32_t nv, uint64_t* off) {
  std::vector<uint64_t> o;
  std::vector<uint32_t> adj;
  build_csr(edges, m, nv, o, adj);
  std::copy(o.begin(), o.end(), off);
}

// Connected components of an undirected graph (each edge stored in both
// directions): label[v] = the smallest vertex id of v's component, found by
// a breadth-first search from every not yet labelled vertex in id order.
extern "C" void orc_cc(const uint64_t* edges, uint64_t m, uint32_t nv, uint32_t* label) {
  std::vector<uint64_t> off;
  std::vector<uint32_t> adj;
  build_csr(edges, m, nv, off, adj);
  for (uint32_t v = 0; v < nv; v++) label[v] = UINT32_MAX;
  for (uint32_t r = 0; r < nv; r++) {
    if (label[r] != UINT32_MAX) continue;
    std::queue<uint32_t> q;
    label[r] = r;
    q.push(r);
    while (!q.empty()) {
      uint32_t u = q.front();
      q.pop();
      for (uint64_t e = off[u]; e < off[u + 1]; e++)
        if (label[adj[e]] == UINT32_MAX) {
          label[adj[e]] = r;
          q.push(adj[e]);
        }
    }
  }
}

// Single-source betweenness centrality (Brandes): sigma[v] = number of
// shortest paths from src to v; delta[v] = sum over the vertices w whose
// shortest paths from src pass through v of sigma[v] / sigma[w] * (1 +
// delta[w]) (the dependency of src on v), in double precision.  Vertices
// unreachable from src get sigma = delta = 0.
extern "C" void orc_bc(const uint64_t* edges, uint64_t m, uint32_t nv, uint32_t src, double* sigma,
                       double* delta) {
  std::vector<uint64_t> off;
  std::vector<uint32_t> adj;
  build_csr(edges, m, nv, off, adj);
  std::vector<uint32_t> level(nv, UINT32_MAX), order;
  for (uint32_t v = 0; v < nv; v++) sigma[v] = delta[v] = 0.0;
  if (src >= nv) return;
  std::queue<uint32_t> q;
  level[src] = 0;
  sigma[src] = 1.0;
  q.push(src);
  while (!q.empty()) {
    uint32_t u = q.front();
    q.pop();
    order.push_back(u);
    for (uint64_t e = off[u]; e < off[u + 1]; e++) {
      uint32_t w = adj[e];
      if (level[w] == UINT32_MAX) {
        level[w] = level[u] + 1;
        q.push(w);
      }
      if (level[w] == level[u] + 1) sigma[w] += sigma[u];
    }
  }
  for (size_t i = order.size(); i-- > 0;) {
    uint32_t v = order[i];
    for (uint64_t e = off[v]; e < off[v + 1]; e++) {
      uint32_t w = adj[e];
      if (level[w] == level[v] + 1) delta[v] += sigma[v] / sigma[w] * (1.0 + delta[w]);
    }
  }
}

// PageRank with a fixed iteration count (the paper runs 10): every vertex u
// pushes p(u)/deg(u) along each of its edges; a vertex without edges pushes
// nothing (no dangling-mass redistribution).
extern "C" void orc_pagerank(const uint64_t* edges, uint64_t m, uint32_t nv, int iters,
                             double damping, double* p) {
  std::vector<uint64_t> deg(nv, 0);
  for (uint64_t e = 0; e < m; e++) deg[edges[e] >> 32]++;
  std::vector<double> cur(nv, 1.0 / (double)nv), acc(nv);
  for (int it = 0; it < iters; it++) {
    std::fill(acc.begin(), acc.end(), 0.0);
    for (uint64_t e = 0; e < m; e++) {
      uint32_t u = (uint32_t)(edges[e] >> 32), v = (uint32_t)(edges[e] & 0xffffffffu);
      acc[v] += cur[u] / (double)deg[u];
    }
    for (uint32_t v = 0; v < nv; v++) cur[v] = (1.0 - damping) / (double)nv + damping * acc[v];
  }
  std::copy(cur.begin(), cur.end(), p);
}
