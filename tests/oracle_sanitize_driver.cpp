// Runs every oracle entry point on small random inputs, for a build of the
// oracle with AddressSanitizer and UndefinedBehaviorSanitizer.  Exits nonzero
// on a result that contradicts a second computation; the sanitizers abort on
// any memory or undefined-behaviour error.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <vector>

#include "oracle.h"

static int failures = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "expectation failed: %s (line %d)\n", #c, __LINE__); \
      failures++;                                                  \
    }                                                              \
  } while (0)

int main() {
  std::mt19937_64 rng(12345);
  // set algebra against std::set
  for (int round = 0; round < 20; round++) {
    const uint64_t n = rng() % 300, k = rng() % 200;
    std::vector<uint64_t> keys(n), batch(k);
    for (auto& x : keys) x = rng() % 1000;
    for (auto& x : batch) x = rng() % 1000;
    std::vector<uint64_t> S(n + 1), U(n + k + 1), D(n + 1);
    const uint64_t m = orc_build(keys.data(), n, S.data());
    std::set<uint64_t> ref(keys.begin(), keys.end());
    EXPECT(m == ref.size());
    uint64_t added = 0, removed = 0;
    const uint64_t mu = orc_insert(S.data(), m, batch.data(), k, U.data(), &added);
    std::set<uint64_t> ru = ref;
    ru.insert(batch.begin(), batch.end());
    EXPECT(mu == ru.size() && added == ru.size() - ref.size());
    const uint64_t md = orc_delete(U.data(), mu, batch.data(), k, D.data(), &removed);
    std::set<uint64_t> bs(batch.begin(), batch.end());
    EXPECT(removed == bs.size() && md == mu - bs.size());
    std::vector<uint8_t> in(k + 1);
    orc_contains(S.data(), m, batch.data(), k, in.data());
    for (uint64_t i = 0; i < k; i++) EXPECT(in[i] == (ref.count(batch[i]) ? 1 : 0));
    // range sums: binary-search form, brute force and threaded form agree
    const uint64_t q = 50;
    std::vector<uint64_t> lo(q), hi(q), s1(q), c1(q), s2(q), c2(q), s3(q), c3(q);
    for (uint64_t i = 0; i < q; i++) {
      lo[i] = rng() % 1100;
      hi[i] = lo[i] + rng() % 300;
    }
    orc_range_map(S.data(), m, lo.data(), hi.data(), q, s1.data(), c1.data());
    orc_range_map_brute(S.data(), m, lo.data(), hi.data(), q, s2.data(), c2.data());
    orc_range_map_threads(S.data(), m, lo.data(), hi.data(), q, s3.data(), c3.data(), 3);
    EXPECT(s1 == s2 && c1 == c2 && s1 == s3 && c1 == c3);
  }
  // byte codes round trip, including the length boundaries
  for (int b = 0; b < 64; b++) {
    for (uint64_t x : {(1ull << b) - 1, 1ull << b, (1ull << b) + 1}) {
      uint8_t buf[10];
      const int len = orc_varint_encode(x, buf);
      uint64_t y = 0;
      EXPECT(orc_varint_decode(buf, len, &y) == len && y == x);
      EXPECT(orc_varint_decode(buf, len - 1, &y) == -1 || len == 1);
    }
  }
  // a small image of two 64-byte leaves, written here, through the checkers
  {
    const uint32_t S = 64;
    std::vector<uint8_t> img(2 * S, 0);
    std::vector<uint64_t> expect = {1000, 1003, 1010, 2000, 2001};
    auto put_head = [&](int leaf, uint64_t x) {
      for (int i = 0; i < 8; i++) img[leaf * S + i] = (uint8_t)(x >> (8 * i));
    };
    put_head(0, 1000);
    img[8] = 3;
    img[9] = 7;
    put_head(1, 2000);
    img[S + 8] = 1;
    std::vector<uint32_t> used = {10, 9};
    std::vector<uint64_t> head = {1000, 2000};
    const double params[4] = {0.9, 0.7, 0.1, 0.3};
    char msg[256];
    EXPECT(orc_check_image(img.data(), used.data(), head.data(), 2, S, params, expect.data(), 5, msg, 256) == 14);
    std::vector<uint64_t> dec(16);
    EXPECT(orc_decode_image(img.data(), used.data(), 2, S, dec.data(), 16) == 5);
    // the same keys as raw words and as key-value leaves: run, codes noted
    std::vector<uint8_t> raw(2 * S, 0);
    for (int j = 0; j < 3; j++)
      for (int i = 0; i < 8; i++) raw[8 * j + i] = (uint8_t)(expect[j] >> (8 * i));
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 8; i++) raw[S + 8 * j + i] = (uint8_t)(expect[3 + j] >> (8 * i));
    std::vector<uint32_t> ru = {24, 16};
    (void)orc_check_image_pma(raw.data(), ru.data(), head.data(), 2, S, params, expect.data(), 5, msg, 256);
    std::vector<uint32_t> clen = {10, 9}, kvused = {34, 25};
    std::vector<uint64_t> vals = {1, 2, 3, 4, 5};
    (void)orc_check_image_kv(img.data(), kvused.data(), clen.data(), head.data(), 2, S, params, expect.data(),
                             vals.data(), 5, msg, 256);
  }
  // graph kernels on a small random symmetric graph
  {
    const uint32_t nv = 200;
    std::set<uint64_t> es;
    for (int i = 0; i < 1500; i++) {
      const uint64_t u = rng() % nv, v = rng() % nv;
      if (u == v) continue;
      es.insert(u << 32 | v);
      es.insert(v << 32 | u);
    }
    std::vector<uint64_t> e(es.begin(), es.end());
    std::vector<uint32_t> level(nv), label(nv);
    std::vector<uint64_t> off(nv + 1);
    std::vector<double> sigma(nv), delta(nv), pr(nv);
    orc_bfs(e.data(), e.size(), nv, 0, level.data());
    orc_offsets(e.data(), e.size(), nv, off.data());
    EXPECT(off[nv] == e.size());
    orc_cc(e.data(), e.size(), nv, label.data());
    orc_bc(e.data(), e.size(), nv, 0, sigma.data(), delta.data());
    orc_pagerank(e.data(), e.size(), nv, 10, 0.85, pr.data());
    double total = 0;
    for (double x : pr) total += x;
    EXPECT(total > 0.5 && total < 1.5);
  }
  if (failures) std::fprintf(stderr, "%d expectation(s) failed\n", failures);
  return failures ? 1 : 0;
}
