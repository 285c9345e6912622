// Concurrent builds of the native structured hierarchy (csrc/hierarchy.cpp):
// serving runs several setup threads, whose parallel loops share the
// builder's worker threads.  Four threads build hierarchies of different
// sides at once, three times each; every result must equal, byte for byte,
// the same hierarchy built alone.  Built with -fsanitize=thread.
#include <cstdint>
#include <cstdio>
#include <thread>
#include <vector>

#include "mgl.h"

namespace {

uint64_t fnv(const void* p, size_t n, uint64_t h) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// FNV-1a over every level's arrays; 0 if the build failed
uint64_t build_hash(int side, int nb, const double* blocks) {
  mg_host_hierarchy* h = nullptr;
  if (mg_square_hierarchy(side, nb, blocks, 3, &h) != MG_OK) return 0;
  mg_hierarchy v;
  mg_host_hierarchy_view(h, &v);
  uint64_t s = 1469598103934665603ull;
  for (int l = 0; l < v.nlevels; ++l) {
    const mg_csr& a = v.A[l];
    s = fnv(a.rowptr, sizeof(int32_t) * (a.nrows + 1), s);
    s = fnv(a.col, sizeof(int32_t) * a.nnz, s);
    s = fnv(a.val, sizeof(double) * a.nnz, s);
  }
  for (int l = 0; l + 1 < v.nlevels; ++l) {
    const mg_csr& p = v.P[l];
    s = fnv(p.col, sizeof(int32_t) * p.nnz, s);
    s = fnv(p.val, sizeof(double) * p.nnz, s);
  }
  mg_host_hierarchy_free(h);
  return s;
}

}  // namespace

int main() {
  const int nb = 16;
  std::vector<double> blocks(nb * nb);
  uint64_t x = 12345;   // fixed coefficients in [0.01, 100) from a 64-bit LCG
  for (double& b : blocks) {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    b = 0.01 + 99.99 * (double)(x >> 11) / 9007199254740992.0;
  }
  const int sides[4] = {65, 129, 257, 129};
  uint64_t alone[4];
  for (int t = 0; t < 4; ++t) alone[t] = build_hash(sides[t], nb, blocks.data());
  uint64_t got[4][3] = {};
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t)
    th.emplace_back([&, t] {
      for (int rep = 0; rep < 3; ++rep) got[t][rep] = build_hash(sides[t], nb, blocks.data());
    });
  for (auto& q : th) q.join();
  int bad = 0;
  for (int t = 0; t < 4; ++t)
    for (int rep = 0; rep < 3; ++rep) bad += alone[t] == 0 || got[t][rep] != alone[t];
  std::printf("%s %d\n", bad ? "mismatch" : "ok", bad);
  return bad ? 1 : 0;
}
