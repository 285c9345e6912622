// Host-side tiling of a level's graph for the fused K-hop graph convolution.
//
// The nodes are split into tiles of about h x w nodes: a breadth-first
// search from the lowest-index node gives level sets, and a tile takes h
// consecutive level sets and, in each, w consecutive nodes in discovery
// order (on a grid searched from a corner: a parallelogram between two
// anti-diagonals; from an interior node: a piece of a ring).  Every
// tile then lists its own nodes followed by the nodes at graph distance
// 1, 2, ..., KM from them (rows -> columns of the graph), so K <= KM hops of
// the convolution over the tile need nothing outside the list: hop h is
// computed on the nodes at distance <= K - h, whose neighbours are all at
// distance <= K - h + 1.  The graph columns of the listed nodes at distance
// <= KM - 1 are stored as local (list) indices plus one; 0 marks a padding
// slot, which the kernel reads from a row of zeros kept before each buffer.
#pragma once
#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

namespace mgl {

struct TilePlan {
  int ntiles = 0;
  int KM = 0;                    // halo depth
  int wg = 0;                    // graph ELL width (a multiple of 4)
  std::vector<int> toff;         // ntiles + 1: start of each tile's node list in `node`
  std::vector<int> node;         // global node ids, own nodes first, then by distance
  std::vector<int> cnt;          // ntiles x (KM + 1): nodes at distance <= d from the own nodes
  std::vector<int> goff;         // ntiles + 1: start of each tile's local columns in `lcol`
  std::vector<uint16_t> lcol;    // rows at distance <= KM - 1, wg local columns + 1 per row (0: padding)
  std::vector<int> maxcnt;       // KM + 1: maxima of cnt over the tiles
};

// LDS layout of one workgroup for a convolution of K >= 2 hops over `cols`
// columns, in 16-byte units: the input on the nodes at distance <= K at xs,
// hop buffers at y0 (distance <= K - 1) and y1 (distance <= K - 2), each of
// the three preceded by one row of zeros (what a padding slot reads), the
// local graph columns (uint16) and row scales (float) of the rows at
// distance <= K - 1 at col and idg; `end` is the total.
struct TileLayout {
  int xs = 0, y0 = 0, y1 = 0, col = 0, idg = 0, end = 0;
};
inline TileLayout tile_layout(const TilePlan& tp, int K, int cols) {
  TileLayout t;
  if (K < 2 || K > tp.KM) return t;
  const int m = tp.maxcnt[K - 1], u = cols / 4;
  t.xs = u;
  t.y0 = t.xs + u * tp.maxcnt[K] + u;
  t.y1 = t.y0 + u * m + u;
  t.col = t.y1 + (K >= 3 ? u * tp.maxcnt[K - 2] : 0);
  t.idg = t.col + (m * tp.wg * 2 + 15) / 16;
  t.end = t.idg + (m * 4 + 15) / 16;
  return t;
}
inline size_t tile_lds_bytes(const TilePlan& tp, int K, int cols) { return (size_t)tile_layout(tp, K, cols).end * 16; }

namespace tiles_detail {

// Breadth-first search from s over the nodes with placed[i] == 0, marking
// them placed.  order receives the visit order, lstart the start of each
// level set in it (level sets are contiguous in breadth-first order).
// adj: row-major graph columns, wg per row.
inline void bfs(int s, int wg, const int* adj, std::vector<char>& placed, std::vector<int>& order,
                std::vector<int>& lstart) {
  order.clear();
  lstart.clear();
  order.push_back(s);
  placed[s] = 1;
  size_t a = 0;
  while (a < order.size()) {
    const size_t e = order.size();
    lstart.push_back((int)a);
    for (size_t h = a; h < e; ++h) {
      const int i = order[h];
      const int* r = adj + (size_t)i * wg;
      for (int k = 0; k < wg; ++k) {
        const int j = r[k];
        if (placed[j]) continue;
        placed[j] = 1;
        order.push_back(j);
      }
    }
    a = e;
  }
  lstart.push_back((int)order.size());
}

// fn(t0, t1) over a split of [0, n) into contiguous ranges, one thread each (at most 8)
template <class F>
void split_run(int n, int per, F&& fn) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::max(1, std::min({hw, 8, n / per + 1}));
  std::vector<std::thread> th;
  for (int q = 1; q < nt; ++q)
    th.emplace_back([&, q] { fn(q, (int)((long long)n * q / nt), (int)((long long)n * (q + 1) / nt)); });
  fn(0, 0, (int)((long long)n / nt));
  for (auto& x : th) x.join();
}

// row-major copy of a slot-major ELL pattern (n rows, wg slots, stride ld)
inline std::vector<int> row_major(int n, int ld, int wg, const int* col) {
  std::vector<int> adj((size_t)n * wg);
  split_run(n, 16384, [&](int, int r0, int r1) {
    for (int k = 0; k < wg; ++k)
      for (int i = r0; i < r1; ++i) adj[(size_t)i * wg + k] = col[(size_t)k * ld + i];
  });
  return adj;
}

}  // namespace tiles_detail

// Partition into tiles of h level sets x w nodes and build the halo lists.
// Tiles are numbered band group by band group (gb bands of h level sets),
// within a group chunk by chunk: consecutive tiles are neighbours, so a
// tile's halo rows were mostly loaded by the tiles just before it.
// Returns false when a tile's list would not fit 16-bit local indices.
inline bool build_tiles(int n, int ld, int wg, const int* col, int KM, int h, int w, TilePlan& tp, int gb = 4) {
  using tiles_detail::bfs;
  tp = TilePlan{};
  tp.KM = KM;
  tp.wg = wg;
  const std::vector<int> adjv = tiles_detail::row_major(n, ld, wg, col);
  const int* adj = adjv.data();
  std::vector<int> tile_of(n, -1), order, lstart;
  std::vector<char> placed(n, 0);
  int ntiles = 0, part = 0;
  struct Key { int part, group, chunk, band; };
  std::vector<Key> key;
  // one search per connected part (reachable set), from its lowest-index node
  for (int s0 = 0; s0 < n; ++s0) {
    if (placed[s0]) continue;
    bfs(s0, wg, adj, placed, order, lstart);
    const int nlev = (int)lstart.size() - 1;
    for (int b0 = 0; b0 < nlev; b0 += h) {
      const int b1 = std::min(b0 + h, nlev);
      int chunks = 0;
      for (int L = b0; L < b1; ++L) chunks = std::max(chunks, (lstart[L + 1] - lstart[L] + w - 1) / w);
      for (int L = b0; L < b1; ++L)
        for (int q = lstart[L]; q < lstart[L + 1]; ++q) tile_of[order[q]] = ntiles + (q - lstart[L]) / w;
      for (int c = 0; c < chunks; ++c) key.push_back(Key{part, b0 / h / gb, c, b0 / h});
      ntiles += chunks;
    }
    ++part;
  }
  {
    std::vector<int> perm(ntiles), rank(ntiles);
    for (int t = 0; t < ntiles; ++t) perm[t] = t;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
      const Key &x = key[a], &y = key[b];
      if (x.part != y.part) return x.part < y.part;
      if (x.group != y.group) return x.group < y.group;
      if (x.chunk != y.chunk) return x.chunk < y.chunk;
      return x.band < y.band;
    });
    for (int t = 0; t < ntiles; ++t) rank[perm[t]] = t;
    for (int i = 0; i < n; ++i) tile_of[i] = rank[tile_of[i]];
  }
  // own nodes per tile, in index order within a tile (counting sort)
  std::vector<int> own_off(ntiles + 1, 0), own(n);
  for (int i = 0; i < n; ++i) ++own_off[tile_of[i] + 1];
  for (int t = 0; t < ntiles; ++t) own_off[t + 1] += own_off[t];
  {
    std::vector<int> pos(own_off.begin(), own_off.end() - 1);
    for (int i = 0; i < n; ++i) own[pos[tile_of[i]]++] = i;
  }
  // drop empty tiles
  {
    std::vector<int> off2(1, 0);
    for (int t = 0; t < ntiles; ++t)
      if (own_off[t + 1] > own_off[t]) off2.push_back(own_off[t + 1]);
    own_off.swap(off2);
    ntiles = (int)own_off.size() - 1;
  }
  tp.ntiles = ntiles;
  tp.cnt.assign((size_t)ntiles * (KM + 1), 0);
  // halo lists, in parallel over tiles; each thread keeps its own marks
  std::vector<std::vector<int>> lists(ntiles);
  std::vector<std::vector<uint16_t>> lcols(ntiles);
  std::vector<char> bad(8, 0);
  tiles_detail::split_run(ntiles, 64, [&](int tid, int t0, int t1) {
    std::vector<int> mark(n, -1), loc(n, 0);
    for (int t = t0; t < t1; ++t) {
      std::vector<int>& L = lists[t];
      L.assign(own.begin() + own_off[t], own.begin() + own_off[t + 1]);
      for (int r = 0; r < (int)L.size(); ++r) { mark[L[r]] = t; loc[L[r]] = r; }
      int* c = &tp.cnt[(size_t)t * (KM + 1)];
      c[0] = (int)L.size();
      int a = 0;
      for (int d = 1; d <= KM; ++d) {
        const int e = (int)L.size();
        for (int r = a; r < e; ++r) {
          const int g = L[r];
          for (int k = 0; k < wg; ++k) {
            const int j = adj[(size_t)g * wg + k];
            if (j == g || mark[j] == t) continue;
            mark[j] = t;
            loc[j] = (int)L.size();
            L.push_back(j);
          }
        }
        a = e;
        c[d] = (int)L.size();
      }
      if (L.size() > 65534) { bad[tid] = 1; continue; }
      const int rows = c[KM - 1];
      std::vector<uint16_t>& lc = lcols[t];
      lc.resize((size_t)rows * wg);
      for (int r = 0; r < rows; ++r) {
        const int g = L[r];
        for (int k = 0; k < wg; ++k) {
          const int j = adj[(size_t)g * wg + k];
          lc[(size_t)r * wg + k] = (uint16_t)(j == g ? 0 : loc[j] + 1);
        }
      }
    }
  });
  for (char b : bad)
    if (b) { tp = TilePlan{}; return false; }
  tp.toff.assign(ntiles + 1, 0);
  tp.goff.assign(ntiles + 1, 0);
  for (int t = 0; t < ntiles; ++t) {
    tp.toff[t + 1] = tp.toff[t] + (int)lists[t].size();
    tp.goff[t + 1] = tp.goff[t] + (int)lcols[t].size();
  }
  tp.node.resize(tp.toff[ntiles]);
  tp.lcol.resize(tp.goff[ntiles]);
  tiles_detail::split_run(ntiles, 64, [&](int, int t0, int t1) {
    for (int t = t0; t < t1; ++t) {
      std::copy(lists[t].begin(), lists[t].end(), tp.node.begin() + tp.toff[t]);
      std::copy(lcols[t].begin(), lcols[t].end(), tp.lcol.begin() + tp.goff[t]);
      std::vector<int>().swap(lists[t]);
      std::vector<uint16_t>().swap(lcols[t]);
    }
  });
  tp.maxcnt.assign(KM + 1, 0);
  for (int t = 0; t < ntiles; ++t)
    for (int d = 0; d <= KM; ++d) tp.maxcnt[d] = std::max(tp.maxcnt[d], tp.cnt[(size_t)t * (KM + 1) + d]);
  return true;
}

// Checks the invariants the kernel relies on: every node is the own node of
// exactly one tile, each stored local column of a row at distance d points
// (minus one) at that neighbour, listed at distance <= d + 1, and padding
// slots hold 0.
inline bool check_tiles(int n, int ld, const int* col, const TilePlan& tp) {
  std::vector<int> owner(n, -1);
  const int KM = tp.KM;
  for (int t = 0; t < tp.ntiles; ++t) {
    const int* c = &tp.cnt[(size_t)t * (KM + 1)];
    const int* L = &tp.node[tp.toff[t]];
    if (tp.toff[t + 1] - tp.toff[t] != c[KM]) return false;
    if (tp.goff[t + 1] - tp.goff[t] != c[KM - 1] * tp.wg) return false;
    for (int r = 0; r < c[0]; ++r) {
      if (L[r] < 0 || L[r] >= n || owner[L[r]] >= 0) return false;
      owner[L[r]] = t;
    }
  }
  for (int i = 0; i < n; ++i)
    if (owner[i] < 0) return false;
  std::vector<char> bad(8, 0);
  tiles_detail::split_run(tp.ntiles, 64, [&](int tid, int t0, int t1) {
    for (int t = t0; t < t1 && !bad[tid]; ++t) {
      const int* c = &tp.cnt[(size_t)t * (KM + 1)];
      const int* L = &tp.node[tp.toff[t]];
      const uint16_t* lc = &tp.lcol[tp.goff[t]];
      for (int r = c[0]; r < c[KM]; ++r)
        if (L[r] < 0 || L[r] >= n) bad[tid] = 1;
      for (int d = 0; d < KM; ++d)
        for (int r = d ? c[d - 1] : 0; r < c[d]; ++r)
          for (int k = 0; k < tp.wg; ++k) {
            const int j = col[(size_t)k * ld + L[r]];
            const int q = lc[(size_t)r * tp.wg + k] - 1;
            if (j == L[r]) { if (q != -1) bad[tid] = 1; continue; }
            if (q < 0 || q >= c[d + 1] || L[q] != j || q == r) bad[tid] = 1;
          }
    }
  });
  for (char b : bad)
    if (b) return false;
  return true;
}

}  // namespace mgl
