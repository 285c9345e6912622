// Native builder of structured multigrid hierarchies (host code).
//
// -div(a grad u) = f on the unit square, P1 elements on the uniform "/" mesh
// (every grid cell split along its south-west to north-east diagonal),
// homogeneous Dirichlet boundary eliminated, a piecewise constant on an
// nb x nb array of square blocks (the block containing a triangle's centroid).
// P_l is the natural inclusion of the nested P1 spaces, R_l = P_l^T, and the
// coarse operators are Galerkin products A_{l+1} = R_l A_l P_l (paper
// Sec. 2.2), symmetrised, with off-diagonal round-off residue
// |a_ij| <= 1e-11 sqrt(|a_ii a_jj|) removed so that the stored pattern is the
// matrix graph {(i, j): A_ij != 0} (Sec. 2.1).  Used for per-request setup
// when serving; it builds inputs of the V-cycle, not the V-cycle itself.
#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "mgl.h"

namespace {

// Host memory of the builders: blocks of 2 MiB and more are 2 MiB aligned
// and marked for transparent huge pages, so that first touching them costs a
// few hundred page faults instead of a few hundred thousand (on a grid of a
// million unknowns: a sixth of the faults, a build 5-10 % shorter; the
// kernel's zeroing of fresh pages remains).
struct HostFree {
  void operator()(void* q) const { std::free(q); }
};
inline void* host_alloc(size_t bytes) {
  constexpr size_t kHuge = size_t(2) << 20;
  bytes = std::max<size_t>(bytes, 1);
  if (bytes < kHuge) {
    void* q = std::malloc(bytes);
    if (!q) throw std::bad_alloc();
    return q;
  }
  const size_t len = (bytes + kHuge - 1) / kHuge * kHuge;
  void* q = std::aligned_alloc(kHuge, len);
  if (!q) throw std::bad_alloc();
  madvise(q, len, MADV_HUGEPAGE);   // advice only: without huge pages nothing changes
  return q;
}

// Array whose elements start uninitialised (filled in parallel by the
// builders, so the pages are first touched by the threads that write them).
template <class T>
struct Buf {
  static_assert(std::is_trivial<T>::value, "Buf holds trivial element types");
  std::unique_ptr<T[], HostFree> p;
  size_t n = 0;
  void resize(size_t m) {
    p.reset(static_cast<T*>(host_alloc(std::max<size_t>(m, 1) * sizeof(T))));
    n = m;
  }
  T& operator[](size_t i) { return p[i]; }
  const T& operator[](size_t i) const { return p[i]; }
  T* data() { return p.get(); }
  const T* data() const { return p.get(); }
  size_t size() const { return n; }
  const T* begin() const { return p.get(); }
  const T* end() const { return p.get() + n; }
};

struct Csr {
  int nrows = 0, ncols = 0;
  Buf<int> rowptr, col;
  Buf<double> val;
};

// Interior unknown of grid point (i, j) of a side x side grid, or -1.
inline int unk(int side, int i, int j) {
  const int m = side - 2;
  if (i < 1 || j < 1 || i > m || j > m) return -1;
  return (j - 1) * m + (i - 1);
}

// Rows assembled from (row, col, val) triplets with a dense per-row accumulator
// (an entry's value is set when its mark first shows the row, so the values
// need no initialisation).
struct RowAcc {
  Buf<double> acc;
  std::vector<int> mark, cols;
  explicit RowAcc(int n) : mark(n, -1) { acc.resize(n); }
  void add(int row, int c, double v) {
    if (mark[c] != row) {
      mark[c] = row;
      acc[c] = 0.0;
      cols.push_back(c);
    }
    acc[c] += v;
  }
};

// Worker threads of the builders, started on first use and kept for the life
// of the process (a build makes a few dozen parallel loops; starting threads
// for each took longer than the loops on grids below ~10^5 unknowns).
class Workers {
 public:
  explicit Workers(int n) {
    for (int i = 0; i < n; ++i) th_.emplace_back([this] { run(); });
  }
  ~Workers() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void submit(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back(std::move(f));
    }
    cv_.notify_one();
  }

 private:
  void run() {
    for (;;) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
        if (q_.empty()) return;   // stop_ and nothing left
        f = std::move(q_.front());
        q_.pop_front();
      }
      f();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> q_;
  std::vector<std::thread> th_;
  bool stop_ = false;
};

inline int host_threads() { return (int)std::max(1u, std::thread::hardware_concurrency()); }
inline Workers& workers() {
  static Workers w(std::min(host_threads(), 8) - 1);
  return w;
}

// fn(r0, r1) over a split of [0, n) into at most 8 contiguous ranges of at
// least about `grain` rows: the calling thread takes the first, the workers the
// others.
// Calls of this library building setup data at the same time (serving runs
// several); their per-row loops share the host's threads between them.
std::atomic<int> g_active_calls{0};
struct ActiveCall {
  ActiveCall() { ++g_active_calls; }
  ~ActiveCall() { --g_active_calls; }
};

template <class F>
void par_rows(int n, F&& fn, int grain = 8192) {
  const int share = std::max(1, host_threads() / std::max(1, g_active_calls.load()));
  const int nt = std::max(1, std::min({share, 8, n / grain + 1}));
  if (nt == 1) {
    fn(0, n);
    return;
  }
  std::mutex m;
  std::condition_variable done;
  int left = nt - 1;
  for (int t = 1; t < nt; ++t)
    workers().submit([&, t] {
      fn((int)((long long)n * t / nt), (int)((long long)n * (t + 1) / nt));
      std::lock_guard<std::mutex> g(m);
      if (--left == 0) done.notify_one();
    });
  fn(0, (int)((long long)n / nt));
  std::unique_lock<std::mutex> lk(m);
  done.wait(lk, [&] { return left == 0; });
}

// CSR with known row lengths: rowptr from the counts, arrays sized once.
Csr alloc_csr(int nrows, int ncols, const std::vector<int>& cnt) {
  Csr c;
  c.nrows = nrows;
  c.ncols = ncols;
  c.rowptr.resize((size_t)nrows + 1);
  c.rowptr[0] = 0;
  for (int i = 0; i < nrows; ++i) c.rowptr[i + 1] = c.rowptr[i] + cnt[i];
  c.col.resize(c.rowptr[nrows]);
  c.val.resize(c.rowptr[nrows]);
  return c;
}

// Five-point rows of the P1 "/" mesh: the triangles around vertex (i, j) are the
// lower-right (v00, v10, v11) and upper-left (v00, v11, v01) triangles of the
// cells (i, j), (i-1, j), (i-1, j-1), (i, j-1), with element matrices
// a/2 [[1,-1,0],[-1,2,-1],[0,-1,1]] and a/2 [[1,0,-1],[0,1,-1],[-1,-1,2]]; the
// diagonal couplings cancel, leaving west, south, east and north neighbours.
Csr assemble(int side, int nb, const double* blocks) {
  const int m = side - 2, n = m * m, cells = side - 1;
  // coefficient of the block containing each triangle's centroid
  // (ci + 2/3, cj + 1/3) (lower-right) and (ci + 1/3, cj + 2/3) (upper-left),
  // exactly in integers
  Buf<double> lr, ul;
  lr.resize((size_t)cells * cells);
  ul.resize((size_t)cells * cells);
  // block index of each coordinate times 3*cells (one division per coordinate, not per triangle)
  std::vector<int> bix((size_t)3 * cells);
  for (int c3 = 0; c3 < 3 * cells; ++c3) bix[c3] = std::min((int)((long long)c3 * nb / (3LL * cells)), nb - 1);
  auto blk = [&](int c3, int d3) { return blocks[(size_t)bix[d3] * nb + bix[c3]]; };
  par_rows(cells, [&](int j0, int j1) {
    for (int cj = j0; cj < j1; ++cj)
      for (int ci = 0; ci < cells; ++ci) {
        lr[(size_t)cj * cells + ci] = blk(3 * ci + 2, 3 * cj + 1);
        ul[(size_t)cj * cells + ci] = blk(3 * ci + 1, 3 * cj + 2);
      }
  });
  auto L = [&](int ci, int cj) { return lr[(size_t)cj * cells + ci]; };
  auto U = [&](int ci, int cj) { return ul[(size_t)cj * cells + ci]; };
  std::vector<int> cnt(n);
  par_rows(n, [&](int r0, int r1) {
    for (int r = r0, i = r0 % m + 1, j = r0 / m + 1; r < r1; ++r, i = i == m ? (++j, 1) : i + 1)
      cnt[r] = 1 + (i > 1) + (j > 1) + (i < m) + (j < m);
  });
  Csr A = alloc_csr(n, n, cnt);
  par_rows(n, [&](int r0, int r1) {
    for (int r = r0, i = r0 % m + 1, j = r0 / m + 1; r < r1; ++r, i = i == m ? (++j, 1) : i + 1) {
      const double a1 = L(i, j), a2 = U(i, j), b1 = L(i - 1, j), c1 = L(i - 1, j - 1), c2 = U(i - 1, j - 1),
                   d2 = U(i, j - 1);
      const double diag = 0.5 * a1 + 0.5 * a2 + b1 + 0.5 * c1 + 0.5 * c2 + d2;
      int p = A.rowptr[r];
      auto put = [&](int c, double v) { A.col[p] = c; A.val[p] = v; ++p; };
      if (j > 1) put(r - m, -0.5 * c1 - 0.5 * d2);   // south (i, j-1)
      if (i > 1) put(r - 1, -0.5 * b1 - 0.5 * c2);   // west (i-1, j)
      put(r, diag);
      if (i < m) put(r + 1, -0.5 * a1 - 0.5 * d2);   // east (i+1, j)
      if (j < m) put(r + m, -0.5 * a2 - 0.5 * b1);   // north (i, j+1)
    }
  });
  return A;
}

// Nested linear interpolation: a fine vertex at an even position is a coarse
// vertex (weight 1); otherwise it is the midpoint of a coarse edge of the "/"
// mesh (weights 1/2 at its two ends, boundary ends dropped).
Csr prolongation(int side_f) {
  const int side_c = (side_f + 1) / 2, mf = side_f - 2;
  const int nf = mf * mf, nc = (side_c - 2) * (side_c - 2);
  // fine row r is grid point (i, j), walked along the rows without divisions
  auto ends = [&](int i, int j, int& c1, int& c2) {
    c1 = unk(side_c, i / 2, j / 2);
    c2 = unk(side_c, (i + 1) / 2, (j + 1) / 2);
  };
  std::vector<int> cnt(nf);
  par_rows(nf, [&](int r0, int r1) {
    for (int r = r0, i = r0 % mf + 1, j = r0 / mf + 1; r < r1; ++r, i = i == mf ? (++j, 1) : i + 1) {
      int c1, c2;
      ends(i, j, c1, c2);
      cnt[r] = c1 == c2 ? (c1 >= 0) : (c1 >= 0) + (c2 >= 0);
    }
  });
  Csr P = alloc_csr(nf, nc, cnt);
  par_rows(nf, [&](int r0, int r1) {
    for (int r = r0, i = r0 % mf + 1, j = r0 / mf + 1; r < r1; ++r, i = i == mf ? (++j, 1) : i + 1) {
      int c1, c2, p = P.rowptr[r];
      ends(i, j, c1, c2);
      if (c1 == c2) {
        if (c1 >= 0) { P.col[p] = c1; P.val[p] = 1.0; }
        continue;
      }
      if (c1 >= 0) { P.col[p] = c1; P.val[p] = 0.5; ++p; }
      if (c2 >= 0) { P.col[p] = c2; P.val[p] = 0.5; }
    }
  });
  return P;
}

// R = P^T of the nested interpolation, row by row: coarse vertex (ci, cj) sits
// at fine (2ci, 2cj) with weight 1 and is an end of the six fine edge
// midpoints around it (horizontal, vertical and the south-west/north-east
// diagonal of the "/" mesh) with weight 1/2; all seven are interior.
Csr restriction(int side_f) {
  const int side_c = (side_f + 1) / 2, mc = side_c - 2, nc = mc * mc, nf = (side_f - 2) * (side_f - 2);
  Csr R = alloc_csr(nc, nf, std::vector<int>(nc, 7));
  par_rows(nc, [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      const int i0 = 2 * (r % mc + 1), j0 = 2 * (r / mc + 1);
      const int di[7] = {-1, 0, -1, 0, 1, 0, 1}, dj[7] = {-1, -1, 0, 0, 0, 1, 1};
      int p = R.rowptr[r];
      for (int k = 0; k < 7; ++k) {
        R.col[p] = unk(side_f, i0 + di[k], j0 + dj[k]);
        R.val[p] = (di[k] == 0 && dj[k] == 0) ? 1.0 : 0.5;
        ++p;
      }
    }
  });
  return R;
}

// Galerkin product A_c = R A P, row by row: for coarse row I,
//   A_c(I, :) = sum_{i in R(I, :)} R_Ii (A P)(i, :),  (A P)(i, :) = sum_{j in A(i, :)} A_ij P(j, :)
// (each row of A P formed on the fly, the sums taken in the order of R (A P)), symmetrised,
// 0.5 (A_c + A_c^T), with off-diagonal round-off residue
// |a_IJ| <= 1e-11 sqrt(|a_II a_JJ|) and exact zeros removed (residue of exactly cancelling
// couplings reaches ~1e-13 on the coarsest levels; genuine couplings stay above ~1e-4).
// Coarse columns of a row of R A P on the structured grids lie within two
// grid steps of the row's own node; Window maps the column offset J - I (the
// coarse grid has mc interior nodes per line, mc >= 5) to one of the 5 x 5
// positions, numbered so that increasing position is increasing J.
struct Window {
  static constexpr int kSide = 5, kHalf = 2, kSize = kSide * kSide;
  int mc = 0, base = 0;
  std::vector<int> pos;   // offset + base -> position, or -1
  explicit Window(int mc_) : mc(mc_), base(kHalf * mc_ + kHalf), pos((size_t)2 * base + 1, -1) {
    for (int dj = -kHalf; dj <= kHalf; ++dj)
      for (int di = -kHalf; di <= kHalf; ++di) pos[(size_t)(dj * mc + di + base)] = (dj + kHalf) * kSide + di + kHalf;
  }
  int at(int off) const {
    const int k = off + base;
    return k < 0 || k >= (int)pos.size() ? -1 : pos[(size_t)k];
  }
  int offset(int w) const { return (w / kSide - kHalf) * mc + (w % kSide - kHalf); }
};

// Galerkin product; mc: interior nodes per line of the coarse grid (the
// window accumulation for mc >= 5, else the general one)
Csr galerkin(const Csr& A, const Csr& P, const Csr& R, int mc) {
  constexpr int kGalerkinGrain = 512;   // rows of R A P per thread at least (~1 us each)
  const int nc = R.nrows;
  // pass 1: the sorted column pattern and values of every row of R A P; each thread keeps its
  // rows in flat buffers of its own, gathered afterwards into one CSR T
  struct Chunk {
    int r0 = 0, r1 = 0;
    std::vector<int> col;
    std::vector<double> val;
  };
  std::vector<int> cnt(nc, 0);
  std::vector<Chunk> chunks;
  std::mutex mu;
  // the window accumulation: the same products and sums, in the same order,
  // into 25 local entries instead of dense arrays of all coarse columns
  std::atomic<bool> outside{mc < Window::kSide};
  if (!outside) {
    const Window win(mc);
    par_rows(nc, [&](int r0, int r1) {
      double ai[Window::kSize], ap[Window::kSize];
      bool ta[Window::kSize] = {}, tp[Window::kSize] = {};
      int la[Window::kSize];
      Chunk ch;
      ch.r0 = r0;
      ch.r1 = r1;
      ch.col.reserve((size_t)(r1 - r0) * 8);
      ch.val.reserve((size_t)(r1 - r0) * 8);
      for (int I = r0; I < r1; ++I) {
        for (int p = R.rowptr[I]; p < R.rowptr[I + 1]; ++p) {
          const int i = R.col[p];
          int na = 0;
          for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            const int j = A.col[q];
            for (int t = P.rowptr[j]; t < P.rowptr[j + 1]; ++t) {
              const int w = win.at(P.col[t] - I);
              if (w < 0) {
                outside = true;
                return;
              }
              if (!ta[w]) {
                ta[w] = true;
                ai[w] = 0.0;
                la[na++] = w;
              }
              ai[w] += A.val[q] * P.val[t];
            }
          }
          for (int k = 0; k < na; ++k) {
            const int w = la[k];
            if (!tp[w]) {
              tp[w] = true;
              ap[w] = 0.0;
            }
            ap[w] += R.val[p] * ai[w];
            ta[w] = false;
          }
        }
        int c = 0;
        for (int w = 0; w < Window::kSize; ++w)
          if (tp[w]) {
            ch.col.push_back(I + win.offset(w));
            ch.val.push_back(ap[w]);
            tp[w] = false;
            ++c;
          }
        cnt[I] = c;
      }
      std::lock_guard<std::mutex> lk(mu);
      chunks.push_back(std::move(ch));
    }, kGalerkinGrain);
    if (outside) chunks.clear();
  }
  if (outside) par_rows(nc, [&](int r0, int r1) {
    RowAcc ap(P.ncols), ai(P.ncols);
    Chunk ch;
    ch.r0 = r0;
    ch.r1 = r1;
    ch.col.reserve((size_t)(r1 - r0) * 8);
    ch.val.reserve((size_t)(r1 - r0) * 8);
    int tag = 0;
    for (int I = r0; I < r1; ++I) {
      for (int p = R.rowptr[I]; p < R.rowptr[I + 1]; ++p) {
        const int i = R.col[p];
        for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
          const int j = A.col[q];
          for (int s = P.rowptr[j]; s < P.rowptr[j + 1]; ++s) ai.add(tag, P.col[s], A.val[q] * P.val[s]);
        }
        // each column J of this row of A P adds to A_c(I, J) once, so the order of the
        // columns does not change the sums (taken over the rows of R in order)
        for (int J : ai.cols) ap.add(I, J, R.val[p] * ai.acc[J]);
        ai.cols.clear();
        ++tag;
      }
      std::sort(ap.cols.begin(), ap.cols.end());
      cnt[I] = (int)ap.cols.size();
      for (int J : ap.cols) {
        ch.col.push_back(J);
        ch.val.push_back(ap.acc[J]);
      }
      ap.cols.clear();
    }
    std::lock_guard<std::mutex> lk(mu);
    chunks.push_back(std::move(ch));
  }, kGalerkinGrain);
  Csr T = alloc_csr(nc, nc, cnt);
  for (const Chunk& ch : chunks) {
    std::copy(ch.col.begin(), ch.col.end(), T.col.data() + T.rowptr[ch.r0]);
    std::copy(ch.val.begin(), ch.val.end(), T.val.data() + T.rowptr[ch.r0]);
  }
  std::vector<Chunk>().swap(chunks);
  // pass 2: symmetrise by merging each row with the matching column
  // (value of (J, I) looked up in row J, whose pattern contains I by symmetry
  // of the pattern), then drop residue
  std::vector<double> d(nc, 0.0);
  par_rows(nc, [&](int r0, int r1) {
    for (int I = r0; I < r1; ++I)
      for (int k = T.rowptr[I]; k < T.rowptr[I + 1]; ++k)
        if (T.col[k] == I) d[I] = std::fabs(T.val[k]);
  });
  auto at = [&](int r, int c) {
    const int* b = T.col.data() + T.rowptr[r];
    const int* e = T.col.data() + T.rowptr[r + 1];
    const int* it = std::lower_bound(b, e, c);
    return (it != e && *it == c) ? T.val[it - T.col.data()] : 0.0;
  };
  Buf<double> sv;
  sv.resize(T.col.size());
  par_rows(nc, [&](int r0, int r1) {
    for (int I = r0; I < r1; ++I) {
      int c = 0;
      for (int k = T.rowptr[I]; k < T.rowptr[I + 1]; ++k) {
        const int J = T.col[k];
        double v = 0.5 * (T.val[k] + at(J, I));
        if (J != I && std::fabs(v) <= 1e-11 * std::sqrt(d[I] * d[J])) v = 0.0;
        sv[k] = v;
        c += v != 0.0;
      }
      cnt[I] = c;
    }
  }, kGalerkinGrain);
  Csr o = alloc_csr(nc, nc, cnt);
  par_rows(nc, [&](int r0, int r1) {
    for (int I = r0; I < r1; ++I) {
      int p = o.rowptr[I];
      for (int k = T.rowptr[I]; k < T.rowptr[I + 1]; ++k)
        if (sv[k] != 0.0) { o.col[p] = T.col[k]; o.val[p] = sv[k]; ++p; }
    }
  });
  return o;
}

// The transfers of a grid side (P_l and R_l = P_l^T of every level) depend on
// the mesh only, not on the coefficients: they are built once per side and
// shared, read-only, by every hierarchy of that side (serving builds the same
// few sides over and over).  At most kSideCache sides are kept; a hierarchy
// holds its side's transfers for as long as it lives.
struct Transfers {
  std::vector<Csr> P, R;
};
constexpr size_t kSideCache = 8;
std::shared_ptr<const Transfers> transfers_of(int side, int J) {
  static std::mutex mu;
  static std::vector<std::pair<int, std::shared_ptr<const Transfers>>> cache;   // oldest first
  {
    std::lock_guard<std::mutex> g(mu);
    for (const auto& e : cache)
      if (e.first == side) return e.second;
  }
  auto t = std::make_shared<Transfers>();
  for (int l = 0, s = side; l + 1 < J; ++l, s = (s + 1) / 2) {
    t->P.push_back(prolongation(s));
    t->R.push_back(restriction(s));
  }
  std::lock_guard<std::mutex> g(mu);
  for (const auto& e : cache)
    if (e.first == side) return e.second;   // built meanwhile by another call: keep that one
  if (cache.size() >= kSideCache) cache.erase(cache.begin());
  cache.emplace_back(side, t);
  return t;
}

}  // namespace

struct mg_host_hierarchy {
  std::vector<Csr> A;
  std::shared_ptr<const Transfers> T;   // P_l (and R_l) of the side, shared
  std::vector<mg_csr> Av, Pv;
};

static thread_local std::string h_err;

extern "C" {

mg_status mg_square_hierarchy(int32_t side, int32_t nb, const double* blocks, int32_t coarsest,
                              mg_host_hierarchy** out) {
  if (!out || !blocks || nb < 1 || coarsest < 1) return MG_ERR_INVALID_ARG;
  *out = nullptr;
  // side = 2^k + 1 coarsening to a coarsest x coarsest interior
  int J = 1, s = side;
  while (s - 2 > coarsest) {
    if (s % 2 == 0 || s < 5) return MG_ERR_SHAPE;
    s = (s + 1) / 2;
    ++J;
  }
  if (s - 2 != coarsest || J < 2) return MG_ERR_SHAPE;
  for (int k = 0; k < nb * nb; ++k)
    if (!(blocks[k] > 0.0) || !std::isfinite(blocks[k])) return MG_ERR_INVALID_ARG;
  const ActiveCall guard;
  auto* h = new mg_host_hierarchy;
  h->T = transfers_of(side, J);
  h->A.push_back(assemble(side, nb, blocks));
  s = side;
  for (int l = 0; l + 1 < J; ++l) {
    h->A.push_back(galerkin(h->A.back(), h->T->P[l], h->T->R[l], (s + 1) / 2 - 2));
    s = (s + 1) / 2;
  }
  auto view = [](const Csr& c) {
    mg_csr v;
    v.nrows = c.nrows;
    v.ncols = c.ncols;
    v.nnz = (int64_t)c.col.size();
    v.rowptr = c.rowptr.data();
    v.col = c.col.data();
    v.val = c.val.data();
    return v;
  };
  for (const Csr& a : h->A) h->Av.push_back(view(a));
  for (const Csr& p : h->T->P) h->Pv.push_back(view(p));
  *out = h;
  return MG_OK;
}

mg_status mg_host_hierarchy_view(const mg_host_hierarchy* h, mg_hierarchy* v) {
  if (!h || !v) return MG_ERR_INVALID_ARG;
  v->nlevels = (int32_t)h->A.size();
  v->A = h->Av.data();
  v->P = h->Pv.data();
  v->R = nullptr;
  v->G = nullptr;
  v->ncolumn_values = 0;
  v->column_values = nullptr;
  return MG_OK;
}

void mg_host_hierarchy_free(mg_host_hierarchy* h) { delete h; }

}  // extern "C"
