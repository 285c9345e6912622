// Host side of a context's setup: validation of the caller's CSR hierarchy
// (paper Sec. 2.2: operators A_l, transfers P_l, R_l, and the graphs of
// Sec. 2.1) and its conversion to the slot-major ELL arrays and per-row
// scalars the device sweeps read, the parameter vector in power-series form,
// and the dense coarsest operator.  Plain C++ (no HIP): the library includes
// it, and a host-only checker builds it with the address and
// undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "chebtab.hpp"
#include "mgl.h"

namespace {

using mgl::ChebTab;

thread_local std::string g_err;

mg_status fail(mg_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define MG_TRY(...)                            \
  do {                                         \
    mg_status s_ = (__VA_ARGS__);              \
    if (s_ != MG_OK) return s_;                \
  } while (0)

// kOuterBlocks: the FP64 outer residual runs at most this many blocks (1024 fill the chip in one
// round on the 513 workload; 4096 were 1.3 % slower end to end; 16384, one row group per wave, made
// the residual sweep itself 11 % shorter but the solve 1.2 % longer, the final reduction then
// summing 16 times as many partial norms per column)
constexpr int kMaxK = 8, kMaxNu = 8, kMaxB = 256, kMaxW = 64, kOuterBlocks = 1024;

inline int round_up(int w, int m) { return (w + m - 1) / m * m; }

// ------------------------------------------------------------------ host-side structures
// Allocator that leaves int / double elements uninitialised, so the large
// setup arrays are written once, in parallel, by the loops that fill them.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind { using other = NoInit<U>; };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept { ::new ((void*)p) U; }
  template <class U, class... Args>
  void construct(U* p, Args&&... a) { ::new ((void*)p) U(std::forward<Args>(a)...); }
};
template <class T>
using uvector = std::vector<T, NoInit<T>>;

struct HEll {          // slot-major ELL
  int n = 0, w = 0;
  int ld = 0;          // slot stride (level operators: n rounded up to 4; transfers: n)
  uvector<int> col;
  uvector<double> val;
};

struct HLevel {
  int n = 0;
  std::vector<double> diag;
  HEll off;            // off-diagonal nonzeros of A
  bool graph_is_A = true;
  HEll graph;          // only when a separate graph was given
  std::vector<double> invdeg;   // row scale of the aggregation operator
  std::vector<double> gval;     // edge weights in the graph's slots (weighted / symmetric aggregation)
  bool sym_graph = false, sym_A = false;
  // per-column operators (HostPlan::nv > 0): off-diagonal values [w][ld][nv] and diagonal [ld][nv]
  std::vector<double> offv, diagv;
};

// fn(r0, r1) over a split of [0, n) into contiguous ranges, one host thread
// each (at most 8; one for small n).  Used by the setup's per-row loops.
// Calls of this library building setup data at the same time (serving runs
// several); their per-row loops share the host's threads between them.
std::atomic<int> g_active_calls{0};
struct ActiveCall {
  ActiveCall() { ++g_active_calls; }
  ~ActiveCall() { --g_active_calls; }
};

template <class F>
void par_rows(int n, F&& fn) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int share = std::max(1, hw / std::max(1, g_active_calls.load()));
  const int nt = std::max(1, std::min({share, 8, n / 16384 + 1}));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t)
    th.emplace_back([&, t] { fn((int)((long long)n * t / nt), (int)((long long)n * (t + 1) / nt)); });
  fn(0, (int)((long long)n / nt));
  for (auto& x : th) x.join();
}

mg_status check_csr(const mg_csr* m, const char* what, int l) {
  const std::string w = std::string(what) + "[" + std::to_string(l) + "]";
  if (!m || !m->rowptr || (m->nnz > 0 && !m->col)) return fail(MG_ERR_INVALID_ARG, w + ": null array");
  if (m->nrows < 1 || m->ncols < 1 || m->nnz < 0) return fail(MG_ERR_SHAPE, w + ": bad dimensions");
  if (m->rowptr[0] != 0 || m->rowptr[m->nrows] != m->nnz) return fail(MG_ERR_SHAPE, w + ": rowptr ends");
  // every row pointer first, so that no column index past nnz is ever read
  for (int i = 0; i < m->nrows; ++i)
    if (m->rowptr[i + 1] < m->rowptr[i]) return fail(MG_ERR_SHAPE, w + ": rowptr not monotone");
  for (int i = 0; i < m->nrows; ++i) {
    for (int p = m->rowptr[i]; p < m->rowptr[i + 1]; ++p) {
      const int j = m->col[p];
      if (j < 0 || j >= m->ncols) return fail(MG_ERR_SHAPE, w + ": column out of range");
      if (p > m->rowptr[i] && m->col[p - 1] >= j) return fail(MG_ERR_SHAPE, w + ": columns not sorted/unique");
    }
  }
  return MG_OK;
}

bool has_entry(const mg_csr* m, int i, int j, double* v) {
  const int* b = m->col + m->rowptr[i];
  const int* e = m->col + m->rowptr[i + 1];
  const int* p = std::lower_bound(b, e, j);
  if (p == e || *p != j) return false;
  if (v) *v = m->val ? m->val[p - m->col] : 0.0;
  return true;
}

// check_sym: determine whether A and the graph are symmetric (only the
// reverse sweep needs it; forward-only contexts skip the check).
mg_status build_level(const mg_csr* A, const mg_csr* G, HLevel& L, int l, int agg, bool check_sym) {
  const int n = A->nrows;
  L.n = n;
  L.diag.assign(n, 0.0);
  if (!A->val) return fail(MG_ERR_INVALID_ARG, "A values missing");
  std::vector<int> cnt(n, 0);
  par_rows(n, [&](int r0, int r1) {
    for (int i = r0; i < r1; ++i)
      for (int p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
        if (A->col[p] == i) L.diag[i] = A->val[p];
        else if (A->val[p] != 0.0) cnt[i]++;
      }
  });
  for (int i = 0; i < n; ++i)
    if (!(L.diag[i] != 0.0) || !std::isfinite(L.diag[i]))
      return fail(MG_ERR_SHAPE, "A[" + std::to_string(l) + "]: zero or non-finite diagonal at row " + std::to_string(i));
  int w = 0;
  for (int c : cnt) w = std::max(w, c);
  if (w > kMaxW) return fail(MG_ERR_UNSUPPORTED, "A[" + std::to_string(l) + "]: more than 64 off-diagonal entries in a row");
  w = round_up(w, 4);   // the sweeps gather four slots at a time
  const int ld = round_up(n, 4);
  L.off.n = n;
  L.off.w = w;
  L.off.ld = ld;
  L.off.col.resize((size_t)w * ld);
  L.off.val.resize((size_t)w * ld);
  par_rows(ld, [&](int r0, int r1) {
    for (int i = r0; i < r1; ++i) {
      int k = 0;
      if (i < n)
        for (int p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
          if (A->col[p] != i && A->val[p] != 0.0) {
            L.off.col[(size_t)k * ld + i] = A->col[p];
            L.off.val[(size_t)k * ld + i] = A->val[p];
            ++k;
          }
      // padding slots point at the row itself; rows [n, ld) at a valid row (n - 1)
      for (; k < w; ++k) {
        L.off.col[(size_t)k * ld + i] = i < n ? i : n - 1;
        L.off.val[(size_t)k * ld + i] = 0.0;
      }
    }
  });
  // graph
  std::vector<int> deg(n, 0);
  L.graph_is_A = (G == nullptr);
  if (G) {
    int wg = 0;
    for (int i = 0; i < n; ++i) {
      int c = 0;
      for (int p = G->rowptr[i]; p < G->rowptr[i + 1]; ++p) c += (G->col[p] != i);
      deg[i] = c;
      wg = std::max(wg, c);
    }
    if (wg > kMaxW) return fail(MG_ERR_UNSUPPORTED, "G: more than 64 neighbours");
    wg = round_up(wg, 4);
    L.graph.n = n;
    L.graph.w = wg;
    L.graph.ld = round_up(n, 4);
    L.graph.col.assign((size_t)wg * L.graph.ld, n - 1);   // rows [n, ld): a valid column
    for (int i = 0; i < n; ++i) {
      int k = 0;
      for (int p = G->rowptr[i]; p < G->rowptr[i + 1]; ++p)
        if (G->col[p] != i) L.graph.col[(size_t)(k++) * L.graph.ld + i] = G->col[p];
      for (; k < wg; ++k) L.graph.col[(size_t)k * L.graph.ld + i] = i;
    }
  } else {
    deg = cnt;
  }
  L.invdeg.assign(n, 0.0);
  for (int i = 0; i < n; ++i) L.invdeg[i] = deg[i] > 0 ? 1.0 / deg[i] : 0.0;
  // aggregation operator G = diag(r) W: weights in the graph's slots, r in invdeg
  if (agg != MG_AGG_MEAN) {
    const HEll& ge = L.graph_is_A ? L.off : L.graph;
    L.gval.assign((size_t)ge.w * ge.ld, 0.0);
    for (int i = 0; i < n; ++i) {
      double rsum = 0.0;
      for (int k = 0; k < ge.w; ++k) {
        const int j = ge.col[(size_t)k * ge.ld + i];
        if (j == i) continue;   // padding slot
        double wv = 0.0;
        if (agg == MG_AGG_WEIGHTED) {
          if (L.graph_is_A) {
            wv = std::fabs(L.off.val[(size_t)k * ge.ld + i]);
          } else {
            if (!G->val) return fail(MG_ERR_INVALID_ARG, "weighted aggregation over a given graph needs its values");
            double gv = 0.0;
            has_entry(G, i, j, &gv);
            wv = std::fabs(gv);
          }
        } else {
          wv = 1.0 / std::sqrt((double)deg[i] * (double)deg[j]);
        }
        L.gval[(size_t)k * ge.ld + i] = wv;
        rsum += wv;
      }
      L.invdeg[i] = agg == MG_AGG_SYM ? 1.0 : (rsum > 0.0 ? 1.0 / rsum : 0.0);
    }
  }
  // symmetry of the graph and of A (needed by the reverse sweep)
  if (!check_sym) {
    L.sym_A = L.sym_graph = false;
    return MG_OK;
  }
  std::vector<char> asym((size_t)std::min(n, 64), 0);   // one flag per row range
  const int nr = (int)asym.size();
  par_rows(nr, [&](int q0, int q1) {
    for (int q = q0; q < q1; ++q) {
      const int i0 = (int)((long long)n * q / nr), i1 = (int)((long long)n * (q + 1) / nr);
      for (int i = i0; i < i1 && !asym[q]; ++i)
        for (int p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
          double v = 0.0;
          if (!has_entry(A, A->col[p], i, &v) || v != A->val[p]) {
            // an explicit zero may lack its mirror
            if (A->val[p] == 0.0 && !has_entry(A, A->col[p], i, nullptr)) continue;
            asym[q] = 1;
            break;
          }
        }
    }
  });
  L.sym_A = std::find(asym.begin(), asym.end(), 1) == asym.end();
  if (!G) {
    L.sym_graph = L.sym_A;
  } else {
    L.sym_graph = true;
    for (int i = 0; i < n && L.sym_graph; ++i)
      for (int p = G->rowptr[i]; p < G->rowptr[i + 1]; ++p) {
        double v = 0.0;
        if (G->col[p] != i && (!has_entry(G, G->col[p], i, &v) ||
                               (agg == MG_AGG_WEIGHTED && G->val && std::fabs(v) != std::fabs(G->val[p])))) {
          L.sym_graph = false;
          break;
        }
      }
  }
  return MG_OK;
}

// Padding slots of a transfer carry weight 0 and point at a column the row
// already reads (its first entry; for an empty row, a column at the same
// relative position), so their loads hit lines in flight rather than every
// row's padding loading the same column 0.
inline int pad_col(int i, int nrows, int ncols) {
  return (int)std::min<long>((long)i * ncols / std::max(nrows, 1), (long)ncols - 1);
}

HEll ell_from_csr(const mg_csr* m, int mult) {
  HEll e;
  e.n = m->nrows;
  int w = 0;
  for (int i = 0; i < m->nrows; ++i) w = std::max(w, m->rowptr[i + 1] - m->rowptr[i]);
  w = round_up(std::max(w, 1), mult);
  e.w = w;
  e.col.resize((size_t)w * e.n);
  e.val.resize((size_t)w * e.n);
  par_rows(e.n, [&](int r0, int r1) {
    for (int i = r0; i < r1; ++i) {
      int k = 0;
      for (int p = m->rowptr[i]; p < m->rowptr[i + 1]; ++p, ++k) {
        e.col[(size_t)k * e.n + i] = m->col[p];
        e.val[(size_t)k * e.n + i] = m->val ? m->val[p] : 0.0;
      }
      const int pc = m->rowptr[i] < m->rowptr[i + 1] ? m->col[m->rowptr[i]] : pad_col(i, m->nrows, m->ncols);
      for (; k < w; ++k) {   // padding: weight 0
        e.col[(size_t)k * e.n + i] = pc;
        e.val[(size_t)k * e.n + i] = 0.0;
      }
    }
  });
  return e;
}

HEll ell_transpose(const mg_csr* m, int mult) {
  std::vector<int> cnt(m->ncols, 0);
  for (int64_t p = 0; p < m->nnz; ++p) cnt[m->col[p]]++;
  HEll e;
  e.n = m->ncols;
  int w = 0;
  for (int c : cnt) w = std::max(w, c);
  w = round_up(std::max(w, 1), mult);
  e.w = w;
  e.col.resize((size_t)w * e.n);
  e.val.resize((size_t)w * e.n);
  par_rows(w, [&](int k0, int k1) {   // weights of the padding slots: 0
    std::fill(e.val.begin() + (size_t)k0 * e.n, e.val.begin() + (size_t)k1 * e.n, 0.0);
  });
  std::vector<int> fill(m->ncols, 0);
  for (int i = 0; i < m->nrows; ++i)
    for (int p = m->rowptr[i]; p < m->rowptr[i + 1]; ++p) {
      const int j = m->col[p];
      const int k = fill[j]++;
      e.col[(size_t)k * e.n + j] = i;
      e.val[(size_t)k * e.n + j] = m->val[p];
    }
  par_rows(e.n, [&](int j0, int j1) {   // padding columns
    for (int j = j0; j < j1; ++j) {
      const int pc = fill[j] ? e.col[j] : pad_col(j, m->ncols, m->nrows);
      for (int k = fill[j]; k < w; ++k) e.col[(size_t)k * e.n + j] = pc;
    }
  });
  return e;
}

struct HostPlan {
  int J = 0, B = 1, prec = 0, KB = 0, KR = 0, KP = 0, nu_pre = 0, nu_post = 0, flags = 0;
  int basis = MG_BASIS_MONOMIAL, agg = MG_AGG_MEAN;
  int max_outer = 1, check_every = 1;
  double rtol = 1e-8, divf = 1e6;
  std::vector<HLevel> lv;
  std::vector<HEll> P, R, PT, RT;
  bool R_is_PT = true;
  std::vector<double> Acoarse;   // dense n_J x n_J row-major
  std::vector<double> params;   // power-series coefficients (converted from the caller's basis)
  bool sym_all = true;
  int nv = 0;                    // columns with their own operator values (0: shared)
  std::vector<double> AcoarseV;  // nv > 0: [nv][n_J][n_J], each column's dense coarsest operator
  // nv > 0: the CSR pattern of every A_l (rowptr, col), kept to place a new column's values
  std::vector<std::vector<int32_t>> prow, pcol;
};

// Rows [r0, r1) of column_arrays; on a value off the rules, the failing row and
// the message.
mg_status column_rows(const mg_csr* A, const double* v, const HLevel& L, double* off, double* dg, int l, int b,
                      int r0, int r1, int& row, std::string& msg) {
  const int ld = L.off.ld, w = L.off.w;
  for (int k = 0; k < w; ++k) std::fill(off + (size_t)k * ld + r0, off + (size_t)k * ld + r1, 0.0);
  for (int i = r0; i < r1; ++i) {
    int k = 0;
    bool has_diag = false;
    for (int p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
      const double x = v[p];
      if (!std::isfinite(x) || x == 0.0) {
        row = i;
        msg = "column " + std::to_string(b) + " of A[" + std::to_string(l) +
              "]: zero or non-finite value on the pattern at row " + std::to_string(i);
        return MG_ERR_SHAPE;
      }
      if (A->col[p] == i) {
        dg[i] = x;
        has_diag = true;
      } else {
        if (k >= w) {
          row = i;
          msg = "column values do not fit the pattern's width";
          return MG_ERR_SHAPE;
        }
        off[(size_t)k * ld + i] = x;
        ++k;
      }
    }
    if (!has_diag) {
      row = i;
      msg = "A[" + std::to_string(l) + "]: no diagonal entry at row " + std::to_string(i);
      return MG_ERR_SHAPE;
    }
  }
  return MG_OK;
}

// One column's operator on the ELL layout of level L (built from the same
// pattern): off[k * ld + i] the k-th off-diagonal entry of row i (CSR order,
// padding 0), dg[i] the diagonal (rows [n, ld): 1).  The values must be finite
// with nonzero off-diagonal entries and diagonal, so the column's graph is the
// pattern's.
mg_status column_arrays(const mg_csr* A, const double* v, const HLevel& L, double* off, double* dg, int l, int b) {
  const int n = A->nrows, ld = L.off.ld, w = L.off.w;
  // rows [n, ld) of the padded layout
  for (int k = 0; k < w; ++k) std::fill(off + (size_t)k * ld + n, off + (size_t)(k + 1) * ld, 0.0);
  std::fill(dg + n, dg + ld, 1.0);
  // rows in parallel; the reported error is the one of the first failing row,
  // as a pass in row order would report it
  std::mutex mu;
  int first = INT_MAX;
  mg_status st = MG_OK;
  std::string msg;
  par_rows(n, [&](int r0, int r1) {
    int row = INT_MAX;
    std::string m;
    const mg_status s = column_rows(A, v, L, off, dg, l, b, r0, r1, row, m);
    if (s == MG_OK) return;
    std::lock_guard<std::mutex> g(mu);
    if (st == MG_OK || row < first) {
      first = row;
      st = s;
      msg = m;
    }
  });
  return st == MG_OK ? MG_OK : fail(st, msg);
}

// Coefficients of the Chebyshev polynomials, T_k(t) = sum_m t[k][m] t^m, k, m <= 8.
ChebTab cheb_table() {
  ChebTab c{};
  c.t[0][0] = 1.0;
  c.t[1][1] = 1.0;
  for (int k = 1; k < 8; ++k)
    for (int m = 0; m <= 8; ++m) c.t[k + 1][m] = (m > 0 ? 2.0 * c.t[k][m - 1] : 0.0) - c.t[k - 1][m];
  return c;
}

// Parameters in the caller's basis -> power-series coefficients of each
// convolution in G: sum_k c_k T_k(-G) = sum_m a_m G^m, a_m = sum_k c_k (-1)^k T_k[m].
void to_power_series(std::vector<double>& v, int J, int KB, int KR, int KP, int basis) {
  if (basis != MG_BASIS_CHEBYSHEV) return;
  const ChebTab T = cheb_table();
  const int per = 2 + (KB + 1) + (KR + 1) + (KP + 1);
  for (int l = 0; l + 1 < J; ++l) {
    int off = l * per + 2;
    for (int K : {KB, KR, KP}) {
      double a[9] = {};
      for (int m = 0; m <= K; ++m)
        for (int k = m; k <= K; ++k) a[m] += v[off + k] * ((k & 1) ? -1.0 : 1.0) * T.t[k][m];
      for (int m = 0; m <= K; ++m) v[off + m] = a[m];
      off += K + 1;
    }
  }
}

int64_t num_params(int J, int KB, int KR, int KP) { return (int64_t)(J - 1) * (2 + (KB + 1) + (KR + 1) + (KP + 1)); }

mg_status build_plan(const mg_hierarchy* h, const mg_params* p, const mg_options* o, HostPlan& pl, bool full) {
  if (!h || !p || !o) return fail(MG_ERR_INVALID_ARG, "null hierarchy, params or options");
  if (h->nlevels < 2 || !h->A || !h->P) return fail(MG_ERR_INVALID_ARG, "need nlevels >= 2 with A and P");
  if (o->nrhs < 1 || o->nrhs > kMaxB) return fail(MG_ERR_INVALID_ARG, "nrhs must be in 1..256");
  if (o->precision < 0 || o->precision > 2) return fail(MG_ERR_INVALID_ARG, "unknown precision");
  if (p->KB < 0 || p->KR < 0 || p->KP < 0 || p->KB > kMaxK || p->KR > kMaxK || p->KP > kMaxK)
    return fail(MG_ERR_INVALID_ARG, "convolution orders must be in 0..8");
  if (p->nu_pre < 0 || p->nu_post < 0 || p->nu_pre > kMaxNu || p->nu_post > kMaxNu)
    return fail(MG_ERR_INVALID_ARG, "smoothing steps must be in 0..8");
  if (o->max_outer < 1 || o->check_every < 1) return fail(MG_ERR_INVALID_ARG, "max_outer and check_every must be >= 1");
  if (!(o->rtol >= 0.0)) return fail(MG_ERR_INVALID_ARG, "rtol must be >= 0");
  const int J = h->nlevels;
  pl.J = J; pl.B = o->nrhs; pl.prec = o->precision; pl.KB = p->KB; pl.KR = p->KR; pl.KP = p->KP;
  pl.nu_pre = p->nu_pre; pl.nu_post = p->nu_post; pl.flags = o->flags;
  if (p->basis < MG_BASIS_MONOMIAL || p->basis > MG_BASIS_CHEBYSHEV) return fail(MG_ERR_INVALID_ARG, "unknown basis");
  if (p->aggregation < MG_AGG_MEAN || p->aggregation > MG_AGG_SYM)
    return fail(MG_ERR_INVALID_ARG, "unknown aggregation");
  pl.basis = p->basis;
  pl.agg = p->aggregation;
  pl.max_outer = o->max_outer; pl.check_every = o->check_every; pl.rtol = o->rtol; pl.divf = o->diverge_factor;
  for (int l = 0; l < J; ++l) {
    MG_TRY(check_csr(&h->A[l], "A", l));
    if (h->A[l].nrows != h->A[l].ncols) return fail(MG_ERR_SHAPE, "A[" + std::to_string(l) + "] not square");
    if (h->G) {
      MG_TRY(check_csr(&h->G[l], "G", l));
      if (h->G[l].nrows != h->A[l].nrows || h->G[l].ncols != h->A[l].nrows) return fail(MG_ERR_SHAPE, "G shape");
    }
  }
  for (int l = 0; l + 1 < J; ++l) {
    MG_TRY(check_csr(&h->P[l], "P", l));
    if (!h->P[l].val) return fail(MG_ERR_INVALID_ARG, "P values missing");
    if (h->P[l].nrows != h->A[l].nrows || h->P[l].ncols != h->A[l + 1].nrows)
      return fail(MG_ERR_SHAPE, "P[" + std::to_string(l) + "] must be n_l x n_{l+1}");
    if (h->R) {
      MG_TRY(check_csr(&h->R[l], "R", l));
      if (!h->R[l].val) return fail(MG_ERR_INVALID_ARG, "R values missing");
      if (h->R[l].nrows != h->A[l + 1].nrows || h->R[l].ncols != h->A[l].nrows)
        return fail(MG_ERR_SHAPE, "R[" + std::to_string(l) + "] must be n_{l+1} x n_l");
    }
  }
  if (h->ncolumn_values != 0) {
    if (h->ncolumn_values != o->nrhs || !h->column_values)
      return fail(MG_ERR_INVALID_ARG, "ncolumn_values must be 0 or nrhs, with column_values");
    if (p->aggregation != MG_AGG_MEAN)
      return fail(MG_ERR_UNSUPPORTED, "per-column operators support the mean aggregation only");
    if (o->flags & MG_FLAG_BACKWARD) return fail(MG_ERR_UNSUPPORTED, "per-column operators have no reverse sweep");
    for (int q = 0; q < J * o->nrhs; ++q)
      if (!h->column_values[q]) return fail(MG_ERR_INVALID_ARG, "null column_values entry");
    pl.nv = o->nrhs;
  }
  if (J > 32) return fail(MG_ERR_UNSUPPORTED, "at most 32 levels");
  if (h->A[J - 1].nrows > 4096) return fail(MG_ERR_UNSUPPORTED, "coarsest level larger than 4096 unknowns");
  if (p->values == nullptr) return fail(MG_ERR_INVALID_ARG, "params.values is null");
  const int64_t np = num_params(J, p->KB, p->KR, p->KP);
  pl.params.assign(p->values, p->values + np);
  for (double v : pl.params)
    if (!std::isfinite(v)) return fail(MG_ERR_INVALID_ARG, "non-finite parameter");
  to_power_series(pl.params, J, p->KB, p->KR, p->KP, p->basis);
  pl.lv.resize(J);
  for (int l = 0; l < J; ++l) {
    if (full && pl.nv) {
      // the pattern with column 0's values, then every column's arrays on its slots
      mg_csr a0 = h->A[l];
      a0.val = h->column_values[(size_t)l * pl.nv];
      HLevel& L = pl.lv[l];
      MG_TRY(build_level(&a0, h->G ? &h->G[l] : nullptr, L, l, p->aggregation, false));
      const int w = L.off.w, ld = L.off.ld, nv = pl.nv;
      L.offv.assign((size_t)w * ld * nv, 0.0);
      L.diagv.assign((size_t)ld * nv, 1.0);
      std::vector<double> off((size_t)w * ld), dg(ld);
      for (int b = 0; b < nv; ++b) {
        MG_TRY(column_arrays(&h->A[l], h->column_values[(size_t)l * nv + b], L, off.data(), dg.data(), l, b));
        for (size_t q = 0; q < off.size(); ++q) L.offv[q * nv + b] = off[q];
        for (int i = 0; i < ld; ++i) L.diagv[(size_t)i * nv + b] = dg[i];
      }
      pl.sym_all = false;
      pl.prow.emplace_back(h->A[l].rowptr, h->A[l].rowptr + h->A[l].nrows + 1);
      pl.pcol.emplace_back(h->A[l].col, h->A[l].col + h->A[l].nnz);
    } else if (full) {
      MG_TRY(build_level(&h->A[l], h->G ? &h->G[l] : nullptr, pl.lv[l], l, p->aggregation,
                         (o->flags & MG_FLAG_BACKWARD) != 0));
      pl.sym_all = pl.sym_all && pl.lv[l].sym_A && pl.lv[l].sym_graph;
    } else {
      // sizes only: widths from row counts
      HLevel& L = pl.lv[l];
      L.n = h->A[l].nrows;
      int w = 0;
      for (int i = 0; i < L.n; ++i) w = std::max(w, h->A[l].rowptr[i + 1] - h->A[l].rowptr[i]);
      L.off.n = L.n;
      L.off.w = round_up(w, 4);
      L.graph_is_A = (h->G == nullptr);
      if (h->G) {
        int wg = 0;
        for (int i = 0; i < L.n; ++i) wg = std::max(wg, h->G[l].rowptr[i + 1] - h->G[l].rowptr[i]);
        L.graph.n = L.n;
        L.graph.w = round_up(wg, 4);
      }
    }
  }
  pl.P.resize(J - 1); pl.R.resize(J - 1); pl.PT.resize(J - 1); pl.RT.resize(J - 1);
  pl.R_is_PT = (h->R == nullptr);
  for (int l = 0; l + 1 < J; ++l) {
    if (full) {
      // P and R^T feed the prolongation sweep (pairs of slots), R and P^T the
      // restriction sweep (four slots at a time)
      pl.P[l] = ell_from_csr(&h->P[l], 2);
      pl.PT[l] = ell_transpose(&h->P[l], 4);
      if (h->R) {
        pl.R[l] = ell_from_csr(&h->R[l], 4);
        pl.RT[l] = ell_transpose(&h->R[l], 2);
        // R == P^T exactly?  then the transposes alias
        bool same = pl.R[l].w == pl.PT[l].w && pl.R[l].col == pl.PT[l].col && pl.R[l].val == pl.PT[l].val;
        pl.R_is_PT = pl.R_is_PT && same;
      }
    } else {
      auto rows_w = [](const mg_csr* m, int mult) {
        int w = 0;
        for (int i = 0; i < m->nrows; ++i) w = std::max(w, m->rowptr[i + 1] - m->rowptr[i]);
        return round_up(std::max(w, 1), mult);
      };
      auto cols_w = [](const mg_csr* m, int mult) {
        std::vector<int> c(m->ncols, 0);
        for (int64_t q = 0; q < m->nnz; ++q) c[m->col[q]]++;
        int w = 0;
        for (int x : c) w = std::max(w, x);
        return round_up(std::max(w, 1), mult);
      };
      pl.P[l].n = h->P[l].nrows; pl.P[l].w = rows_w(&h->P[l], 2);
      pl.PT[l].n = h->P[l].ncols; pl.PT[l].w = cols_w(&h->P[l], 4);
      if (h->R) {
        pl.R[l].n = h->R[l].nrows; pl.R[l].w = rows_w(&h->R[l], 4);
        pl.RT[l].n = h->R[l].ncols; pl.RT[l].w = cols_w(&h->R[l], 2);
      }
    }
  }
  if (h->R == nullptr) pl.R_is_PT = true;
  if (full) {
    const mg_csr* Ac = &h->A[J - 1];
    const int n = Ac->nrows;
    pl.Acoarse.assign((size_t)n * n, 0.0);
    const double* av = pl.nv ? h->column_values[(size_t)(J - 1) * pl.nv] : Ac->val;
    for (int i = 0; i < n; ++i)
      for (int q = Ac->rowptr[i]; q < Ac->rowptr[i + 1]; ++q) pl.Acoarse[(size_t)i * n + Ac->col[q]] = av[q];
    if (pl.nv) {
      pl.AcoarseV.assign((size_t)pl.nv * n * n, 0.0);
      for (int b = 0; b < pl.nv; ++b) {
        const double* cv = h->column_values[(size_t)(J - 1) * pl.nv + b];
        double* Ab = &pl.AcoarseV[(size_t)b * n * n];
        for (int i = 0; i < n; ++i)
          for (int q = Ac->rowptr[i]; q < Ac->rowptr[i + 1]; ++q) Ab[(size_t)i * n + Ac->col[q]] = cv[q];
      }
    }
  }
  return MG_OK;
}

}  // namespace
