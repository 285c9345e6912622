// Native builder of structured multigrid hierarchies (host code).
//
// -div(a grad u) = f on the unit square, P1 elements on the uniform "/" mesh
// (every grid cell split along its south-west to north-east diagonal),
// homogeneous Dirichlet boundary eliminated, a piecewise constant on an
// nb x nb array of square blocks (the block containing a triangle's centroid).
// P_l is the natural inclusion of the nested P1 spaces, R_l = P_l^T, and the
// coarse operators are Galerkin products A_{l+1} = R_l A_l P_l (paper
// Sec. 2.2), symmetrised, with off-diagonal round-off residue
// |a_ij| <= 1e-14 sqrt(|a_ii a_jj|) removed so that the stored pattern is the
// matrix graph {(i, j): A_ij != 0} (Sec. 2.1).  Used for per-request setup
// when serving; it builds inputs of the V-cycle, not the V-cycle itself.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mgl.h"

namespace {

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> rowptr, col;
  std::vector<double> val;
};

// Interior unknown of grid point (i, j) of a side x side grid, or -1.
inline int unk(int side, int i, int j) {
  const int m = side - 2;
  if (i < 1 || j < 1 || i > m || j > m) return -1;
  return (j - 1) * m + (i - 1);
}

// Rows assembled from (row, col, val) triplets with a dense per-row accumulator.
struct RowAcc {
  std::vector<double> acc;
  std::vector<int> mark, cols;
  explicit RowAcc(int n) : acc(n, 0.0), mark(n, -1) {}
  void add(int row, int c, double v) {
    if (mark[c] != row) {
      mark[c] = row;
      acc[c] = 0.0;
      cols.push_back(c);
    }
    acc[c] += v;
  }
  void flush(Csr& out, bool drop_zero) {
    std::sort(cols.begin(), cols.end());
    for (int c : cols)
      if (!drop_zero || acc[c] != 0.0) {
        out.col.push_back(c);
        out.val.push_back(acc[c]);
      }
    cols.clear();
    out.rowptr.push_back((int)out.col.size());
  }
};

Csr assemble(int side, int nb, const double* blocks) {
  const int m = side - 2, n = m * m, cells = side - 1;
  Csr A;
  A.nrows = A.ncols = n;
  A.rowptr.assign(1, 0);
  RowAcc ra(n);
  // block of the centroid (ci + 2/3, cj + 1/3) (lower-right triangle) or
  // (ci + 1/3, cj + 2/3) (upper-left), exactly in integers
  auto blk = [&](int c3, int d3) {   // coordinates times 3*cells
    int bi = (int)((long long)c3 * nb / (3LL * cells));
    int bj = (int)((long long)d3 * nb / (3LL * cells));
    bi = std::min(bi, nb - 1);
    bj = std::min(bj, nb - 1);
    return blocks[(size_t)bj * nb + bi];
  };
  for (int j = 1; j <= m; ++j)
    for (int i = 1; i <= m; ++i) {
      const int row = unk(side, i, j);
      // the six triangles around vertex (i, j); element matrices of the
      // lower-right triangle (v00, v10, v11): a/2 [[1,-1,0],[-1,2,-1],[0,-1,1]]
      // and of the upper-left triangle (v00, v11, v01): a/2 [[1,0,-1],[0,1,-1],[-1,-1,2]]
      double diag = 0.0;
      // cell (i, j): vertex is v00 of both triangles
      if (i < cells && j < cells) {
        const double a1 = blk(3 * i + 2, 3 * j + 1), a2 = blk(3 * i + 1, 3 * j + 2);
        diag += 0.5 * a1 + 0.5 * a2;
        const int e = unk(side, i + 1, j), nn = unk(side, i, j + 1);
        if (e >= 0) ra.add(row, e, -0.5 * a1);
        if (nn >= 0) ra.add(row, nn, -0.5 * a2);
      }
      // cell (i-1, j): vertex is v10 of the lower-right triangle only
      if (i - 1 >= 0 && j < cells) {
        const double a1 = blk(3 * (i - 1) + 2, 3 * j + 1);
        diag += a1;
        const int w = unk(side, i - 1, j), ne = unk(side, i, j + 1);
        if (w >= 0) ra.add(row, w, -0.5 * a1);
        if (ne >= 0) ra.add(row, ne, -0.5 * a1);
      }
      // cell (i-1, j-1): vertex is v11 of both triangles
      if (i - 1 >= 0 && j - 1 >= 0) {
        const double a1 = blk(3 * (i - 1) + 2, 3 * (j - 1) + 1), a2 = blk(3 * (i - 1) + 1, 3 * (j - 1) + 2);
        diag += 0.5 * a1 + 0.5 * a2;
        const int s = unk(side, i, j - 1), w = unk(side, i - 1, j);
        if (s >= 0) ra.add(row, s, -0.5 * a1);
        if (w >= 0) ra.add(row, w, -0.5 * a2);
      }
      // cell (i, j-1): vertex is v01 of the upper-left triangle only
      if (i < cells && j - 1 >= 0) {
        const double a2 = blk(3 * i + 1, 3 * (j - 1) + 2);
        diag += a2;
        const int s = unk(side, i, j - 1), e = unk(side, i + 1, j);
        if (s >= 0) ra.add(row, s, -0.5 * a2);
        if (e >= 0) ra.add(row, e, -0.5 * a2);
      }
      ra.add(row, row, diag);
      ra.flush(A, true);
    }
  return A;
}

Csr prolongation(int side_f) {
  const int side_c = (side_f + 1) / 2, mf = side_f - 2;
  Csr P;
  P.nrows = mf * mf;
  P.ncols = (side_c - 2) * (side_c - 2);
  P.rowptr.assign(1, 0);
  RowAcc ra(P.ncols);
  for (int j = 1; j <= mf; ++j)
    for (int i = 1; i <= mf; ++i) {
      const int row = unk(side_f, i, j);
      const int c1 = unk(side_c, i / 2, j / 2), c2 = unk(side_c, (i + 1) / 2, (j + 1) / 2);
      if (c1 >= 0) ra.add(row, c1, 0.5);
      if (c2 >= 0) ra.add(row, c2, 0.5);
      ra.flush(P, true);
    }
  return P;
}

Csr transpose(const Csr& a) {
  Csr t;
  t.nrows = a.ncols;
  t.ncols = a.nrows;
  std::vector<int> cnt(a.ncols + 1, 0);
  for (int c : a.col) cnt[c + 1]++;
  for (int i = 0; i < a.ncols; ++i) cnt[i + 1] += cnt[i];
  t.rowptr = cnt;
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  std::vector<int> pos(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < a.nrows; ++i)
    for (int p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p) {
      const int q = pos[a.col[p]]++;
      t.col[q] = i;
      t.val[q] = a.val[p];
    }
  return t;
}

Csr spgemm(const Csr& a, const Csr& b) {
  Csr c;
  c.nrows = a.nrows;
  c.ncols = b.ncols;
  c.rowptr.assign(1, 0);
  RowAcc ra(b.ncols);
  for (int i = 0; i < a.nrows; ++i) {
    for (int p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p)
      for (int q = b.rowptr[a.col[p]]; q < b.rowptr[a.col[p] + 1]; ++q) ra.add(i, b.col[q], a.val[p] * b.val[q]);
    ra.flush(c, false);
  }
  return c;
}

// 0.5 (C + C^T), then drop off-diagonal residue and exact zeros
Csr sym_drop(const Csr& c) {
  const Csr t = transpose(c);
  Csr s;
  s.nrows = s.ncols = c.nrows;
  s.rowptr.assign(1, 0);
  RowAcc ra(c.ncols);
  for (int i = 0; i < c.nrows; ++i) {
    for (int p = c.rowptr[i]; p < c.rowptr[i + 1]; ++p) ra.add(i, c.col[p], c.val[p]);
    for (int p = t.rowptr[i]; p < t.rowptr[i + 1]; ++p) ra.add(i, t.col[p], t.val[p]);
    for (int cc : ra.cols) ra.acc[cc] *= 0.5;
    ra.flush(s, false);
  }
  std::vector<double> d(s.nrows, 0.0);
  for (int i = 0; i < s.nrows; ++i)
    for (int p = s.rowptr[i]; p < s.rowptr[i + 1]; ++p)
      if (s.col[p] == i) d[i] = std::fabs(s.val[p]);
  Csr o;
  o.nrows = o.ncols = s.nrows;
  o.rowptr.assign(1, 0);
  for (int i = 0; i < s.nrows; ++i) {
    for (int p = s.rowptr[i]; p < s.rowptr[i + 1]; ++p) {
      const int j = s.col[p];
      double v = s.val[p];
      if (j != i && std::fabs(v) <= 1e-14 * std::sqrt(d[i] * d[j])) v = 0.0;
      if (v != 0.0) {
        o.col.push_back(j);
        o.val.push_back(v);
      }
    }
    o.rowptr.push_back((int)o.col.size());
  }
  return o;
}

}  // namespace

struct mg_host_hierarchy {
  std::vector<Csr> A, P;
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
  auto* h = new mg_host_hierarchy;
  h->A.push_back(assemble(side, nb, blocks));
  s = side;
  for (int l = 0; l + 1 < J; ++l) {
    h->P.push_back(prolongation(s));
    const Csr R = transpose(h->P.back());
    h->A.push_back(sym_drop(spgemm(R, spgemm(h->A.back(), h->P.back()))));
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
  for (const Csr& p : h->P) h->Pv.push_back(view(p));
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
  return MG_OK;
}

void mg_host_hierarchy_free(mg_host_hierarchy* h) { delete h; }

}  // extern "C"
