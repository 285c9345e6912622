// Host-only check of the setup path under the address and undefined-behaviour
// sanitizers: the native hierarchy builder (csrc/hierarchy.cpp) and the CSR
// validation / ELL conversion of a context's plan (csrc/plan.hpp), no GPU.
//
// Usage: plan_check SIDE NB SEED
// Builds the block-diffusion hierarchy of side SIDE with an NB x NB block
// field (log10 a uniform in [-2, 2] from a seeded generator), builds the plan
// of the full setup (with the symmetry checks of the reverse sweep), then
// feeds malformed copies of the hierarchy to the validation and prints one
// line per case:  <case> <status>.  Exit status 0 unless a case returns a
// status other than the expected one.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <random>
#include <vector>

#include "plan.hpp"

namespace {

int g_bad = 0;

void expect(const char* name, mg_status got, mg_status want) {
  std::printf("%s %d\n", name, (int)got);
  if (got != want) {
    std::printf("  expected %d: %s\n", (int)want, g_err.c_str());
    ++g_bad;
  }
}

struct CsrCopy {   // an editable copy of one CSR matrix
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  mg_csr m{};
  explicit CsrCopy(const mg_csr& s) : rowptr(s.rowptr, s.rowptr + s.nrows + 1), col(s.col, s.col + s.nnz),
                                      val(s.val, s.val + s.nnz) {
    m = s;
    wire();
  }
  void wire() {
    m.rowptr = rowptr.data();
    m.col = col.data();
    m.val = val.data();
    m.nnz = (int64_t)col.size();
  }
};

mg_status plan_of(const mg_hierarchy& h, int flags, HostPlan& pl) {
  const int J = h.nlevels;
  const int K = 3;
  std::vector<double> prm((size_t)num_params(J, K, K, K), 0.0);
  mg_params p{K, K, K, 2, 2, prm.data(), MG_BASIS_MONOMIAL, MG_AGG_MEAN};
  mg_options o{MG_FP32, 16, 100, 10, 1e-8, 1e6, flags};
  return build_plan(&h, &p, &o, pl, true);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const int side = std::atoi(argv[1]), nb = std::atoi(argv[2]);
  std::mt19937_64 gen((uint64_t)std::atoll(argv[3]));
  std::uniform_real_distribution<double> U(-2.0, 2.0);
  std::vector<double> blocks((size_t)nb * nb);
  for (double& b : blocks) b = std::pow(10.0, U(gen));
  mg_host_hierarchy* hh = nullptr;
  mg_status st = mg_square_hierarchy(side, nb, blocks.data(), 3, &hh);
  if (st != MG_OK) { std::printf("hierarchy %d %s\n", (int)st, g_err.c_str()); return 1; }
  mg_hierarchy h{};
  expect("view", mg_host_hierarchy_view(hh, &h), MG_OK);
  {
    HostPlan pl;
    expect("plan", plan_of(h, MG_FLAG_BACKWARD, pl), MG_OK);
    std::printf("levels %d finest %d sym %d\n", pl.J, pl.lv[0].n, (int)pl.sym_all);
    if (!pl.sym_all) ++g_bad;
  }
  // malformed copies of the finest operator
  const int n0 = h.A[0].nrows;
  auto with_A0 = [&](const char* name, auto edit, mg_status want) {
    CsrCopy c(h.A[0]);
    edit(c);
    c.wire();
    std::vector<mg_csr> A(h.A, h.A + h.nlevels);
    A[0] = c.m;
    mg_hierarchy h2 = h;
    h2.A = A.data();
    HostPlan pl;
    expect(name, plan_of(h2, MG_FLAG_BACKWARD, pl), want);
  };
  with_A0("unsorted", [](CsrCopy& c) { std::swap(c.col[c.rowptr[1]], c.col[c.rowptr[1] + 1]); }, MG_ERR_SHAPE);
  with_A0("col-range", [&](CsrCopy& c) { c.col[c.rowptr[2] + 1] = n0; }, MG_ERR_SHAPE);
  with_A0("rowptr-end", [](CsrCopy& c) { c.rowptr.back() -= 1; }, MG_ERR_SHAPE);
  // a middle row pointer past nnz: must be refused before any column is read
  with_A0("rowptr-overrun", [](CsrCopy& c) { c.rowptr[1] = (int32_t)c.col.size() + 1000; }, MG_ERR_SHAPE);
  with_A0("rowptr-negative", [](CsrCopy& c) { c.rowptr[1] = -5; }, MG_ERR_SHAPE);
  with_A0("zero-diagonal", [](CsrCopy& c) {
    for (int p = c.rowptr[3]; p < c.rowptr[4]; ++p)
      if (c.col[p] == 3) c.val[p] = 0.0;
  }, MG_ERR_SHAPE);
  with_A0("asymmetric", [](CsrCopy& c) {
    for (int p = c.rowptr[5]; p < c.rowptr[6]; ++p)
      if (c.col[p] != 5) { c.val[p] *= 2.0; break; }
  }, MG_OK);
  {
    // P with the wrong column count
    std::vector<mg_csr> P(h.P, h.P + h.nlevels - 1);
    P[0].ncols += 1;
    mg_hierarchy h2 = h;
    h2.P = P.data();
    HostPlan pl;
    expect("P-shape", plan_of(h2, 0, pl), MG_ERR_SHAPE);
  }
  {
    // two rows whose columns stay sorted across the row boundary: a middle row
    // pointer past nnz would read past the column array unless the row
    // pointers are checked before any column
    std::vector<int32_t> rp = {0, 7, 2}, cl = {0, 1};
    std::vector<double> vl = {1.0, 1.0};
    mg_csr m{2, 2, 2, rp.data(), cl.data(), vl.data()};
    expect("rowptr-overrun-sorted", check_csr(&m, "A", 0), MG_ERR_SHAPE);
  }
  {
    // one column's operator arrays (per-column operators, converted by row
    // ranges in parallel): equal to the plan's own ELL arrays; with bad values
    // in two rows, far apart, the error names the first of them, as a pass in
    // row order would
    HostPlan pl;
    expect("plan-columns", plan_of(h, 0, pl), MG_OK);
    const HLevel& L0 = pl.lv[0];
    const int w = L0.off.w, ld = L0.off.ld;
    std::vector<double> off((size_t)w * ld, -1.0), dg(ld, -1.0);
    expect("column", column_arrays(&h.A[0], h.A[0].val, L0, off.data(), dg.data(), 0, 0), MG_OK);
    for (size_t k = 0; k < off.size(); ++k)
      if (off[k] != L0.off.val[k]) {
        std::printf("  column arrays differ from the plan's at slot %zu\n", k);
        ++g_bad;
        break;
      }
    for (int i = 0; i < ld; ++i)
      if (dg[i] != (i < n0 ? L0.diag[i] : 1.0)) {
        std::printf("  column diagonal differs from the plan's at row %d\n", i);
        ++g_bad;
        break;
      }
    std::vector<double> bad(h.A[0].val, h.A[0].val + h.A[0].nnz);
    const int ra = n0 / 2 + 3, rb = n0 - 5;
    bad[h.A[0].rowptr[rb]] = 0.0;
    bad[h.A[0].rowptr[ra] + 1] = std::nan("");
    expect("column-bad-values", column_arrays(&h.A[0], bad.data(), L0, off.data(), dg.data(), 0, 7), MG_ERR_SHAPE);
    const std::string want = "column 7 of A[0]: zero or non-finite value on the pattern at row " + std::to_string(ra);
    std::printf("column-bad-message %s\n", g_err.c_str());
    if (g_err != want) ++g_bad;
  }
  mg_host_hierarchy_free(hh);
  // sides that do not coarsen to the coarsest size are refused
  mg_host_hierarchy* bad = nullptr;
  expect("side", mg_square_hierarchy(side + 1, nb, blocks.data(), 3, &bad), MG_ERR_SHAPE);
  if (bad) mg_host_hierarchy_free(bad);
  std::printf(g_bad ? "FAIL\n" : "ok\n");
  return g_bad ? 1 : 0;
}
