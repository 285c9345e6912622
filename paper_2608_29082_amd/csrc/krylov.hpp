// Device kernels of flexible GMRES (Saad's FGMRES with right preconditioning
// and restarts) around the learnable cycle, for B independent columns at once
// ([n][B] layout, FP64 Krylov vectors, preconditioned vectors in the cycle
// type).
//
// The basis is kept unnormalised: vector i is stored as vt_i with a
// per-column scale sig_i, v_i = sig_i vt_i, so the sweep that orthogonalises
// the new vector also writes it (and its cycle-type copy, the next
// preconditioner input) and its squared norm, and no separate normalisation
// sweep is needed.  Orthogonalisation is classical Gram-Schmidt with one
// reorthogonalisation pass when the first pass left less than a given
// fraction eta of the vector's norm (eta = 1/sqrt 2: "twice is enough",
// Kahan-Parlett).  The update sweep
// of the first pass also forms the second pass's dot products from the basis
// values it already holds, so a vector costs three streams of the basis with
// the second pass and two without.  Dot products are reduced per block and then over blocks in
// a fixed order (deterministic).  The small per-column problems (Hessenberg
// columns, Givens rotations, least squares) run one work-item per column.
//
// Row sweeps map 2^lbk >= B lanes onto each row (one lane per column, B <=
// 256), 256 >> lbk rows per block pass; logical block blk owns the rows
// [blk * chunk, min(n, (blk + 1) * chunk)).
#pragma once
#include "kernels.hpp"

namespace mgl {

#define MGL_KR_CHUNK                                                   \
  const int LB = 1 << lbk, rpb = 256 >> lbk;                           \
  const int b = threadIdx.x & (LB - 1);                                \
  const int rg = (int)(threadIdx.x >> lbk);                            \
  const int blk = xcd_block();                                         \
  const long lo = (long)blk * chunk;                                   \
  const long hi = lo + chunk < n ? lo + chunk : (long)n;               \
  const bool lane_ok = b < B;

// Per-block sum over the row groups of a value per lane, stored to out[b]
// (LDS scratch red[256]; fixed pairwise tree, deterministic).
__device__ __forceinline__ void kr_block_sum(double v, int lbk, int B, double* red, double* out) {
  const int LB = 1 << lbk, rpb = 256 >> lbk;
  const int b = threadIdx.x & (LB - 1), rg = (int)(threadIdx.x >> lbk);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = rpb >> 1; h > 0; h >>= 1) {
    if (rg < h) red[threadIdx.x] += red[threadIdx.x + h * LB];
    __syncthreads();
  }
  if (rg == 0 && b < B) out[b] = red[b];
  __syncthreads();
}

// Basis layout: vector t of row i, column b at V[(i * mp1 + t) * B + b]
// (mp1 = m + 1 vectors per row), so one row of every basis vector is one
// contiguous run and a sweep touches few memory pages at a time.

// Gram-Schmidt dot sweep: part[(blk * (nv + 1) + t) * B + b] =
//   sig_t(b) * sum over the block's rows of w(row, b) * vt_t(row, b)   (t < nv)
// and part[(blk * (nv + 1) + nv) * B + b] = sum of w(row, b)^2 (w with a
// row stride of wrs elements).  NG >= nv accumulators in registers, so w and
// every basis vector are read once; the register budget of two waves per SIMD
// lets every load of a row be in flight at once.  skip: when non-null and *skip == 0 the
// sweep does nothing.
template <int NG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_kr_dot(int n, int B, int lbk, int chunk, int nv,
                                                const double* __restrict__ V, int mp1,
                                                const double* __restrict__ sig, const double* __restrict__ w,
                                                long wrs, double* __restrict__ part, const int* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip == 0) return;
  MGL_KR_CHUNK
  double acc[NG], ww = 0.0;
#pragma unroll
  for (int t = 0; t < NG; ++t) acc[t] = 0.0;
  if (lane_ok) {
    for (long i = lo + rg; i < hi; i += rpb) {
      const double wv = w[(size_t)i * wrs + b];
      const double* vr = V + (size_t)i * mp1 * B + b;
      ww += wv * wv;
      // every load is issued (indices past nv - 1 repeat the last vector and
      // are discarded) so that all of them are in flight together
      double x[NG];
#pragma unroll
      for (int t = 0; t < NG; ++t) x[t] = vr[(size_t)(t < nv ? t : nv - 1) * B];
#pragma unroll
      for (int t = 0; t < NG; ++t) acc[t] += wv * x[t];
    }
  }
  double* out = part + (size_t)blk * (nv + 1) * B;
#pragma unroll
  for (int t = 0; t < NG; ++t)
    if (t < nv) kr_block_sum(lane_ok ? acc[t] * sig[(size_t)t * B + b] : 0.0, lbk, B, red, out + (size_t)t * B);
  kr_block_sum(ww, lbk, B, red, out + (size_t)nv * B);
}

// Gram-Schmidt update sweep: wo = wi - sum_{t < nv} h_t(b) sig_t(b) vt_t
// (wi, wo with row strides wis, wos elements; wo may alias wi),
// wc = fl(wo) in the cycle type ([n][B]).  DOTS: also the dot products of
// the new vector with the basis, from the basis values already in registers
// (the second Gram-Schmidt pass's, speculatively), to
// part[(blk * (nv + 1) + t) * B + b], and its squared norm to row nv; else
// the squared norm to part[blk * B + b].  skip: when non-null and *skip == 0
// the sweep does nothing.
template <int NG, class TU, bool DOTS>
__global__ __launch_bounds__(256) void k_kr_upd(int n, int B, int lbk, int chunk, int nv,
                                                const double* __restrict__ V, int mp1,
                                                const double* __restrict__ sig, const double* __restrict__ h,
                                                const double* wi, long wis, double* wo, long wos,
                                                TU* __restrict__ wc, double* __restrict__ part,
                                                const int* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip == 0) return;
  MGL_KR_CHUNK
  constexpr int NA = DOTS ? NG : 1;
  double hs[NG], acc[NA], ww = 0.0;
#pragma unroll
  for (int t = 0; t < NG; ++t) hs[t] = (lane_ok && t < nv) ? h[(size_t)t * B + b] * sig[(size_t)t * B + b] : 0.0;
#pragma unroll
  for (int t = 0; t < NA; ++t) acc[t] = 0.0;
  if (lane_ok) {
    for (long i = lo + rg; i < hi; i += rpb) {
      const double* vrow = V + (size_t)i * mp1 * B + b;
      // every load is issued (indices past nv - 1 repeat the last vector,
      // whose coefficient hs is zero there) so that all are in flight together
      double vr[NG];
#pragma unroll
      for (int t = 0; t < NG; ++t) vr[t] = vrow[(size_t)(t < nv ? t : nv - 1) * B];
      double v = wi[(size_t)i * wis + b];
#pragma unroll
      for (int t = 0; t < NG; ++t) v -= hs[t] * vr[t];
      wo[(size_t)i * wos + b] = v;
      put(wc + (size_t)i * B + b, v);
      ww += v * v;
      if constexpr (DOTS) {
#pragma unroll
        for (int t = 0; t < NG; ++t) acc[t] += v * vr[t];
      }
    }
  }
  if constexpr (DOTS) {
    double* out = part + (size_t)blk * (nv + 1) * B;
#pragma unroll
    for (int t = 0; t < NG; ++t)
      if (t < nv) kr_block_sum(lane_ok ? acc[t] * sig[(size_t)t * B + b] : 0.0, lbk, B, red, out + (size_t)t * B);
    kr_block_sum(ww, lbk, B, red, out + (size_t)nv * B);
  } else {
    kr_block_sum(ww, lbk, B, red, part + (size_t)blk * B);
  }
}

// vt_0 = r: the residual ([n][B]) into basis slot 0
__global__ __launch_bounds__(256) void k_kr_put0(int n, int B, int lbs, const double* __restrict__ r,
                                                 double* __restrict__ V, int mp1) {
  MGL_ROW_LANE(n)
  for (int b = lane; b < B; b += (1 << lbs)) V[(size_t)i * mp1 * B + b] = r[(size_t)i * B + b];
}

// out[i * B + b] = sum over blocks of part[(blk * nv + i) * B + b]; one
// workgroup of 1024 per i, one lane per column (2^lbk >= B lanes), each
// lane group summing a fixed strided subset of the blocks with eight
// independent partial sums, then a fixed pairwise tree (deterministic).
// skip: when non-null and *skip == 0, out = 0.
__global__ __launch_bounds__(1024) void k_kr_reduce(const double* __restrict__ part, int nblk, int nv, int B,
                                                    int lbk, double* __restrict__ out, const int* __restrict__ skip) {
  __shared__ double red[1024];
  const int i = blockIdx.x;
  const int LB = 1 << lbk, G = 1024 >> lbk;
  const int b = threadIdx.x & (LB - 1), g = (int)(threadIdx.x >> lbk);
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (b < B && !(skip && *skip == 0)) {
    int k = g;
    for (; k + 7 * G < nblk; k += 8 * G) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += part[((size_t)(k + u * G) * nv + i) * B + b];
    }
    for (; k < nblk; k += G) s[0] += part[((size_t)k * nv + i) * B + b];
  }
  red[threadIdx.x] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  __syncthreads();
  for (int h = G >> 1; h > 0; h >>= 1) {
    if (g < h) red[threadIdx.x] += red[threadIdx.x + h * LB];
    __syncthreads();
  }
  if (g == 0 && b < B) out[(size_t)i * B + b] = red[b];
}

// w = sig_j(b) * A z (FP64 operator, z in the cycle type); row tiles as the
// cycle sweeps.
template <int ROWS, bool WIDE, class TZ>
__global__ __launch_bounds__(256) void k_kr_amul(Lvl<double> L, int B, int lbs, const TZ* __restrict__ z,
                                                 const double* __restrict__ sig, double* __restrict__ w) {
  constexpr bool CS = WIDE && ROWS == 4;
  const Tile<ROWS, WIDE> t(L.n, lbs);
  if (WIDE && !t.any) return;
  double dg[ROWS];
  row_vals<WIDE, CS>(L.diag, t.row, t.row0, dg);
  for (int b = t.lane; b < B; b += t.LB) {
    double zv[ROWS], s[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      zv[r] = ldc<double>(z + (size_t)t.row[r] * B + b);
      s[r] = 0.0;
    }
    ell_dot<WIDE, CS>(L.w, L.ld, L.col, L.val, t.row, t.row0, z, B, b, s);
    const double sc = sig[b];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
      if (t.ok[r]) w[(size_t)t.row[r] * B + b] = sc * (s[r] + dg[r] * zv[r]);
  }
}

// Per-column state of one restart cycle, all arrays [.. * B + b]:
//   H[(i * m + j) * B + b]  Hessenberg (i <= m, j < m), rotated in place
//   cs, sn [m], g [m + 1]   Givens rotations and the rotated right-hand side
//   sig [m + 1]             basis scales, v_i = sig_i vt_i (0 once the column stopped)
//   act [B]                 1 while the column iterates in this cycle
//   jd  [B]                 iterations of this cycle that count for the column
//   flag [1]                1 when the current vector needs the second Gram-Schmidt pass
//   st  [3B + 1]            st[b] converged flag, st[B+b] total iterations,
//                           st[2B+b] status (0 met rtol, 5 not yet, 6 non-finite),
//                           st[3B] active count
struct KrState {
  double *H, *cs, *sn, *g, *sig, *fnorm;
  int *act, *jd, *flag, *st;
  int m;
};

__device__ __forceinline__ int kr_count(int act) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = act;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) cnt[threadIdx.x] += cnt[threadIdx.x + k];
    __syncthreads();
  }
  return cnt[0];
}

// Start of a restart cycle from beta[b] = ||f - A x|| (the residual is the
// unnormalised first basis vector): a column iterates if beta > rtol ||f||
// and beta is finite.  first: also records ||f|| (= beta of x = 0) and clears
// the totals.  One workgroup of 256, B <= 256.
__global__ __launch_bounds__(256) void k_kr_start(KrState S, int B, const double* __restrict__ beta, double rtol,
                                                  int first) {
  const int b = threadIdx.x;
  int a = 0;
  if (b < B) {
    const double bt = beta[b];
    if (first) { S.fnorm[b] = bt; S.st[B + b] = 0; }
    const double fn = S.fnorm[b];
    const bool conv = bt <= rtol * fn;
    const bool bad = !(bt == bt) || bt > 1.79e308;
    a = (!conv && !bad) ? 1 : 0;
    S.act[b] = a;
    S.jd[b] = 0;
    S.g[b] = bt;
    S.sig[b] = a ? 1.0 / bt : 0.0;
    S.st[b] = conv ? 1 : 0;
    S.st[2 * B + b] = conv ? 0 : (bad ? 6 : 5);
  }
  const int c = kr_count(a);
  if (threadIdx.x == 0) S.st[3 * B] = c;
}

// Second Gram-Schmidt pass needed when, for an active column, the first pass
// left less than eta of the vector's norm (n2 < eta^2 n1, squared norms).
__global__ __launch_bounds__(256) void k_kr_reorth(KrState S, int B, const double* __restrict__ n1,
                                                   const double* __restrict__ n2, double eta2) {
  const int b = threadIdx.x;
  const int need = (b < B && S.act[b] && !(n2[b] >= eta2 * n1[b])) ? 1 : 0;
  const int c = kr_count(need);
  if (threadIdx.x == 0) *S.flag = c > 0 ? 1 : 0;
}

// Column j of the Hessenberg matrix: h_ij = h1_i + h2_i with a second pass
// (else h1_i), h_{j+1,j} = ||w|| (n4 after a second pass, else n2);
// previous rotations applied, new rotation, residual estimate |g_{j+1}|.  A
// column stops at the first j with |g_{j+1}| <= rtol ||f|| (or at a
// breakdown, where the Krylov space is invariant and the least-squares
// solution exact); sig_{j+1} = 1 / ||w|| while it continues.  One workgroup
// of 256, B <= 256.
__global__ __launch_bounds__(256) void k_kr_givens(KrState S, int B, int j, const double* __restrict__ h1,
                                                   const double* __restrict__ h2, const double* __restrict__ n2,
                                                   const double* __restrict__ n4, double rtol) {
  const int b = threadIdx.x;
  int a = 0;
  if (b < B && S.act[b]) {
    const int m = S.m;
    double* H = S.H;
    auto at = [&](int i, int jj) -> double& { return H[((size_t)i * m + jj) * B + b]; };
    const bool two = *S.flag != 0;
    for (int i = 0; i <= j; ++i) at(i, j) = h1[(size_t)i * B + b] + (two ? h2[(size_t)i * B + b] : 0.0);
    const double beta = sqrt(two ? n4[b] : n2[b]);
    at(j + 1, j) = beta;
    for (int i = 0; i < j; ++i) {
      const double c = S.cs[(size_t)i * B + b], s = S.sn[(size_t)i * B + b];
      const double x = at(i, j), y = at(i + 1, j);
      at(i, j) = c * x + s * y;
      at(i + 1, j) = -s * x + c * y;
    }
    const double x = at(j, j), y = at(j + 1, j);
    const double d = hypot(x, y);
    const double fn = S.fnorm[b];
    if (!(d > 0.0) || !(d <= 1.79e308)) {
      // the preconditioned vector vanished or is not finite: stop before it
      a = 0;
    } else {
      const double c = x / d, s = y / d;
      S.cs[(size_t)j * B + b] = c;
      S.sn[(size_t)j * B + b] = s;
      at(j, j) = d;
      at(j + 1, j) = 0.0;
      const double gj = S.g[(size_t)j * B + b];
      S.g[(size_t)(j + 1) * B + b] = -s * gj;
      S.g[(size_t)j * B + b] = c * gj;
      S.jd[b] = j + 1;
      a = (fabs(s * gj) > rtol * fn && beta > 0.0) ? 1 : 0;
    }
    S.act[b] = a;
    S.sig[(size_t)(j + 1) * B + b] = a ? 1.0 / beta : 0.0;
  } else if (b < B) {
    S.sig[(size_t)(j + 1) * B + b] = 0.0;
  }
  const int c = kr_count(a);
  if (threadIdx.x == 0) S.st[3 * B] = c;
}

// y = R^{-1} g over the column's jd iterations (back substitution on the
// rotated Hessenberg matrix), then y_k <- y_k sig_k so that x += sum y_k zt_k
// with the stored (unscaled) preconditioned vectors zt_k; y_k = 0 for k >= jd.
// Adds jd to the column's total.
__global__ __launch_bounds__(256) void k_kr_lsq(KrState S, int B, int nz, double* __restrict__ y) {
  const int b = threadIdx.x;
  if (b >= B) return;
  const int m = S.m, k = S.jd[b];
  const double* H = S.H;
  for (int i = nz - 1; i >= 0; --i) {
    double v = 0.0;
    if (i < k) {
      v = S.g[(size_t)i * B + b];
      for (int l = i + 1; l < k; ++l) v -= H[((size_t)i * m + l) * B + b] * y[(size_t)l * B + b];
      const double r = H[((size_t)i * m + i) * B + b];
      v = r != 0.0 ? v / r : 0.0;
    }
    y[(size_t)i * B + b] = v;
  }
  for (int i = 0; i < nz; ++i) y[(size_t)i * B + b] *= S.sig[(size_t)i * B + b];
  S.st[B + b] += k;
}

// x(row, b) += sum_{k < nz} y[k * B + b] * Z_k(row, b), Z_k = Z + k * zs.
template <class TZ>
__global__ __launch_bounds__(256) void k_kr_xupd(int n, int B, int lbs, int nz, const TZ* __restrict__ Z, long zs,
                                                 const double* __restrict__ y, double* __restrict__ x) {
  MGL_ROW_LANE(n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    double v = x[o];
    for (int k = 0; k < nz; ++k) v += y[(size_t)k * B + b] * ldc<double>(Z + (size_t)k * zs + o);
    x[o] = v;
  }
}

}  // namespace mgl
