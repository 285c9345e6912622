// Device kernels of flexible GMRES (Saad's FGMRES with right preconditioning
// and restarts) around the learnable cycle, for B independent columns at once
// ([n][B] layout, FP64 Krylov vectors, preconditioned vectors in the cycle
// type).  Orthogonalisation is classical Gram-Schmidt applied twice (CGS2):
// every pass is one streaming sweep over the basis, and the dot products are
// reduced in a fixed order (deterministic).  The small per-column problems
// (Hessenberg columns, Givens rotations, least squares) run one work-item per
// column.
#pragma once
#include "kernels.hpp"

namespace mgl {

constexpr int kKrNG = 8;   // basis vectors per accumulation group of the dot sweep

// Rows [blk * chunk, min(n, (blk + 1) * chunk)) of logical block blk.
#define MGL_KR_CHUNK                                                   \
  const int LB = 1 << lbs, rpb = 256 >> lbs;                           \
  const int lane = threadIdx.x & (LB - 1);                             \
  const int rg = (int)(threadIdx.x >> lbs);                            \
  const int blk = xcd_block();                                         \
  const long lo = (long)blk * chunk;                                   \
  const long hi = lo + chunk < n ? lo + chunk : (long)n;

// part[(blk * nv + i) * B + b] = sum over the block's rows of w(row, b) * V_i(row, b),
// V_i = V + i * vs.  B <= 256 (at most 4 columns per work-item).
__global__ __launch_bounds__(256) void k_kr_dots(int n, int B, int lbs, int chunk, int nv,
                                                 const double* __restrict__ V, long vs,
                                                 const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[256];
  MGL_KR_CHUNK
  for (int i0 = 0; i0 < nv; i0 += kKrNG) {
    double acc[kKrNG][4];
#pragma unroll
    for (int t = 0; t < kKrNG; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[t][q] = 0.0;
    for (long i = lo + rg; i < hi; i += rpb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = lane + q * LB;
        if (b >= B) break;
        const size_t o = (size_t)i * B + b;
        const double wv = w[o];
#pragma unroll
        for (int t = 0; t < kKrNG; ++t)
          if (i0 + t < nv) acc[t][q] += wv * V[(size_t)(i0 + t) * vs + o];
      }
    }
#pragma unroll
    for (int t = 0; t < kKrNG; ++t) {
      if (i0 + t >= nv) break;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q * LB >= B) break;
        red[threadIdx.x] = acc[t][q];
        __syncthreads();
        const int b = q * LB + lane;
        if (rg == 0 && b < B) {
          double sum = 0.0;
          for (int g = 0; g < rpb; ++g) sum += red[g * LB + lane];
          part[((size_t)blk * nv + i0 + t) * B + b] = sum;
        }
        __syncthreads();
      }
    }
  }
}

// out[i * B + b] (+)= sum over blocks of part[(blk * nv + i) * B + b]; one
// workgroup per i, fixed strided order and fixed sequential combine.
__global__ __launch_bounds__(256) void k_kr_reduce(const double* __restrict__ part, int nblk, int nv, int B,
                                                   int lbs, double* __restrict__ out, int add) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const int LB = 1 << lbs, G = 256 >> lbs;
  const int lane = threadIdx.x & (LB - 1), g = (int)(threadIdx.x >> lbs);
  for (int b0 = 0; b0 < B; b0 += LB) {
    const int b = b0 + lane;
    double s = 0.0;
    if (b < B)
      for (int k = g; k < nblk; k += G) s += part[((size_t)k * nv + i) * B + b];
    red[threadIdx.x] = s;
    __syncthreads();
    if (g == 0 && b < B) {
      double t = 0.0;
      for (int k = 0; k < G; ++k) t += red[k * LB + lane];
      out[(size_t)i * B + b] = add ? out[(size_t)i * B + b] + t : t;
    }
    __syncthreads();
  }
}

// w(row, b) -= sum_{i < nv} h[i * B + b] * V_i(row, b) over the block's rows;
// norm2: part[blk * B + b] = sum of the new w(row, b)^2 (else part unused).
__global__ __launch_bounds__(256) void k_kr_orth(int n, int B, int lbs, int chunk, int nv,
                                                 const double* __restrict__ V, long vs,
                                                 const double* __restrict__ h, double* __restrict__ w,
                                                 int norm2, double* __restrict__ part) {
  __shared__ double red[256];
  MGL_KR_CHUNK
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i = lo + rg; i < hi; i += rpb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = lane + q * LB;
      if (b >= B) break;
      const size_t o = (size_t)i * B + b;
      double wv = w[o];
      for (int k = 0; k < nv; ++k) wv -= h[(size_t)k * B + b] * V[(size_t)k * vs + o];
      w[o] = wv;
      acc[q] += wv * wv;
    }
  }
  if (!norm2) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q * LB >= B) break;
    red[threadIdx.x] = acc[q];
    __syncthreads();
    const int b = q * LB + lane;
    if (rg == 0 && b < B) {
      double sum = 0.0;
      for (int g = 0; g < rpb; ++g) sum += red[g * LB + lane];
      part[(size_t)blk * B + b] = sum;
    }
    __syncthreads();
  }
}

// w = A z (FP64 operator, z in the cycle type); row tiles as the cycle sweeps.
template <int ROWS, bool WIDE, class TZ>
__global__ __launch_bounds__(256) void k_kr_amul(Lvl<double> L, int B, int lbs, const TZ* __restrict__ z,
                                                 double* __restrict__ w) {
  constexpr bool CS = WIDE && ROWS == 4;
  const Tile<ROWS, WIDE> t(L.n, lbs);
  if (WIDE && !t.any) return;
  double dg[ROWS];
  row_vals<WIDE, CS>(L.diag, t.row, t.row0, dg);
  for (int b = t.lane; b < B; b += t.LB) {
    double s[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) s[r] = dg[r] * ldc<double>(z + (size_t)t.row[r] * B + b);
    ell_dot<WIDE, CS>(L.w, L.ld, L.col, L.val, t.row, t.row0, z, B, b, s);
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
      if (t.ok[r]) w[(size_t)t.row[r] * B + b] = s[r];
  }
}

// v = w * s[b] (v may alias w); vc = fl(v) in the cycle type (the
// preconditioner's input), optional.
template <class TU>
__global__ __launch_bounds__(256) void k_kr_scale(int n, int B, int lbs, const double* w,
                                                  const double* __restrict__ s, double* v, TU* __restrict__ vc) {
  MGL_ROW_LANE(n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    const double x = w[o] * s[b];
    v[o] = x;
    if (vc) put(vc + o, x);
  }
}

// Per-column state of one restart cycle, all arrays [.. * B + b]:
//   H[(i * m + j) * B + b]  Hessenberg (i <= m, j < m), rotated in place
//   cs, sn [m], g [m + 1]   Givens rotations and the rotated right-hand side
//   act [B]                 1 while the column iterates in this cycle
//   jd  [B]                 iterations of this cycle that count for the column
//   s   [B]                 scale of the next basis vector (1/beta, 0 if frozen)
//   st  [3B + 1]            st[b] converged flag, st[B+b] total iterations,
//                           st[2B+b] status (0 met rtol, 5 not yet, 6 non-finite),
//                           st[3B] active count
struct KrState {
  double *H, *cs, *sn, *g, *s, *fnorm;
  int *act, *jd, *st;
  int m;
};

__device__ __forceinline__ void kr_count(int act, int* out) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = act;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) cnt[threadIdx.x] += cnt[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = cnt[0];
}

// Start of a restart cycle from beta[b] = ||f - A x||: a column iterates if
// beta > rtol ||f|| and beta is finite.  first: also records ||f|| (= beta of x = 0) and clears
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
    S.s[b] = a ? 1.0 / bt : 0.0;
    S.st[b] = conv ? 1 : 0;
    S.st[2 * B + b] = conv ? 0 : (bad ? 6 : 5);
  }
  kr_count(a, S.st + 3 * B);
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes
// (h1 + h2) and ||w|| (nrm2 = ||w||^2), previous rotations applied, new
// rotation, residual estimate |g_{j+1}|; a column stops at the first j with
// |g_{j+1}| <= rtol ||f|| (or at a breakdown, where the Krylov space is
// invariant and the least-squares solution exact).  One workgroup of 256, B <= 256.
__global__ __launch_bounds__(256) void k_kr_givens(KrState S, int B, int j, const double* __restrict__ h1,
                                                   const double* __restrict__ h2, const double* __restrict__ nrm2,
                                                   double rtol) {
  const int b = threadIdx.x;
  int a = 0;
  if (b < B && S.act[b]) {
    const int m = S.m;
    double* H = S.H;
    auto at = [&](int i, int jj) -> double& { return H[((size_t)i * m + jj) * B + b]; };
    for (int i = 0; i <= j; ++i) at(i, j) = h1[(size_t)i * B + b] + h2[(size_t)i * B + b];
    const double beta = sqrt(nrm2[b]);
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
    S.s[b] = a ? 1.0 / beta : 0.0;
  } else if (b < B) {
    S.s[b] = 0.0;
  }
  kr_count(a, S.st + 3 * B);
}

// y = R^{-1} g over the column's jd iterations (back substitution on the
// rotated Hessenberg matrix); y[k] = 0 for k >= jd.  Adds jd to the total.
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
