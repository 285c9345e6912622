// Device kernels of the learnable V-cycle for gfx950 (CDNA4, wave64).
//
// Every sweep is bandwidth bound: a thread block of 256 work-items maps
// 2^lbs lanes onto each matrix row and the lanes onto the B right-hand sides
// stored contiguously ([n][B] layout), so one neighbour row is one coalesced
// load per wavefront and the (wave-uniform) ELL index/value loads are shared
// by all columns.  With B = 1 one lane is one row and the slot-major ELL
// arrays are read fully coalesced.  Block ids are remapped so that every XCD
// walks one contiguous range of rows: neighbour rows (+-1, +-grid line) are
// then reused from that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgl {

struct bf16_t { uint16_t bits; };

__device__ __forceinline__ double cvt_d(double v) { return v; }
__device__ __forceinline__ double cvt_d(float v) { return (double)v; }
__device__ __forceinline__ float cvt_f(double v) { return (float)v; }
__device__ __forceinline__ float cvt_f(float v) { return v; }
__device__ __forceinline__ float cvt_f(bf16_t v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

template <class C> struct Cv;
template <> struct Cv<double> {
  template <class T> __device__ static __forceinline__ double ld(T v) { return cvt_d(v); }
};
template <> struct Cv<float> {
  template <class T> __device__ static __forceinline__ float ld(T v) { return cvt_f(v); }
};
template <class C, class T> __device__ __forceinline__ C ldc(const T* p) { return Cv<C>::ld(*p); }

// round-to-nearest-even FP32 -> BF16 (quiet NaN kept)
__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16_t{(uint16_t)((u >> 16) | 0x40u)};
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16_t{(uint16_t)(u >> 16)};
}
__device__ __forceinline__ void put(double* p, double v) { *p = v; }
__device__ __forceinline__ void put(float* p, float v) { *p = v; }
__device__ __forceinline__ void put(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void put(bf16_t* p, float v) { *p = f2bf(v); }

// Level operator in ELL form.  Off-diagonal slots are slot-major
// (entry (k, i) at k*n + i); a padding slot has col == i and val == 0.
template <class C> struct Lvl {
  int n;
  int w;                    // off-diagonal ELL width of A
  const int* col;
  const C* val;
  const C* diag;
  const C* invdiag;
  int wg;                   // ELL width of the graph
  const int* gcol;          // graph neighbours (padding col == i)
  const C* invdeg;          // 1/|N(i)|, 0 for an isolated node
};

// Transfer operator (P, R or their transposes) in ELL form, padding val == 0.
template <class C> struct Xfer {
  int n;                    // rows
  int w;
  const int* col;
  const C* val;
};

// Remap hardware block ids (dispatched round-robin over the 8 XCDs) so that
// XCD x processes one contiguous range of logical blocks.
__device__ __forceinline__ int xcd_block() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

#define MGL_ROW_LANE(NROWS)                                                   \
  const long gt_ = (long)xcd_block() * blockDim.x + threadIdx.x;              \
  const int i = (int)(gt_ >> lbs);                                            \
  const int lane = (int)(gt_ & ((1 << lbs) - 1));                             \
  if (i >= (NROWS)) return;

// (A u)_i for column b
template <class C, class TU>
__device__ __forceinline__ C row_Au(const Lvl<C>& L, const TU* __restrict__ u, int i, int B, int b) {
  C au = L.diag[i] * ldc<C>(u + (size_t)i * B + b);
  for (int k = 0; k < L.w; ++k) {
    const int j = L.col[(size_t)k * L.n + i];
    au += L.val[(size_t)k * L.n + i] * ldc<C>(u + (size_t)j * B + b);
  }
  return au;
}

// (M y)_i = invdeg_i * sum_{j in N(i)} y_j
template <class C, class TY>
__device__ __forceinline__ C row_My(const Lvl<C>& L, const TY* __restrict__ y, int i, int B, int b) {
  C s = C(0);
  for (int k = 0; k < L.wg; ++k) {
    const int j = L.gcol[(size_t)k * L.n + i];
    if (j != i) s += ldc<C>(y + (size_t)j * B + b);
  }
  return L.invdeg[i] * s;
}

// (M^T z)_i = sum_{j in N(i)} invdeg_j z_j   (graph pattern is symmetric)
template <class C, class TY>
__device__ __forceinline__ C row_MTz(const Lvl<C>& L, const TY* __restrict__ z, int i, int B, int b) {
  C s = C(0);
  for (int k = 0; k < L.wg; ++k) {
    const int j = L.gcol[(size_t)k * L.n + i];
    if (j != i) s += L.invdeg[j] * ldc<C>(z + (size_t)j * B + b);
  }
  return s;
}

// out = [invdiag *] (f - A u); uz: u is identically zero.
template <class C, class TU, class TO>
__global__ __launch_bounds__(256) void k_resid(Lvl<C> L, int B, int lbs, const TU* __restrict__ f,
                                               const TU* __restrict__ u, int uz, int jacobi,
                                               TO* __restrict__ out) {
  MGL_ROW_LANE(L.n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    C v = ldc<C>(f + o);
    if (!uz) v -= row_Au(L, u, i, B, b);
    if (jacobi) v *= L.invdiag[i];
    put(out + o, v);
  }
}

// Horner hop v = a * (M yin)_i + c * x_i.
//   mode 0: out = v (type TO)
//   mode 1: out = (oz ? 0 : out) + scale * v
template <class C, class TY, class TX, class TO>
__global__ __launch_bounds__(256) void k_hop(Lvl<C> L, int B, int lbs, const TY* __restrict__ yin, C a,
                                             const TX* __restrict__ x, C c, TO* out, int mode, C scale,
                                             int oz) {
  MGL_ROW_LANE(L.n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    const C v = a * row_My(L, yin, i, B, b) + c * ldc<C>(x + o);
    if (mode == 0) put(out + o, v);
    else put(out + o, (oz ? C(0) : ldc<C>(out + o)) + scale * v);
  }
}

// out = (oz ? 0 : out) + alpha * x
template <class C, class TX, class TO>
__global__ __launch_bounds__(256) void k_axpy(int n, int B, int lbs, const TX* __restrict__ x, C alpha,
                                              TO* out, int oz) {
  MGL_ROW_LANE(n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    put(out + o, (oz ? C(0) : ldc<C>(out + o)) + alpha * ldc<C>(x + o));
  }
}

// Restriction onto coarse row I:  rc_I = scale * sum_j R_Ij v_j  with
//   mode 0: v = y
//   mode 1: v = a (M y)_j + c x_j       (last hop of Phi_R fused)
//   mode 2: v = f_j - (A u)_j           (residual fused; uz: u == 0)
template <class C, class TU, class TY, class TX>
__global__ __launch_bounds__(256) void k_restrict(Xfer<C> R, Lvl<C> L, int B, int lbs, int mode,
                                                  const TY* __restrict__ y, C a, const TX* __restrict__ x,
                                                  C c, const TU* __restrict__ f, const TU* __restrict__ u,
                                                  int uz, C scale, TU* __restrict__ rc) {
  MGL_ROW_LANE(R.n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    C acc = C(0);
    for (int k = 0; k < R.w; ++k) {
      const C wgt = R.val[(size_t)k * R.n + i];
      if (wgt == C(0)) continue;
      const int j = R.col[(size_t)k * R.n + i];
      C v;
      if (mode == 0) {
        v = ldc<C>(y + (size_t)j * B + b);
      } else if (mode == 1) {
        v = a * row_My(L, y, j, B, b) + c * ldc<C>(x + (size_t)j * B + b);
      } else {
        v = ldc<C>(f + (size_t)j * B + b);
        if (!uz) v -= row_Au(L, u, j, B, b);
      }
      acc += wgt * v;
    }
    put(rc + (size_t)i * B + b, scale * acc);
  }
}

// Prolongation (or any ELL transfer applied to a coarse vector):
//   mode 0: out = scale * (P ec)     mode 1: out = (oz ? 0 : out) + scale * (P ec)
template <class C, class TU, class TO>
__global__ __launch_bounds__(256) void k_prolong(Xfer<C> P, int B, int lbs, const TU* __restrict__ ec,
                                                 TO* out, int mode, C scale, int oz) {
  MGL_ROW_LANE(P.n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    C acc = C(0);
    for (int k = 0; k < P.w; ++k) {
      const C wgt = P.val[(size_t)k * P.n + i];
      const int j = P.col[(size_t)k * P.n + i];
      acc += wgt * ldc<C>(ec + (size_t)j * B + b);
    }
    const size_t o = (size_t)i * B + b;
    if (mode == 0) put(out + o, scale * acc);
    else put(out + o, (oz ? C(0) : ldc<C>(out + o)) + scale * acc);
  }
}

// Coarsest level: u = Ainv f (or Ainv^T f), Ainv dense row-major FP64.
template <class TU>
__global__ __launch_bounds__(256) void k_coarse(int n, int B, const double* __restrict__ Ainv,
                                                const TU* __restrict__ f, TU* __restrict__ u, int trans) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * B) return;
  const int i = (int)(t / B), b = (int)(t % B);
  double acc = 0.0;
  for (int j = 0; j < n; ++j) {
    const double a = trans ? Ainv[(size_t)j * n + i] : Ainv[(size_t)i * n + j];
    acc += a * (double)f[(size_t)j * B + b];
  }
  put(u + (size_t)i * B + b, acc);
}

// Gauss-Jordan inversion with partial pivoting of the dense matrix held in
// W[0:n, 0:n] of the row-major n x 2n array W (W[:, n:2n] must be I on
// entry).  One block of 1024 threads.  On exit W[:, n:2n] = A^{-1}.
// *info = 0 on success, k+1 if the pivot of column k is zero.
__global__ __launch_bounds__(1024) void k_gauss_jordan(int n, double* W, int* info) {
  __shared__ double sval[1024];
  __shared__ int sidx[1024];
  __shared__ int piv_s;
  __shared__ int fail;
  const int t = threadIdx.x, T = blockDim.x, m = 2 * n;
  if (t == 0) fail = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int r = k + t; r < n; r += T) {
      const double v = fabs(W[(size_t)r * m + k]);
      if (v > best) { best = v; bi = r; }
    }
    sval[t] = best;
    sidx[t] = bi;
    __syncthreads();
    for (int s = T / 2; s > 0; s >>= 1) {
      if (t < s) {
        const double o = sval[t + s];
        const int oi = sidx[t + s];
        if (o > sval[t] || (o == sval[t] && oi < sidx[t])) { sval[t] = o; sidx[t] = oi; }
      }
      __syncthreads();
    }
    if (t == 0) {
      piv_s = sidx[0];
      if (!(sval[0] > 0.0)) fail = k + 1;
    }
    __syncthreads();
    if (fail) break;
    const int p = piv_s;
    if (p != k)
      for (int c = t; c < m; c += T) {
        const double a = W[(size_t)k * m + c];
        W[(size_t)k * m + c] = W[(size_t)p * m + c];
        W[(size_t)p * m + c] = a;
      }
    __syncthreads();
    const double inv = 1.0 / W[(size_t)k * m + k];
    __syncthreads();
    for (int c = t; c < m; c += T) W[(size_t)k * m + c] *= inv;
    __syncthreads();
    for (long e = t; e < (long)n * m; e += T) {
      const int r = (int)(e / m), c = (int)(e % m);
      if (r == k) continue;
      const double fr = W[(size_t)r * m + k];
      if (c == k) continue;  // column k is cleared after the sweep
      W[(size_t)r * m + c] -= fr * W[(size_t)k * m + c];
    }
    __syncthreads();
    for (int r = t; r < n; r += T)
      if (r != k) W[(size_t)r * m + k] = 0.0;
    __syncthreads();
  }
  if (t == 0) *info = fail;
}

// ------------------------------------------------------------------ FP64 outer residual
// r = f - A u in FP64; writes r64 (optional) and rc = fl(r) in the cycle type
// (optional); per-block, per-column partial sums of r^2 to part[block][B].
// Fixed grid; rows are visited grid-stride in a fixed order (deterministic).
template <class TR>
__global__ __launch_bounds__(256) void k_outer_resid(Lvl<double> L, int B, int lbs, const double* __restrict__ f,
                                                     const double* __restrict__ u, double* __restrict__ r64,
                                                     TR* __restrict__ rc, double* __restrict__ part) {
  __shared__ double red[256 * 4];
  const int LB = 1 << lbs, rows_per_block = 256 >> lbs;
  const int lane = threadIdx.x & (LB - 1), rg = threadIdx.x >> lbs;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = blockIdx.x * rows_per_block + rg; i < L.n; i += gridDim.x * rows_per_block) {
    int q = 0;
    for (int b = lane; b < B; b += LB, ++q) {
      const size_t o = (size_t)i * B + b;
      const double v = f[o] - row_Au(L, u, i, B, b);
      if (r64) r64[o] = v;
      if (rc) put(rc + o, v);
      acc[q] += v * v;
    }
  }
  for (int q = 0; q < 4; ++q) red[q * 256 + threadIdx.x] = acc[q];
  __syncthreads();
  if (rg == 0) {
    int q = 0;
    for (int b = lane; b < B; b += LB, ++q) {
      double s = 0.0;
      for (int g = 0; g < rows_per_block; ++g) s += red[q * 256 + g * LB + lane];
      part[(size_t)blockIdx.x * B + b] = s;
    }
  }
}

// norms[b] = sqrt(sum over blocks of part[block][b]) (fixed order)
__global__ void k_norm_final(const double* __restrict__ part, int nblk, int B, double* __restrict__ norms) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int g = 0; g < nblk; ++g) s += part[(size_t)g * B + b];
  norms[b] = sqrt(s);
}

// Per-column solver bookkeeping after the residual of iterate m.
// st: [0,B) active, [B,2B) iters, [2B,3B) status; 3B: active count.
__global__ void k_solve_check(const double* __restrict__ norms, double* __restrict__ fnorm,
                              double* __restrict__ init, int* st, int B, double rtol, double divf, int first) {
  __shared__ int cnt[256];
  const int b = threadIdx.x;
  int act = 0;
  if (b < B) {
    const double nr = norms[b];
    if (first) { init[b] = nr; st[b] = 1; st[B + b] = 0; st[2 * B + b] = 5; }
    act = st[b];
    if (act) {
      const double fn = fnorm[b];
      const double rel = fn > 0.0 ? nr / fn : nr;
      if (!(nr == nr) || nr > 1.79e308 || (divf > 0.0 && nr > divf * init[b] && nr > 0.0)) {
        act = 0; st[2 * B + b] = 6;
      } else if (rel <= rtol) {
        act = 0; st[2 * B + b] = 0;
      }
      st[b] = act;
      if (act) st[B + b] += 1;
    }
  }
  cnt[threadIdx.x] = act;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) st[3 * B] = cnt[0];
}

// u += e for active columns (act == nullptr: all columns)
template <class TU>
__global__ __launch_bounds__(256) void k_update(int n, int B, int lbs, const TU* __restrict__ e,
                                                double* u, const int* __restrict__ act, double sign) {
  MGL_ROW_LANE(n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    if (act && !act[b]) continue;
    const size_t o = (size_t)i * B + b;
    u[o] += sign * (double)e[o];
  }
}

template <class TI, class TO>
__global__ __launch_bounds__(256) void k_copy(long cnt, const TI* __restrict__ in, TO* __restrict__ out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) put(out + t, in[t]);
}

template <class T>
__global__ __launch_bounds__(256) void k_fill0(long cnt, T* out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) out[t] = T(0);
}

// ------------------------------------------------------------------ adjoint sweeps
// Block-wide FP64 sum, written to part[blockIdx.x] (deterministic tree).
__device__ __forceinline__ void block_sum_store(double v, double* part, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One power step of a transposed convolution:
//   zin == nullptr: z = zsrc (k = 0);  else z = M^T zin
//   acc = (first ? 0 : acc) + c * z;  zout = z (if zout);  part <- sum(z * s)
// The launch must cover every row (no early return before the block sum).
template <class C, class TZ, class TS>
__global__ __launch_bounds__(256) void k_hopT(Lvl<C> L, int B, int lbs, const TZ* __restrict__ zin,
                                              const TZ* __restrict__ zsrc, TZ* __restrict__ zout, C c,
                                              TZ* acc, int first, const TS* __restrict__ s,
                                              double* __restrict__ part) {
  __shared__ double red[256];
  const long gt = (long)xcd_block() * blockDim.x + threadIdx.x;
  const int i = (int)(gt >> lbs), lane = (int)(gt & ((1 << lbs) - 1));
  double d = 0.0;
  if (i < L.n) {
    for (int b = lane; b < B; b += (1 << lbs)) {
      const size_t o = (size_t)i * B + b;
      const C z = zin ? row_MTz(L, zin, i, B, b) : ldc<C>(zsrc + o);
      if (zout) put(zout + o, z);
      put(acc + o, (first ? C(0) : ldc<C>(acc + o)) + c * z);
      d += (double)z * (double)ldc<C>(s + o);
    }
  }
  block_sum_store(d, part, red);
}

// Tail of a transposed smoothing / residual step:
//   q = alpha * [invdiag *] acc;  gf = (gz ? 0 : gf) + q  (gf optional)
template <class C, class TZ>
__global__ __launch_bounds__(256) void k_scale_acc(Lvl<C> L, int B, int lbs, const TZ* __restrict__ acc,
                                                   C alpha, int jacobi, TZ* __restrict__ q, TZ* gf, int gz) {
  MGL_ROW_LANE(L.n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    C v = alpha * ldc<C>(acc + o);
    if (jacobi) v *= L.invdiag[i];
    put(q + o, v);
    if (gf) put(gf + o, (gz ? C(0) : ldc<C>(gf + o)) + v);
  }
}

// g_out = g_in - A q  (A symmetric, so A^T q = A q); g_out may alias g_in.
template <class C, class TZ>
__global__ __launch_bounds__(256) void k_sub_Aq(Lvl<C> L, int B, int lbs, const TZ* gin,
                                                const TZ* __restrict__ q, TZ* gout) {
  MGL_ROW_LANE(L.n)
  for (int b = lane; b < B; b += (1 << lbs)) {
    const size_t o = (size_t)i * B + b;
    put(gout + o, ldc<C>(gin + o) - row_Au(L, q, i, B, b));
  }
}

// dots[s] = sum_{g < cnt[s]} part[off[s] + g]
__global__ void k_dots_final(const double* __restrict__ part, const long* __restrict__ off,
                             const int* __restrict__ cnt, int nslots, double* __restrict__ dots) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  if (s >= nslots) return;
  double v = 0.0;
  for (int g = threadIdx.x; g < cnt[s]; g += blockDim.x) v += part[off[s] + g];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) dots[s] = red[0];
}

// Parameter gradients from the dot products, in a fixed order.
// desc[s] = {kind (0 smoother, 1 restriction, 2 prolongation), level, k}.
// Smoother dot e = <(M^T)^k g, s> with s = D^{-1}(f - A u):
//   dc_k += eta theta e,  deta += theta c_k e,  dtheta += eta c_k e.
// Transfer dots give dc_k directly.
__global__ void k_grad_combine(const double* __restrict__ dots, const int* __restrict__ desc, int nslots,
                               const double* __restrict__ prm, int per, int KB, int KR, double* __restrict__ g,
                               int np) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int t = 0; t < np; ++t) g[t] = 0.0;
  for (int s = 0; s < nslots; ++s) {
    const int kind = desc[3 * s], l = desc[3 * s + 1], k = desc[3 * s + 2];
    const double* p = prm + (size_t)l * per;
    double* gl = g + (size_t)l * per;
    const double e = dots[s];
    if (kind == 0) {
      const double th = p[0], et = p[1], ck = p[2 + k];
      gl[2 + k] += et * th * e;
      gl[1] += th * ck * e;
      gl[0] += et * ck * e;
    } else if (kind == 1) {
      gl[2 + KB + 1 + k] += e;
    } else {
      gl[2 + KB + 1 + KR + 1 + k] += e;
    }
  }
}

}  // namespace mgl
