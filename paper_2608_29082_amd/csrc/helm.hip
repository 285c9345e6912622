// Learnable V-cycle for complex Helmholtz systems with two features per node
// (see include/mgh.h), its full multigrid and complex flexible GMRES.
//
// Vectors are complex [n][B] arrays (float2 / double2 per value): one
// work-item per (row, column) with the B columns of a row on adjacent lanes,
// so every neighbour row is one coalesced load.  Operators are slot-major ELL
// arrays (entry (s, i) at s * n + i).  The per-level sweeps (residual with the
// complex Jacobi scale, the convolution hops with 2 x 2 feature mixing, the
// transfers, the dense coarsest solve) are bandwidth bound and stream their
// operands once.  A GMRES smoothing step (v Arnoldi steps with block-wide
// reductions, the small least-squares problem and the update) runs as one
// kernel with one work-group per column, its vectors in LDS where they fit:
// the levels that use it are the coarse ones (k h > 1/2), where a launch per
// Arnoldi sweep would cost more than the sweep.  The outer FGMRES runs in
// FP64 with multi-block reductions in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "mgh.h"

namespace {

thread_local std::string h_err;

mg_status hfail(mg_status s, const std::string& m) {
  h_err = m;
  return s;
}

#define H_TRY(...)                             \
  do {                                         \
    mg_status s_ = (__VA_ARGS__);              \
    if (s_ != MG_OK) return s_;                \
  } while (0)
#define H_HIP(x)                                                                                 \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) return hfail(MG_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define H_LAUNCH()                                                                               \
  do {                                                                                           \
    hipError_t e_ = hipGetLastError();                                                           \
    if (e_ != hipSuccess)                                                                        \
      return hfail(MG_ERR_HIP, std::string("kernel launch at line ") + std::to_string(__LINE__) + ": " + \
                                   hipGetErrorString(e_));                                       \
  } while (0)

constexpr int kMaxK = 8, kMaxV = 8, kMaxNu = 8, kMaxB = 256, kGT = 512, kKrBlocks = 1024, kNG = 8;
// per-work-item partial sums of a GMRES smoothing step: 2 (kMaxV + 1) dot
// products (re, im) and one squared norm in the last slot
constexpr int kAcc = 2 * (kMaxV + 1) + 1, kNorm = kAcc - 1;
// vectors of a GMRES smoothing step: r, d0, V_0 .. V_v, and at least the two
// Horner buffers in slots 3 and 4
constexpr int hz_slots(int v) { return v + 3 > 5 ? v + 3 : 5; }
// dynamic LDS of the LDS-resident GMRES smoothing step (static shared ~4 KB besides)
constexpr int kGmresLds = 144 * 1024;
// work-items of the GMRES smoothing step with its vectors in HBM scratch
constexpr int kGTH = 1024;

template <class T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };
template <class T> using cx = typename C2<T>::t;

template <class T> struct W2 { T a, b, c, d; };          // [[a, b], [c, d]] acting on (re, im)
template <class T> struct WK { W2<T> w[kMaxK + 1]; };

template <class T> struct CEll { int n, w; const int* col; const cx<T>* val; };   // complex, square
template <class T> struct REll { int n, w; const int* col; const T* val; };       // real transfer
struct GEll { int n, w; const int* col; };                                         // graph (padding col == i)

template <class T>
__device__ __forceinline__ cx<T> mkc(T r, T i) {
  cx<T> z;
  z.x = r;
  z.y = i;
  return z;
}
template <class T>
__device__ __forceinline__ cx<T> mixw(const W2<T>& W, cx<T> x) {
  return mkc<T>(W.a * x.x + W.b * x.y, W.c * x.x + W.d * x.y);
}
// (A x)_i of a complex ELL matrix, accumulated in AT.  Slots go in groups of
// kSlots: all column indices and values of a group are loaded before the
// gathers, so a row costs one dependent round trip per group.
constexpr int kSlots = 8;
template <class AT, class T, class X, int SG = kSlots>
__device__ __forceinline__ void ell_cmul(const CEll<T>& A, const cx<X>* x, int i, int B, int b, AT& ar, AT& ai) {
  // a group's slots past the width repeat the group's first slot (loaded, not
  // summed), so every load of the group is issued before the sums
  for (int s0 = 0; s0 < A.w; s0 += SG) {
    int c[SG];
    cx<T> a[SG];
    cx<X> t[SG];
#pragma unroll
    for (int q = 0; q < SG; ++q) {
      const size_t o = (size_t)(s0 + q < A.w ? s0 + q : s0) * A.n + i;
      c[q] = A.col[o];
      a[q] = A.val[o];
    }
#pragma unroll
    for (int q = 0; q < SG; ++q) t[q] = x[(size_t)c[q] * B + b];
#pragma unroll
    for (int q = 0; q < SG; ++q) {
      if (s0 + q < A.w) {
        const AT tr = (AT)t[q].x, ti = (AT)t[q].y;
        ar += (AT)a[q].x * tr - (AT)a[q].y * ti;
        ai += (AT)a[q].x * ti + (AT)a[q].y * tr;
      }
    }
  }
}

// Hardware block ids go round-robin over the 8 XCDs; remap them so that XCD x
// walks one contiguous range of rows and neighbour rows meet in its L2.
__device__ __forceinline__ int hz_block() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

#define HZ_ROW(N)                                                      \
  const long gt_ = (long)hz_block() * blockDim.x + threadIdx.x;       \
  const int i = (int)(gt_ >> lb);                                      \
  const int b = (int)(gt_ & ((1 << lb) - 1));                          \
  if (i >= (N) || b >= B) return;                                      \
  const size_t o = (size_t)i * B + b;

// ------------------------------------------------------------------ per-level sweeps
// out = f - A u (u null: u = 0); JAC: out = theta D^{-1} (f - A u)
template <class T, bool JAC>
__global__ __launch_bounds__(256) void k_hz_resid(CEll<T> A, int B, int lb, const cx<T>* __restrict__ f,
                                                  const cx<T>* __restrict__ u, const cx<T>* __restrict__ dinv,
                                                  T theta, cx<T>* __restrict__ out) {
  HZ_ROW(A.n)
  const cx<T> fi = f[o];
  T ar = 0, ai = 0;
  if (u) ell_cmul<T, T, T>(A, u, i, B, b, ar, ai);
  T rr = fi.x - ar, ri = fi.y - ai;
  if (JAC) {
    const cx<T> d = dinv[i];
    const T tr = d.x * rr - d.y * ri, ti = d.x * ri + d.y * rr;
    rr = theta * tr;
    ri = theta * ti;
  }
  out[o] = mkc<T>(rr, ri);
}

// one Horner hop of a two-feature convolution: v = [M y] + W x, or with MIXN
// v = Wn (M y) + W x (y = x: the first two Horner steps in one sweep, since
// the feature mixing commutes with the neighbour mean); ADD: out += s v,
// else out = s v
template <class T, bool NB, bool ADD, bool MIXN = false>
__global__ __launch_bounds__(256) void k_hz_hop(GEll G, const T* __restrict__ invdeg, int B, int lb,
                                                const cx<T>* __restrict__ y, const cx<T>* __restrict__ x, W2<T> W,
                                                T s, cx<T>* __restrict__ out, W2<T> Wn = W2<T>{}) {
  HZ_ROW(G.n)
  cx<T> v = mixw(W, x[o]);
  if (NB) {
    T mr = 0, mi = 0;
    // slots in groups, every load of a group issued before its sums
    for (int q0 = 0; q0 < G.w; q0 += kSlots) {
      int j[kSlots];
      cx<T> t[kSlots];
#pragma unroll
      for (int q = 0; q < kSlots; ++q) j[q] = G.col[(size_t)(q0 + q < G.w ? q0 + q : q0) * G.n + i];
#pragma unroll
      for (int q = 0; q < kSlots; ++q) t[q] = y[(size_t)j[q] * B + b];
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        if (q0 + q < G.w && j[q] != i) {
          mr += t[q].x;
          mi += t[q].y;
        }
      }
    }
    const T r = invdeg[i];
    cx<T> m = mkc<T>(r * mr, r * mi);
    if (MIXN) m = mixw(Wn, m);
    v.x += m.x;
    v.y += m.y;
  }
  if (ADD) {
    cx<T> u = out[o];
    u.x += s * v.x;
    u.y += s * v.y;
    out[o] = u;
  } else {
    out[o] = mkc<T>(s * v.x, s * v.y);
  }
}

// transfer with feature mixing: v = W (X in)_i; ADD: out += v, else out = v
template <class T, bool ADD>
__global__ __launch_bounds__(256) void k_hz_xfer(REll<T> X, int B, int lb, const cx<T>* __restrict__ in, W2<T> W,
                                                 cx<T>* __restrict__ out) {
  HZ_ROW(X.n)
  T ar = 0, ai = 0;
  for (int s = 0; s < X.w; ++s) {
    const int j = X.col[(size_t)s * X.n + i];
    const T a = X.val[(size_t)s * X.n + i];
    const cx<T> t = in[(size_t)j * B + b];
    ar += a * t.x;
    ai += a * t.y;
  }
  const cx<T> v = mixw(W, mkc<T>(ar, ai));
  if (ADD) {
    cx<T> u = out[o];
    u.x += v.x;
    u.y += v.y;
    out[o] = u;
  } else {
    out[o] = v;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_hz_zero(size_t cnt, cx<T>* __restrict__ p) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t < cnt) p[t] = mkc<T>(0, 0);
}

template <class T>
__global__ __launch_bounds__(256) void k_hz_copy(size_t cnt, const cx<T>* __restrict__ a, cx<T>* __restrict__ p) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t < cnt) p[t] = a[t];
}

// ------------------------------------------------------------------ GMRES smoothing step
// Sum over the 64 lanes of a wavefront, left in every lane: a butterfly of
// lane exchanges (each step adds the value of the lane whose index differs in
// one bit; the same pairing order in every lane, so the sum is deterministic).
__device__ __forceinline__ double hz_wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Block-wide sums of the first cnt of N doubles (and of the last one when
// last is set), broadcast to every work-item: wavefront sums (hz_wave_sum),
// then work-item k adds the waves' totals of value k in wave order (a fixed
// order: deterministic).  lds: N x 16 doubles, tot: N.
template <int N>
__device__ __forceinline__ void hz_block_sum(double (&a)[N], int cnt, double* lds, double* tot, bool last = false) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k < cnt || (last && k == N - 1)) {
      const double x = hz_wave_sum(a[k]);
      if (ln == 0) lds[k * 16 + wv] = x;
    }
  }
  __syncthreads();
  const int k0 = (int)threadIdx.x < cnt ? (int)threadIdx.x : (last && (int)threadIdx.x == cnt ? N - 1 : -1);
  if (k0 >= 0) {
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += lds[k0 * 16 + q];
    tot[k0] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k)
    if (k < cnt || (last && k == N - 1)) a[k] = tot[k];
}

__device__ __forceinline__ double2 zc(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) { return zc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 zconj(double2 a) { return zc(a.x, -a.y); }
__device__ __forceinline__ double zabs(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return zc((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Complex Givens least squares min || beta e_1 - H y || for the (m+1) x m
// upper Hessenberg H (row stride ldh), rotations [c s; -conj(s) c] with real
// c; y[0..m) by back substitution (a zero pivot gives a zero component).
// g, cs, sn: work arrays of kMaxV + 1, kMaxV, kMaxV entries.
__device__ void hz_givens_lsq(double2* H, int ldh, int m, double beta, double2* y, double2* g, double* cs,
                              double2* sn) {
  for (int k = 0; k <= kMaxV; ++k) g[k] = zc(0.0, 0.0);
  g[0] = zc(beta, 0.0);
  for (int j = 0; j < m; ++j) {
    for (int k = 0; k < j; ++k) {
      const double2 a = H[k * ldh + j], bb = H[(k + 1) * ldh + j];
      const double2 t = zc(cs[k] * a.x + zmul(sn[k], bb).x, cs[k] * a.y + zmul(sn[k], bb).y);
      const double2 u = zmul(zconj(sn[k]), a);
      H[(k + 1) * ldh + j] = zc(cs[k] * bb.x - u.x, cs[k] * bb.y - u.y);
      H[k * ldh + j] = t;
    }
    const double2 a = H[j * ldh + j], bb = H[(j + 1) * ldh + j];
    const double na = zabs(a), d = hypot(na, zabs(bb));
    if (d == 0.0) {
      cs[j] = 1.0;
      sn[j] = zc(0.0, 0.0);
    } else if (na == 0.0) {
      cs[j] = 0.0;
      sn[j] = zc(1.0, 0.0);
    } else {
      cs[j] = na / d;
      const double2 ph = zc(a.x / na, a.y / na);
      const double2 t = zmul(ph, zconj(bb));
      sn[j] = zc(t.x / d, t.y / d);
    }
    const double2 sb = zmul(sn[j], bb);
    H[j * ldh + j] = zc(cs[j] * a.x + sb.x, cs[j] * a.y + sb.y);
    H[(j + 1) * ldh + j] = zc(0.0, 0.0);
    const double2 gj = g[j];
    const double2 ng = zmul(zconj(sn[j]), gj);
    g[j + 1] = zc(-ng.x, -ng.y);
    g[j] = zc(cs[j] * gj.x, cs[j] * gj.y);
  }
  for (int j = m - 1; j >= 0; --j) {
    double2 s = g[j];
    for (int k = j + 1; k < m; ++k) {
      const double2 t = zmul(H[j * ldh + k], y[k]);
      s = zc(s.x - t.x, s.y - t.y);
    }
    const double2 p = H[j * ldh + j];
    y[j] = (p.x == 0.0 && p.y == 0.0) ? zc(0.0, 0.0) : zdiv(s, p);
  }
}

// Sweeps of an Arnoldi step over the rows of this work-item (rows threadIdx.x
// + k blockDim.x of one column; the column's vectors are contiguous).  The
// restrict-qualified parameters let the compiler issue the loads of the next
// row before the store of the current one.
// sweep 1: w = s (A x), stored to wn; acc_t += conj(V_t) w for t <= j and
// acc[kNorm] += |w|^2 (slots loaded in groups of SG, as in ell_cmul)
template <class T, int SG>
__device__ __forceinline__ void gm_sweep1(int n, int w_, const int* __restrict__ col, const cx<T>* __restrict__ val,
                                          const cx<T>* __restrict__ x, T s, const cx<T>* __restrict__ V, size_t NB,
                                          int j, cx<T>* __restrict__ wn, double (&acc)[kAcc]) {
#pragma unroll 2
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T ar = 0, ai = 0;
    for (int s0 = 0; s0 < w_; s0 += SG) {
      // slots past the width repeat the group's first (loaded, not summed)
      int c[SG];
      cx<T> a[SG], t[SG];
#pragma unroll
      for (int q = 0; q < SG; ++q) {
        const size_t o = (size_t)(s0 + q < w_ ? s0 + q : s0) * n + i;
        c[q] = col[o];
        a[q] = val[o];
      }
#pragma unroll
      for (int q = 0; q < SG; ++q) t[q] = x[c[q]];
#pragma unroll
      for (int q = 0; q < SG; ++q) {
        if (s0 + q < w_) {
          ar += a[q].x * t[q].x - a[q].y * t[q].y;
          ai += a[q].x * t[q].y + a[q].y * t[q].x;
        }
      }
    }
    const cx<T> w = mkc<T>(ar * s, ai * s);
    wn[i] = w;
    acc[kNorm] += (double)w.x * w.x + (double)w.y * w.y;
#pragma unroll
    for (int t = 0; t <= kMaxV; ++t) {
      if (t <= j) {
        const cx<T> q = V[(size_t)t * NB + i];     // conj(q) w
        acc[2 * t] += (double)q.x * w.x + (double)q.y * w.y;
        acc[2 * t + 1] += (double)q.x * w.y - (double)q.y * w.x;
      }
    }
  }
}

// update sweep: w -= sum_{t <= j} cf_t V_t in place; DOTS: acc_t += conj(V_t) w
// and acc[kNorm] += |w|^2, else acc_0 += |w|^2
template <class T, bool DOTS>
__device__ __forceinline__ void gm_sweep_upd(int n, const cx<T>* __restrict__ V, size_t NB, int j,
                                             const double (&cf)[2 * (kMaxV + 1)], cx<T>* __restrict__ wn,
                                             double (&acc)[kAcc]) {
#pragma unroll 2
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    cx<T> w = wn[i];
#pragma unroll
    for (int t = 0; t <= kMaxV; ++t) {
      if (t <= j) {
        const cx<T> q = V[(size_t)t * NB + i];
        const T hr = (T)cf[2 * t], hi = (T)cf[2 * t + 1];
        w.x -= hr * q.x - hi * q.y;
        w.y -= hr * q.y + hi * q.x;
      }
    }
    wn[i] = w;
    if (DOTS) {
#pragma unroll
      for (int t = 0; t <= kMaxV; ++t) {
        if (t <= j) {
          const cx<T> q = V[(size_t)t * NB + i];
          acc[2 * t] += (double)q.x * w.x + (double)q.y * w.y;
          acc[2 * t + 1] += (double)q.x * w.y - (double)q.y * w.x;
        }
      }
      acc[kNorm] += (double)w.x * w.x + (double)w.y * w.y;
    } else {
      acc[0] += (double)w.x * w.x + (double)w.y * w.y;
    }
  }
}

// One GMRES smoothing step on column blockIdx.x of level (A, G):
//   r = f - A u;  d0 = theta Phi_B(r);  u += eta GMRES(A, r, d0, v)
// The step needs hz_slots(v) vectors of the column: r, d0, V_0 .. V_v (the
// Horner buffers reuse V_1, V_2).  MODE 1: all of them live in the
// work-group's LDS (dynamic shared memory of hz_slots(v) n values); MODE 2:
// the basis vectors V_0 .. V_{v-1}, which every sweep reads, live in LDS (v n
// values, v >= 3) and r, d0 and V_v in scr; MODE 0: all in scr.  scr holds
// n x B values per slot stored column by column (column b of slot t at
// scr + t n B + b n) so the sweeps over a column are coalesced.  f and u keep
// the [n][B] layout.  Orthogonalisation: classical
// Gram-Schmidt applied twice per Arnoldi step; dot products and norms are
// accumulated in FP64.
template <class T, int MODE>
__global__ __launch_bounds__(MODE == 1 ? kGT : kGTH) void k_hz_gmres(CEll<T> A, GEll G, const T* __restrict__ invdeg, int B,
                                                  const cx<T>* __restrict__ f, cx<T>* __restrict__ u, T theta,
                                                  T eta, WK<T> W, int K, int v, cx<T>* __restrict__ scr) {
  __shared__ double red[kAcc * 16], tot[kAcc];
  __shared__ double2 H[(kMaxV + 1) * kMaxV];
  __shared__ double2 yls[kMaxV], gw[kMaxV + 1], snw[kMaxV];
  __shared__ double csw[kMaxV];
  extern __shared__ __align__(16) unsigned char hz_dyn[];
  const int b = blockIdx.x, n = A.n, nt = blockDim.x, t0 = threadIdx.x;
  // slot group of the SpMVs: the HBM-scratch form runs 1024 work-items with
  // half the registers per work-item
  constexpr int SG = MODE == 1 ? kSlots : kSlots / 2;
  cx<T>* lds = reinterpret_cast<cx<T>*>(hz_dyn);
  cx<T>* gcol = scr + (size_t)b * n;           // this column's slot 0 in the global scratch
  const size_t GS = (size_t)n * B;             // global slot stride
  cx<T>* R = MODE == 1 ? lds : gcol;
  cx<T>* D0 = MODE == 1 ? lds + n : gcol + GS;
  // V_t = V + t NB for t < v; the Horner buffers are V_1 and V_2
  const size_t NB = MODE == 0 ? GS : (size_t)n;
  cx<T>* V = MODE == 0 ? gcol + 2 * GS : (MODE == 1 ? lds + 2 * (size_t)n : lds);
  cx<T>* Vlast = MODE == 2 ? gcol + 2 * GS : V + (size_t)v * NB;     // V_v
  // 1. residual
  for (int i = t0; i < n; i += nt) {
    T ar = 0, ai = 0;
    ell_cmul<T, T, T, SG>(A, u, i, B, b, ar, ai);
    const cx<T> fi = f[(size_t)i * B + b];
    R[i] = mkc<T>(fi.x - ar, fi.y - ai);
  }
  __syncthreads();
  // 2. initial guess d0 = theta Phi_B(r) (Horner over the neighbour mean)
  if (K == 0) {
    for (int i = t0; i < n; i += nt) {
      const cx<T> t = mixw(W.w[0], R[i]);
      D0[i] = mkc<T>(theta * t.x, theta * t.y);
    }
  } else {
    // the Horner buffers take basis slots 1 and 2, unused until the Arnoldi
    // steps; hop k forms M y + W_k r, and the first one W_{K-1} r + W_K (M r)
    // (the feature mixing commutes with the neighbour mean)
    int cur = 0;
    for (int k = K - 1; k >= 0; --k) {
      cx<T>* dst = k == 0 ? D0 : V + (size_t)(2 - cur) * NB;     // the other Horner buffer
      const T s = k == 0 ? theta : (T)1;
      const cx<T>* yc = k == K - 1 ? R : V + (size_t)(1 + cur) * NB;
      for (int i = t0; i < n; i += nt) {
        T mr = 0, mi = 0;
        for (int q0 = 0; q0 < G.w; q0 += kSlots) {   // every load of a group before its sums
          int jj[kSlots];
          cx<T> tv[kSlots];
#pragma unroll
          for (int q = 0; q < kSlots; ++q) jj[q] = G.col[(size_t)(q0 + q < G.w ? q0 + q : q0) * n + i];
#pragma unroll
          for (int q = 0; q < kSlots; ++q) tv[q] = yc[jj[q]];
#pragma unroll
          for (int q = 0; q < kSlots; ++q) {
            if (q0 + q < G.w && jj[q] != i) {
              mr += tv[q].x;
              mi += tv[q].y;
            }
          }
        }
        cx<T> t = mixw(W.w[k], R[i]);
        const T r = invdeg[i];
        cx<T> m = mkc<T>(r * mr, r * mi);
        if (k == K - 1) m = mixw(W.w[K], m);
        t.x += m.x;
        t.y += m.y;
        dst[i] = mkc<T>(s * t.x, s * t.y);
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  __syncthreads();
  // 3. r0 = r - A d0 and beta = ||r0||
  double acc[kAcc];
  acc[0] = 0.0;
  for (int i = t0; i < n; i += nt) {
    T ar = 0, ai = 0;
    ell_cmul<T, T, T, SG>(A, D0, i, 1, 0, ar, ai);
    const cx<T> ri = R[i];
    const cx<T> t = mkc<T>(ri.x - ar, ri.y - ai);
    V[i] = t;
    acc[0] += (double)t.x * t.x + (double)t.y * t.y;
  }
  hz_block_sum(acc, 1, red, tot);
  const double beta = sqrt(acc[0]);
  // Arnoldi with a lazily normalised basis: slot t holds Vt_t and the actual
  // basis vector is v_t = sc[t] Vt_t.  Each step is three sweeps, each ending
  // in one block reduction: w = A v_j with the first-pass dots, the first
  // update with the second-pass dots, the second update with the norm.
  double sc[kMaxV + 1], cf[2 * (kMaxV + 1)];
#pragma unroll
  for (int t = 0; t <= kMaxV; ++t) sc[t] = 0.0;
  int m = 0;
  if (beta > 0.0) {
    sc[0] = 1.0 / beta;
    if (t0 == 0)
      for (int k = 0; k < (kMaxV + 1) * kMaxV; ++k) H[k] = zc(0.0, 0.0);
    m = v;
    for (int j = 0; j < v; ++j) {
      double sj = 0.0;
#pragma unroll
      for (int t = 0; t <= kMaxV; ++t)
        if (t == j) sj = sc[t];
      const T sjt = (T)sj;
      const cx<T>* Vj = V + (size_t)j * NB;
      cx<T>* Wn = j + 1 < v ? V + (size_t)(j + 1) * NB : Vlast;
      // sweep 1: w = A v_j, <Vt_t, w> and |w|^2
#pragma unroll
      for (int t = 0; t <= kMaxV; ++t)
        if (t <= j) acc[2 * t] = acc[2 * t + 1] = 0.0;
      acc[kNorm] = 0.0;
      gm_sweep1<T, SG>(n, A.w, A.col, A.val, Vj, sjt, V, NB, j, Wn, acc);
      hz_block_sum(acc, 2 * (j + 1), red, tot, true);
      const double w2 = acc[kNorm];
      // h_t = sc[t] acc_t; an update subtracts h_t v_t = (h_t sc[t]) Vt_t.  The
      // first update also forms the second pass's dot products and the new
      // norm; the second update runs only when the first cancelled more than
      // 1 - 1/sqrt 2 of the norm (Kahan-Parlett), uniformly over the block.
      double hn2 = 0.0;
      for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int t = 0; t <= kMaxV; ++t) {
          if (t <= j) {
            cf[2 * t] = acc[2 * t] * sc[t] * sc[t];
            cf[2 * t + 1] = acc[2 * t + 1] * sc[t] * sc[t];
          }
        }
        if (t0 == 0)
#pragma unroll
          for (int t = 0; t <= kMaxV; ++t) {
            if (t <= j) {
              const double2 h = H[t * kMaxV + j];
              H[t * kMaxV + j] = zc(h.x + acc[2 * t] * sc[t], h.y + acc[2 * t + 1] * sc[t]);
            }
          }
#pragma unroll
        for (int t = 0; t <= kMaxV; ++t)
          if (t <= j) acc[2 * t] = acc[2 * t + 1] = 0.0;
        acc[kNorm] = 0.0;
        if (pass == 0) {
          gm_sweep_upd<T, true>(n, V, NB, j, cf, Wn, acc);
          hz_block_sum(acc, 2 * (j + 1), red, tot, true);
          hn2 = acc[kNorm];
          if (!(hn2 < 0.5 * w2)) break;
        } else {
          gm_sweep_upd<T, false>(n, V, NB, j, cf, Wn, acc);
          hz_block_sum(acc, 1, red, tot);
          hn2 = acc[0];
        }
      }
      const double hn = sqrt(hn2);
      if (t0 == 0) H[(j + 1) * kMaxV + j] = zc(hn, 0.0);
      if (hn == 0.0) {
        m = j + 1;
        break;
      }
#pragma unroll
      for (int t = 0; t <= kMaxV; ++t)
        if (t == j + 1) sc[t] = 1.0 / hn;
    }
    __syncthreads();
    if (t0 == 0) hz_givens_lsq(H, kMaxV, m, beta, yls, gw, csw, snw);
    __syncthreads();
    // fold the lazy scales into the coefficients: v_t y_t = Vt_t (sc[t] y_t)
    if (t0 == 0)
#pragma unroll
      for (int t = 0; t < kMaxV; ++t)
        if (t < m) yls[t] = zc(yls[t].x * sc[t], yls[t].y * sc[t]);
    __syncthreads();
  }
  // 4. u += eta (d0 + V y)
  for (int i = t0; i < n; i += nt) {
    const cx<T> d = D0[i];
    double dr = d.x, di = d.y;
    for (int t = 0; t < m; ++t) {
      const double2 y = yls[t];
      const cx<T> q = V[(size_t)t * NB + i];
      dr += y.x * q.x - y.y * q.y;
      di += y.x * q.y + y.y * q.x;
    }
    cx<T> ui = u[(size_t)i * B + b];
    ui.x += eta * (T)dr;
    ui.y += eta * (T)di;
    u[(size_t)i * B + b] = ui;
  }
}

// ------------------------------------------------------------------ FP64 Krylov sweeps (outer FGMRES)
// Rows are split into nblk chunks; 2^lb >= B lanes per row, 256 >> lb rows per pass.
#define HZ_KR                                                          \
  const int rpb = 256 >> lb;                                           \
  const int b = threadIdx.x & ((1 << lb) - 1);                         \
  const int rg = (int)(threadIdx.x >> lb);                             \
  const int blk = blockIdx.x;                                          \
  const long lo = (long)blk * chunk;                                   \
  const long hi = lo + chunk < n ? lo + chunk : (long)n;               \
  const bool lane_ok = b < B;

// per-block sum over the row groups of one value per lane (fixed tree)
__device__ __forceinline__ double kr_rowsum(double v, int lb, double* red) {
  const int rpb = 256 >> lb, LB = 1 << lb;
  const int rg = (int)(threadIdx.x >> lb);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = rpb >> 1; h > 0; h >>= 1) {
    if (rg < h) red[threadIdx.x] += red[threadIdx.x + h * LB];
    __syncthreads();
  }
  const double r = red[threadIdx.x & (LB - 1)];
  __syncthreads();
  return r;
}

// coarsest level: u = A^{-1} f with the FP64 inverse; one work-group per row
// i, the 256 >> lb lane groups splitting the sum over j (fixed tree)
template <class T>
__global__ __launch_bounds__(256) void k_hz_dense(int n, int B, int lb, const double2* __restrict__ Ainv,
                                                  const cx<T>* __restrict__ f, cx<T>* __restrict__ u) {
  __shared__ double red[256];
  const int i = blockIdx.x, ng = 256 >> lb;
  const int b = threadIdx.x & ((1 << lb) - 1), jg = (int)(threadIdx.x >> lb);
  double ar = 0.0, ai = 0.0;
  if (b < B) {
    for (int j = jg; j < n; j += ng) {
      const double2 a = Ainv[(size_t)i * n + j];
      const cx<T> t = f[(size_t)j * B + b];
      const double tr = (double)t.x, ti = (double)t.y;
      ar += a.x * tr - a.y * ti;
      ai += a.x * ti + a.y * tr;
    }
  }
  ar = kr_rowsum(ar, lb, red);
  ai = kr_rowsum(ai, lb, red);
  if (jg == 0 && b < B) u[(size_t)i * B + b] = mkc<T>((T)ar, (T)ai);
}

// w = f - A x (x null: w = f), FP64
__global__ __launch_bounds__(256) void k_fx_resid(CEll<double> A, int B, int lb, const double2* __restrict__ f,
                                                  const double2* __restrict__ x, double2* __restrict__ w) {
  HZ_ROW(A.n)
  double ar = 0.0, ai = 0.0;
  if (x) ell_cmul<double, double, double>(A, x, i, B, b, ar, ai);
  const double2 fi = f[o];
  w[o] = zc(fi.x - ar, fi.y - ai);
}

// w = A z (z in the cycle type), FP64
template <class T>
__global__ __launch_bounds__(256) void k_fx_amul(CEll<double> A, int B, int lb, const cx<T>* __restrict__ z,
                                                 double2* __restrict__ w) {
  HZ_ROW(A.n)
  double ar = 0.0, ai = 0.0;
  ell_cmul<double, double, T>(A, z, i, B, b, ar, ai);
  w[o] = zc(ar, ai);
}

// Dot sweep: for the kNG basis vectors t = blockIdx.y * kNG + q < nv,
// part[(blk * (nv + 1) + t) * B + b] = sum over the block's rows of conj(v_t) w,
// and (blockIdx.y == 0) part[(blk * (nv + 1) + nv) * B + b].x = sum |w|^2.
// Basis: v_t(i, b) at V[(i * mp1 + t) * B + b]; w(i, b) at w[i * wrs + b].
// skip: when non-null and *skip == 0 the sweep does nothing.
__global__ __launch_bounds__(256) void k_fx_dot(int n, int B, int lb, int chunk, const double2* __restrict__ V,
                                                int mp1, int nv, const double2* w, long wrs,
                                                double2* __restrict__ part, const int* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip == 0) return;
  HZ_KR
  const int tb = blockIdx.y * kNG;
  double ar[kNG], ai[kNG], ww = 0.0;
#pragma unroll
  for (int q = 0; q < kNG; ++q) ar[q] = ai[q] = 0.0;
  if (lane_ok) {
    for (long i = lo + rg; i < hi; i += rpb) {
      const double2 wv = w[(size_t)i * wrs + b];
      ww += wv.x * wv.x + wv.y * wv.y;
#pragma unroll
      for (int q = 0; q < kNG; ++q) {
        if (tb + q < nv) {
          const double2 v = V[((size_t)i * mp1 + tb + q) * B + b];
          ar[q] += v.x * wv.x + v.y * wv.y;
          ai[q] += v.x * wv.y - v.y * wv.x;
        }
      }
    }
  }
  const bool st = rg == 0 && lane_ok;
  for (int q = 0; q < kNG; ++q) {
    if (tb + q >= nv) break;                     // uniform over the block
    const double sr = kr_rowsum(ar[q], lb, red);
    const double si = kr_rowsum(ai[q], lb, red);
    if (st) part[((size_t)blk * (nv + 1) + tb + q) * B + b] = zc(sr, si);
  }
  if (blockIdx.y == 0) {
    const double s = kr_rowsum(ww, lb, red);
    if (st) part[((size_t)blk * (nv + 1) + nv) * B + b] = zc(s, 0.0);
  }
}

// out[t * B + b] = sum over blocks of part[(blk * rows + t) * B + b]: one
// wavefront per output, lane q summing blocks q, q + 64, ... in order, then a
// butterfly over the lanes (a fixed order: deterministic)
__global__ __launch_bounds__(256) void k_fx_reduce(int nblk, int rows, int B, const double2* __restrict__ part,
                                                   double2* __restrict__ out, const int* __restrict__ skip) {
  if (skip && *skip == 0) return;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
  if (t >= rows * B) return;                   // uniform over the wavefront
  double sr = 0.0, si = 0.0;
  for (int k = ln; k < nblk; k += 64) {
    const double2 p = part[(size_t)k * rows * B + t];
    sr += p.x;
    si += p.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off);
    si += __shfl_xor(si, off);
  }
  if (ln == 0) out[t] = zc(sr, si);
}

// wo = wi - sum_{t < nv} h_t v_t and part[blk * B + b].x = sum |wo|^2 (wi may equal wo)
__global__ __launch_bounds__(256) void k_fx_upd(int n, int B, int lb, int chunk, const double2* __restrict__ V,
                                                int mp1, int nv, const double2* __restrict__ h, const double2* wi,
                                                long wis, double2* wo, long wos, double2* __restrict__ part,
                                                const int* __restrict__ skip) {
  __shared__ double red[256];
  if (skip && *skip == 0) return;
  HZ_KR
  double ww = 0.0;
  if (lane_ok) {
    for (long i = lo + rg; i < hi; i += rpb) {
      double2 w = wi[(size_t)i * wis + b];
      for (int t = 0; t < nv; ++t) {
        const double2 c = h[(size_t)t * B + b];
        const double2 v = V[((size_t)i * mp1 + t) * B + b];
        w.x -= c.x * v.x - c.y * v.y;
        w.y -= c.x * v.y + c.y * v.x;
      }
      wo[(size_t)i * wos + b] = w;
      ww += w.x * w.x + w.y * w.y;
    }
  }
  const double s = kr_rowsum(ww, lb, red);
  if (rg == 0 && lane_ok) part[(size_t)blk * B + b] = zc(s, 0.0);
}

// Per-column FGMRES state (device).
struct FxState {
  double2* H;      // [(m + 1) * m][B]: entry (r, c) at (r * m + c) * B + b
  double* cs;      // [m][B]
  double2* sn;     // [m][B]
  double2* g;      // [(m + 1)][B]
  double2* y;      // [m][B]
  double* sig;     // [B] scale of the newest basis vector
  double* fnorm;   // [B]
  double* beta;    // [B] norm of the last true residual
  int* act;        // [B] iterating in this restart cycle
  int* jd;         // [B] iterations done in this restart cycle
  int* iters;      // [B] total iterations
  int* status;     // [B] -1 running, else an mg_status
  int* cnt;        // [1] active columns
  int* flag;       // [1] second Gram-Schmidt pass needed
};

__device__ __forceinline__ void fx_count(const FxState& S, int B) {
  __shared__ int c[256];
  c[threadIdx.x] = (threadIdx.x < (unsigned)B && S.act[threadIdx.x]) ? 1 : 0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) c[threadIdx.x] += c[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *S.cnt = c[0];
}

// first call (init): fnorm = ||f||, status running, iters 0.  Then per
// restart: beta = ||r||; a column iterates when running, beta > rtol fnorm and
// iterations remain; g = beta e_1, sig = 1 / beta.
__global__ __launch_bounds__(256) void k_fx_start(FxState S, int B, int m, const double2* __restrict__ nrm2,
                                                  double rtol, int max_iter, int init) {
  const int b = threadIdx.x;
  if (b < B) {
    const double nr = sqrt(nrm2[b].x);
    if (init) {
      S.fnorm[b] = nr;
      S.status[b] = -1;
      S.iters[b] = 0;
      S.beta[b] = nr;
      S.act[b] = 0;
    } else {
      S.beta[b] = nr;
      int a = 0;
      if (S.status[b] == -1) {
        if (!isfinite(nr)) S.status[b] = MG_ERR_DIVERGED;
        else if (nr <= rtol * S.fnorm[b]) S.status[b] = MG_OK;
        else if (S.iters[b] >= max_iter) S.status[b] = MG_ERR_NOT_CONVERGED;
        else a = 1;
      }
      S.act[b] = a;
      S.jd[b] = 0;
      for (int k = 0; k <= m; ++k) S.g[(size_t)k * B + b] = zc(k == 0 ? nr : 0.0, 0.0);
      S.sig[b] = a ? 1.0 / nr : 0.0;
    }
  }
  __syncthreads();
  fx_count(S, B);
}

// flag = some active column lost more than 1 - thr of its norm in the first pass
__global__ __launch_bounds__(256) void k_fx_flag(FxState S, int B, const double2* __restrict__ w2,
                                                 const double2* __restrict__ n2, double thr2) {
  __shared__ int c[256];
  const int b = threadIdx.x;
  c[b] = (b < B && S.act[b] && n2[b].x < thr2 * w2[b].x) ? 1 : 0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (b < h) c[b] |= c[b + h];
    __syncthreads();
  }
  if (b == 0) *S.flag = c[0];
}

// Hessenberg column j of every active column: h1 (+ h2 after a second pass),
// subdiagonal from the final squared norm; earlier rotations, a new complex
// Givens rotation, the residual estimate and the stopping tests.
__global__ __launch_bounds__(256) void k_fx_givens(FxState S, int B, int m, int j, const double2* __restrict__ h1,
                                                   const double2* __restrict__ h2, const double2* __restrict__ n2,
                                                   const double2* __restrict__ n4, double rtol, int max_iter) {
  const int b = threadIdx.x;
  const bool two = *S.flag != 0;
  if (b < B && S.act[b]) {
    auto Hat = [&](int r, int c) -> double2& { return S.H[((size_t)r * m + c) * B + b]; };
    for (int t = 0; t <= j; ++t) {
      double2 h = h1[(size_t)t * B + b];
      if (two) {
        const double2 e = h2[(size_t)t * B + b];
        h = zc(h.x + e.x, h.y + e.y);
      }
      Hat(t, j) = h;
    }
    const double hn = sqrt(two ? n4[b].x : n2[b].x);
    Hat(j + 1, j) = zc(hn, 0.0);
    for (int k = 0; k < j; ++k) {
      const double c = S.cs[(size_t)k * B + b];
      const double2 s = S.sn[(size_t)k * B + b];
      const double2 a = Hat(k, j), bb = Hat(k + 1, j);
      const double2 sb = zmul(s, bb), ca = zmul(zconj(s), a);
      Hat(k, j) = zc(c * a.x + sb.x, c * a.y + sb.y);
      Hat(k + 1, j) = zc(c * bb.x - ca.x, c * bb.y - ca.y);
    }
    const double2 a = Hat(j, j), bb = Hat(j + 1, j);
    const double na = zabs(a), d = hypot(na, zabs(bb));
    double c;
    double2 s;
    if (d == 0.0) {
      c = 1.0;
      s = zc(0.0, 0.0);
    } else if (na == 0.0) {
      c = 0.0;
      s = zc(1.0, 0.0);
    } else {
      c = na / d;
      const double2 t = zmul(zc(a.x / na, a.y / na), zconj(bb));
      s = zc(t.x / d, t.y / d);
    }
    S.cs[(size_t)j * B + b] = c;
    S.sn[(size_t)j * B + b] = s;
    const double2 sb = zmul(s, bb);
    Hat(j, j) = zc(c * a.x + sb.x, c * a.y + sb.y);
    Hat(j + 1, j) = zc(0.0, 0.0);
    const double2 gj = S.g[(size_t)j * B + b];
    const double2 ng = zmul(zconj(s), gj);
    S.g[(size_t)(j + 1) * B + b] = zc(-ng.x, -ng.y);
    S.g[(size_t)j * B + b] = zc(c * gj.x, c * gj.y);
    S.iters[b] += 1;
    S.jd[b] = j + 1;
    const double est = zabs(S.g[(size_t)(j + 1) * B + b]);
    const bool stop = !(est > rtol * S.fnorm[b]) || S.iters[b] >= max_iter || hn == 0.0 || !isfinite(hn) ||
                      j + 1 >= m;
    S.sig[b] = (stop || !(hn > 0.0)) ? 0.0 : 1.0 / hn;
    if (stop) S.act[b] = 0;
  }
  __syncthreads();
  fx_count(S, B);
}

// v = sig w (w plain [n][B] or a basis slot), written to basis slot t and as
// the cycle-type preconditioner input
template <class T>
__global__ __launch_bounds__(256) void k_fx_scale(int n, int B, int lb, const double* __restrict__ sig,
                                                  const double2* w, long wrs, double2* vo, long vrs,
                                                  cx<T>* __restrict__ zin) {
  HZ_ROW(n)
  const double s = sig[b];
  const double2 x = w[(size_t)i * wrs + b];
  const double2 r = zc(s * x.x, s * x.y);
  vo[(size_t)i * vrs + b] = r;
  zin[o] = mkc<T>((T)r.x, (T)r.y);
  (void)o;
}

// y = R^{-1} g over the first jd[b] rotated rows (upper triangular)
__global__ __launch_bounds__(256) void k_fx_lsq(FxState S, int B, int m) {
  const int b = threadIdx.x;
  if (b >= B) return;
  const int k = S.jd[b];
  for (int j = k - 1; j >= 0; --j) {
    double2 s = S.g[(size_t)j * B + b];
    for (int c = j + 1; c < k; ++c) {
      const double2 t = zmul(S.H[((size_t)j * m + c) * B + b], S.y[(size_t)c * B + b]);
      s = zc(s.x - t.x, s.y - t.y);
    }
    const double2 p = S.H[((size_t)j * m + j) * B + b];
    S.y[(size_t)j * B + b] = (p.x == 0.0 && p.y == 0.0) ? zc(0.0, 0.0) : zdiv(s, p);
  }
}

// x += sum_{t < jd[b]} y_t z_t
template <class T>
__global__ __launch_bounds__(256) void k_fx_xupd(int n, int B, int lb, const int* __restrict__ jd,
                                                 const double2* __restrict__ y, const cx<T>* __restrict__ Z,
                                                 size_t zs, double2* __restrict__ x) {
  HZ_ROW(n)
  const int k = jd[b];
  double2 xv = x[o];
  for (int t = 0; t < k; ++t) {
    const double2 c = y[(size_t)t * B + b];
    const cx<T> z = Z[(size_t)t * zs + o];
    xv.x += c.x * z.x - c.y * z.y;
    xv.y += c.x * z.y + c.y * z.x;
  }
  x[o] = xv;
}

__global__ __launch_bounds__(256) void k_fx_sqrt(int B, const double2* __restrict__ in, double* __restrict__ out) {
  const int b = threadIdx.x;
  if (b < B) out[b] = sqrt(in[b].x);
}

// stationary solve: u[:, b] = w[:, b] for the columns still iterating
__global__ __launch_bounds__(256) void k_hz_take(int n, int B, int lb, const int* __restrict__ act,
                                                 const double2* __restrict__ w, double2* __restrict__ u) {
  HZ_ROW(n)
  if (act[b]) u[o] = w[o];
}

// stationary solve, after each cycle (first: the start): per column the
// residual norm beta = sqrt(nrm2), a column stops at the first iterate with
// beta <= rtol fnorm (MG_OK) or a non-finite beta (MG_ERR_DIVERGED); iters
// counts the cycles applied to it; cnt = columns still iterating
__global__ __launch_bounds__(256) void k_hz_solve_check(FxState S, int B, const double2* __restrict__ nrm2,
                                                        double rtol, int first) {
  const int b = threadIdx.x;
  if (b < B) {
    const double nr = sqrt(nrm2[b].x);
    if (first) {
      S.status[b] = -1;
      S.iters[b] = 0;
      S.act[b] = 1;
    } else if (S.act[b]) {
      S.iters[b] += 1;
    }
    if (S.act[b]) {
      S.beta[b] = nr;
      if (!isfinite(nr)) {
        S.status[b] = MG_ERR_DIVERGED;
        S.act[b] = 0;
      } else if (nr <= rtol * S.fnorm[b]) {
        S.status[b] = MG_OK;
        S.act[b] = 0;
      }
    }
  }
  __syncthreads();
  fx_count(S, B);
}

// ------------------------------------------------------------------ host side
using zd = std::complex<double>;

struct HostCsrC {
  int nr, nc;
  const int32_t* rp;
  const int32_t* col;
  const double* re;
  const double* im;
};

mg_status check_csr(int nr, int nc, int64_t nnz, const int32_t* rp, const int32_t* col, const char* what) {
  if (nr <= 0 || nc <= 0 || !rp || (nnz > 0 && !col)) return hfail(MG_ERR_SHAPE, std::string(what) + ": empty or null");
  if (rp[0] != 0 || rp[nr] != nnz) return hfail(MG_ERR_SHAPE, std::string(what) + ": bad row pointers");
  for (int i = 0; i < nr; ++i) {
    if (rp[i + 1] < rp[i]) return hfail(MG_ERR_SHAPE, std::string(what) + ": row pointers decrease");
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= nc) return hfail(MG_ERR_SHAPE, std::string(what) + ": column out of range");
      if (k > rp[i] && col[k] <= col[k - 1]) return hfail(MG_ERR_SHAPE, std::string(what) + ": columns not sorted/unique");
    }
  }
  return MG_OK;
}

struct DevMem {
  std::vector<void*> ptrs;
  template <class X>
  mg_status alloc(X** p, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, count * sizeof(X)) != hipSuccess) {
      (void)hipGetLastError();
      return hfail(MG_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(X)) + " bytes failed");
    }
    ptrs.push_back(q);
    *p = static_cast<X*>(q);
    return MG_OK;
  }
  template <class X>
  mg_status upload(X** p, const std::vector<X>& h, hipStream_t st) {
    H_TRY(alloc(p, h.size()));
    H_HIP(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice, st));
    return MG_OK;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct mgh_ctx {
  virtual ~mgh_ctx() = default;
  virtual mg_status set_params(const double* v, hipStream_t st) = 0;
  virtual mg_status vcycle(const void* f, void* u, hipStream_t st) = 0;
  virtual mg_status fmg(const void* f, void* u, hipStream_t st) = 0;
  virtual mg_status residual(const double* f, const double* u, double* r, double* norms, hipStream_t st) = 0;
  virtual mg_status fgmres(const double* f, double* u, const mg_krylov_options* o, mg_rhs_info* info,
                           hipStream_t st) = 0;
  virtual mg_status solve(const double* f, double* u, double rtol, int max_cycles, int check_every,
                          mg_rhs_info* info, hipStream_t st) = 0;
  std::vector<int64_t> sizes;
};

namespace {

template <class T>
struct HzEngine final : mgh_ctx {
  struct Lv {
    int n = 0;
    CEll<T> A{};
    GEll G{};
    const T* invdeg = nullptr;
    const cx<T>* dinv = nullptr;
    REll<T> P{}, R{};            // P: n_l x n_{l+1}; R: n_{l+1} x n_l
    cx<T>*F = nullptr, *U = nullptr, *Rb = nullptr, *D = nullptr, *Y0 = nullptr, *Y1 = nullptr, *Tb = nullptr;
    cx<T>* scr = nullptr;        // GMRES scratch (global), or null when the step runs in LDS
    size_t lds = 0;              // dynamic LDS bytes of the GMRES step
    int gmode = 0;               // placement of its vectors (k_hz_gmres MODE)
    int kind = MGH_JACOBI, pre = 0, post = 0;
  };
  int J = 0, Bn = 0, lb = 0, KB = 0, KR = 0, KP = 0, v = 4;
  std::vector<Lv> lv;
  CEll<double> A64{};
  double2* Ainv = nullptr;
  int nc = 0;
  std::vector<double> theta, eta;
  std::vector<WK<T>> WB;
  WK<T> WR{}, WP{};
  DevMem mem, kmem;
  // Krylov workspace
  int km = -1;
  double2 *KV = nullptr, *KW = nullptr, *Kpart = nullptr, *Kh1 = nullptr, *Kh2 = nullptr, *Kn2 = nullptr,
          *Kn4 = nullptr;
  cx<T>*KZ = nullptr, *Kin = nullptr;
  FxState S{};
  int kblk = 0, kchunk = 0;
  int* hcnt = nullptr;

  ~HzEngine() override {
    (void)hipDeviceSynchronize();
    mem.release();
    kmem.release();
    if (hcnt) (void)hipHostFree(hcnt);
  }

  static W2<T> w2(const double* p) { return W2<T>{(T)p[0], (T)p[1], (T)p[2], (T)p[3]}; }
  static W2<T> eye() { return W2<T>{(T)1, (T)0, (T)0, (T)1}; }

  mg_status set_params(const double* vals, hipStream_t) override {
    if (!vals) return hfail(MG_ERR_INVALID_ARG, "null parameter values");
    const int per = 2 + 4 * (KB + 1);
    theta.assign(J - 1, 0.0);
    eta.assign(J - 1, 0.0);
    WB.assign(J - 1, WK<T>{});
    for (int l = 0; l < J - 1; ++l) {
      const double* p = vals + (size_t)l * per;
      theta[l] = p[0];
      eta[l] = p[1];
      for (int k = 0; k <= KB; ++k) WB[l].w[k] = w2(p + 2 + 4 * k);
    }
    const double* q = vals + (size_t)(J - 1) * per;
    WR = WK<T>{};
    WP = WK<T>{};
    for (int k = 0; k <= KR; ++k) WR.w[k] = w2(q + 4 * k);
    for (int k = 0; k <= KP; ++k) WP.w[k] = w2(q + 4 * (KR + 1) + 4 * k);
    return MG_OK;
  }

  unsigned rows_grid(int n) const { return (unsigned)(((size_t)n * (1u << lb) + 255) / 256); }
  unsigned lin_grid(size_t cnt) const { return (unsigned)((cnt + 255) / 256); }

  mg_status zero(cx<T>* p, int n, hipStream_t st) {
    const size_t c = (size_t)n * Bn;
    hipLaunchKernelGGL((k_hz_zero<T>), dim3(lin_grid(c)), dim3(256), 0, st, c, p);
    H_LAUNCH();
    return MG_OK;
  }

  // out (+)= s Phi(x) with weights W[0..K] on level l; the first sweep forms
  // W_{K-1} x + W_K (M x), the two leading Horner steps at once
  mg_status conv(int l, const WK<T>& W, int K, const cx<T>* x, cx<T>* out, T s, bool add, hipStream_t st) {
    Lv& L = lv[l];
    const dim3 g(rows_grid(L.n));
    if (K == 0) {
      if (add) hipLaunchKernelGGL((k_hz_hop<T, false, true>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb,
                                  (const cx<T>*)nullptr, x, W.w[0], s, out, W2<T>{});
      else hipLaunchKernelGGL((k_hz_hop<T, false, false>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb,
                              (const cx<T>*)nullptr, x, W.w[0], s, out, W2<T>{});
      H_LAUNCH();
      return MG_OK;
    }
    if (K == 1) {
      if (add) hipLaunchKernelGGL((k_hz_hop<T, true, true, true>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb, x,
                                  x, W.w[0], s, out, W.w[1]);
      else hipLaunchKernelGGL((k_hz_hop<T, true, false, true>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb, x, x,
                              W.w[0], s, out, W.w[1]);
      H_LAUNCH();
      return MG_OK;
    }
    hipLaunchKernelGGL((k_hz_hop<T, true, false, true>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb, x, x,
                       W.w[K - 1], (T)1, L.Y0, W.w[K]);
    H_LAUNCH();
    cx<T>* cur = L.Y0;
    cx<T>* nxt = L.Y1;
    for (int k = K - 2; k >= 1; --k) {
      hipLaunchKernelGGL((k_hz_hop<T, true, false>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb,
                         (const cx<T>*)cur, x, W.w[k], (T)1, nxt, W2<T>{});
      H_LAUNCH();
      std::swap(cur, nxt);
    }
    if (add) hipLaunchKernelGGL((k_hz_hop<T, true, true>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb,
                                (const cx<T>*)cur, x, W.w[0], s, out, W2<T>{});
    else hipLaunchKernelGGL((k_hz_hop<T, true, false>), g, dim3(256), 0, st, L.G, L.invdeg, Bn, lb,
                            (const cx<T>*)cur, x, W.w[0], s, out, W2<T>{});
    H_LAUNCH();
    return MG_OK;
  }

  mg_status smooth(int l, const cx<T>* f, cx<T>* u, hipStream_t st) {
    Lv& L = lv[l];
    if (L.kind == MGH_JACOBI) {
      hipLaunchKernelGGL((k_hz_resid<T, true>), dim3(rows_grid(L.n)), dim3(256), 0, st, L.A, Bn, lb, f,
                         (const cx<T>*)u, L.dinv, (T)theta[l], L.D);
      H_LAUNCH();
      return conv(l, WB[l], KB, L.D, u, (T)eta[l], true, st);
    }
    if (L.gmode == 1)
      hipLaunchKernelGGL((k_hz_gmres<T, 1>), dim3(Bn), dim3(kGT), L.lds, st, L.A, L.G, L.invdeg, Bn, f, u,
                         (T)theta[l], (T)eta[l], WB[l], KB, v, L.scr);
    else if (L.gmode == 2)
      hipLaunchKernelGGL((k_hz_gmres<T, 2>), dim3(Bn), dim3(kGTH), L.lds, st, L.A, L.G, L.invdeg, Bn, f, u,
                         (T)theta[l], (T)eta[l], WB[l], KB, v, L.scr);
    else
      hipLaunchKernelGGL((k_hz_gmres<T, 0>), dim3(Bn), dim3(kGTH), 0, st, L.A, L.G, L.invdeg, Bn, f, u,
                         (T)theta[l], (T)eta[l], WB[l], KB, v, L.scr);
    H_LAUNCH();
    return MG_OK;
  }

  // r_{l+1} = R_l Phi_R(x) into F[l+1]
  mg_status restrict_(int l, const cx<T>* x, hipStream_t st) {
    Lv& L = lv[l];
    Lv& C = lv[l + 1];
    const dim3 g(rows_grid(C.n));
    if (KR == 0) {
      hipLaunchKernelGGL((k_hz_xfer<T, false>), g, dim3(256), 0, st, L.R, Bn, lb, x, WR.w[0], C.F);
    } else {
      H_TRY(conv(l, WR, KR, x, L.D, (T)1, false, st));
      hipLaunchKernelGGL((k_hz_xfer<T, false>), g, dim3(256), 0, st, L.R, Bn, lb, (const cx<T>*)L.D, eye(), C.F);
    }
    H_LAUNCH();
    return MG_OK;
  }
  // out (+)= Phi_P(P_l U[l+1])
  mg_status prolong(int l, cx<T>* out, bool add, hipStream_t st) {
    Lv& L = lv[l];
    const dim3 g(rows_grid(L.n));
    const cx<T>* ec = lv[l + 1].U;
    if (KP == 0) {
      if (add) hipLaunchKernelGGL((k_hz_xfer<T, true>), g, dim3(256), 0, st, L.P, Bn, lb, ec, WP.w[0], out);
      else hipLaunchKernelGGL((k_hz_xfer<T, false>), g, dim3(256), 0, st, L.P, Bn, lb, ec, WP.w[0], out);
      H_LAUNCH();
      return MG_OK;
    }
    hipLaunchKernelGGL((k_hz_xfer<T, false>), g, dim3(256), 0, st, L.P, Bn, lb, ec, eye(), L.Tb);
    H_LAUNCH();
    return conv(l, WP, KP, L.Tb, out, (T)1, add, st);
  }

  mg_status coarse(const cx<T>* f, cx<T>* u, hipStream_t st) {
    hipLaunchKernelGGL((k_hz_dense<T>), dim3(nc), dim3(256), 0, st, nc, Bn, lb, (const double2*)Ainv, f, u);
    H_LAUNCH();
    return MG_OK;
  }

  mg_status cycle(int l, const cx<T>* f, cx<T>* u, hipStream_t st) {
    if (l == J - 1) return coarse(f, u, st);
    Lv& L = lv[l];
    for (int s = 0; s < L.pre; ++s) H_TRY(smooth(l, f, u, st));
    hipLaunchKernelGGL((k_hz_resid<T, false>), dim3(rows_grid(L.n)), dim3(256), 0, st, L.A, Bn, lb, f,
                       (const cx<T>*)u, (const cx<T>*)nullptr, (T)0, L.Rb);
    H_LAUNCH();
    H_TRY(restrict_(l, L.Rb, st));
    if (l + 1 < J - 1) H_TRY(zero(lv[l + 1].U, lv[l + 1].n, st));
    H_TRY(cycle(l + 1, lv[l + 1].F, lv[l + 1].U, st));
    H_TRY(prolong(l, u, true, st));
    for (int s = 0; s < L.post; ++s) H_TRY(smooth(l, f, u, st));
    return MG_OK;
  }

  // the cycle reads f after it has started writing u
  mg_status check_disjoint(const void* f, const void* u) const {
    const size_t bytes = (size_t)lv[0].n * Bn * sizeof(cx<T>);
    const char* a = static_cast<const char*>(f);
    const char* b = static_cast<const char*>(u);
    if (a < b + bytes && b < a + bytes) return hfail(MG_ERR_INVALID_ARG, "f and u overlap");
    return MG_OK;
  }

  mg_status vcycle(const void* f, void* u, hipStream_t st) override {
    if (!f || !u) return hfail(MG_ERR_INVALID_ARG, "null vector");
    H_TRY(check_disjoint(f, u));
    return cycle(0, static_cast<const cx<T>*>(f), static_cast<cx<T>*>(u), st);
  }

  mg_status fmg_(const cx<T>* f, cx<T>* u, hipStream_t st) {
    std::vector<const cx<T>*> fs(J);
    fs[0] = f;
    for (int l = 0; l < J - 1; ++l) {
      H_TRY(restrict_(l, fs[l], st));
      fs[l + 1] = lv[l + 1].F;
    }
    H_TRY(coarse(fs[J - 1], lv[J - 1].U, st));
    for (int l = J - 2; l >= 0; --l) {
      cx<T>* ul = l == 0 ? u : lv[l].U;
      H_TRY(prolong(l, ul, false, st));
      H_TRY(cycle(l, fs[l], ul, st));
    }
    return MG_OK;
  }
  mg_status fmg(const void* f, void* u, hipStream_t st) override {
    if (!f || !u) return hfail(MG_ERR_INVALID_ARG, "null vector");
    H_TRY(check_disjoint(f, u));
    return fmg_(static_cast<const cx<T>*>(f), static_cast<cx<T>*>(u), st);
  }

  // ------------------------------------------------------------ Krylov
  mg_status kr_alloc(int m, hipStream_t st) {
    if (km >= m) return MG_OK;
    H_HIP(hipStreamSynchronize(st));
    kmem.release();
    km = -1;
    const int n = lv[0].n;
    const size_t nB = (size_t)n * Bn;
    kblk = std::min(kKrBlocks, std::max(1, (n + (256 >> lb) - 1) / (256 >> lb)));
    kchunk = (n + kblk - 1) / kblk;
    H_TRY(kmem.alloc(&KV, nB * (m + 1)));
    H_TRY(kmem.alloc(&KW, nB));
    H_TRY(kmem.alloc(&KZ, nB * m));
    H_TRY(kmem.alloc(&Kin, nB));
    H_TRY(kmem.alloc(&Kpart, (size_t)kblk * (m + 2) * Bn));
    H_TRY(kmem.alloc(&Kh1, (size_t)(m + 2) * Bn));
    H_TRY(kmem.alloc(&Kh2, (size_t)(m + 2) * Bn));
    H_TRY(kmem.alloc(&Kn2, (size_t)Bn));
    H_TRY(kmem.alloc(&Kn4, (size_t)Bn));
    H_TRY(kmem.alloc(&S.H, (size_t)(m + 1) * m * Bn));
    H_TRY(kmem.alloc(&S.cs, (size_t)m * Bn));
    H_TRY(kmem.alloc(&S.sn, (size_t)m * Bn));
    H_TRY(kmem.alloc(&S.g, (size_t)(m + 1) * Bn));
    H_TRY(kmem.alloc(&S.y, (size_t)m * Bn));
    H_TRY(kmem.alloc(&S.sig, (size_t)Bn));
    H_TRY(kmem.alloc(&S.fnorm, (size_t)Bn));
    H_TRY(kmem.alloc(&S.beta, (size_t)Bn));
    H_TRY(kmem.alloc(&S.act, (size_t)Bn));
    H_TRY(kmem.alloc(&S.jd, (size_t)Bn));
    H_TRY(kmem.alloc(&S.iters, (size_t)Bn));
    H_TRY(kmem.alloc(&S.status, (size_t)Bn));
    H_TRY(kmem.alloc(&S.cnt, 1));
    H_TRY(kmem.alloc(&S.flag, 1));
    H_HIP(hipMemsetAsync(S.flag, 0, sizeof(int), st));
    km = m;
    return MG_OK;
  }
  // out[0..nv) = <v_t, w>, out[nv].x = ||w||^2 (zero work when skipped)
  mg_status kr_dot(int nv, const double2* w, long wrs, double2* out, const int* skip, hipStream_t st) {
    const int n = lv[0].n, mp1 = km + 1;
    const dim3 g(kblk, std::max(1, (nv + kNG - 1) / kNG));
    hipLaunchKernelGGL(k_fx_dot, g, dim3(256), 0, st, n, Bn, lb, kchunk, (const double2*)KV, mp1, nv, w, wrs,
                       Kpart, skip);
    H_LAUNCH();
    const int rows = nv + 1;
    hipLaunchKernelGGL(k_fx_reduce, dim3(((size_t)rows * Bn + 3) / 4), dim3(256), 0, st, kblk, rows, Bn,
                       (const double2*)Kpart, out, skip);
    H_LAUNCH();
    return MG_OK;
  }
  mg_status kr_upd(int nv, const double2* h, const double2* wi, long wis, double2* wo, long wos, double2* n2,
                   const int* skip, hipStream_t st) {
    const int n = lv[0].n, mp1 = km + 1;
    hipLaunchKernelGGL(k_fx_upd, dim3(kblk), dim3(256), 0, st, n, Bn, lb, kchunk, (const double2*)KV, mp1, nv, h,
                       wi, wis, wo, wos, Kpart, skip);
    H_LAUNCH();
    hipLaunchKernelGGL(k_fx_reduce, dim3(((size_t)Bn + 3) / 4), dim3(256), 0, st, kblk, 1, Bn,
                       (const double2*)Kpart, n2, skip);
    H_LAUNCH();
    return MG_OK;
  }
  mg_status read_cnt(int* c, hipStream_t st) {
    H_HIP(hipMemcpyAsync(hcnt, S.cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    H_HIP(hipStreamSynchronize(st));
    *c = *hcnt;
    return MG_OK;
  }

  mg_status residual(const double* f, const double* u, double* r, double* norms, hipStream_t st) override {
    if (!f || !u) return hfail(MG_ERR_INVALID_ARG, "null vector");
    H_TRY(kr_alloc(std::max(km, 1), st));
    const int n = lv[0].n;
    double2* w = r ? reinterpret_cast<double2*>(r) : KW;
    hipLaunchKernelGGL(k_fx_resid, dim3(rows_grid(n)), dim3(256), 0, st, A64, Bn, lb,
                       reinterpret_cast<const double2*>(f), reinterpret_cast<const double2*>(u), w);
    H_LAUNCH();
    if (norms) {
      H_TRY(kr_dot(0, w, Bn, Kh1, nullptr, st));
      hipLaunchKernelGGL(k_fx_sqrt, dim3(1), dim3(256), 0, st, Bn, (const double2*)Kh1, norms);
      H_LAUNCH();
    }
    return MG_OK;
  }

  // per-column results of a solve (status, iterations, final relative residual)
  mg_status report(mg_rhs_info* info, hipStream_t st) {
    std::vector<int> hs(Bn), hi(Bn);
    std::vector<double> hb(Bn), hf(Bn);
    H_HIP(hipMemcpyAsync(hs.data(), S.status, Bn * sizeof(int), hipMemcpyDeviceToHost, st));
    H_HIP(hipMemcpyAsync(hi.data(), S.iters, Bn * sizeof(int), hipMemcpyDeviceToHost, st));
    H_HIP(hipMemcpyAsync(hb.data(), S.beta, Bn * sizeof(double), hipMemcpyDeviceToHost, st));
    H_HIP(hipMemcpyAsync(hf.data(), S.fnorm, Bn * sizeof(double), hipMemcpyDeviceToHost, st));
    H_HIP(hipStreamSynchronize(st));
    mg_status ret = MG_OK;
    for (int b = 0; b < Bn; ++b) {
      const int s = hs[b] == -1 ? MG_ERR_NOT_CONVERGED : hs[b];
      if (info) {
        info[b].iters = hi[b];
        info[b].status = s;
        info[b].relres = hf[b] > 0 ? hb[b] / hf[b] : hb[b];
      }
      if (s == MG_ERR_DIVERGED) ret = MG_ERR_DIVERGED;
      else if (s != MG_OK && ret == MG_OK) ret = MG_ERR_NOT_CONVERGED;
    }
    if (ret != MG_OK) h_err = ret == MG_ERR_DIVERGED ? "a column's residual is not finite" : "a column did not converge";
    return ret;
  }

  // Stationary iteration u <- LMG(A, f, u) (FP64 cycles): each cycle runs on a
  // copy of u, which the columns still iterating take over; their FP64
  // residuals are checked on the device after every cycle.
  mg_status solve(const double* fd, double* ud, double rtol, int max_cycles, int check_every, mg_rhs_info* info,
                  hipStream_t st) override {
    if (!fd || !ud) return hfail(MG_ERR_INVALID_ARG, "null vector");
    if (!std::is_same<T, double>::value)
      return hfail(MG_ERR_UNSUPPORTED, "the stationary solve needs FP64 cycles (the cycle is not affine, so there is "
                                       "no refinement form for lower-precision cycles)");
    if (max_cycles < 1 || check_every < 1 || !(rtol >= 0.0)) return hfail(MG_ERR_INVALID_ARG, "bad solve options");
    H_TRY(check_disjoint(fd, ud));
    H_TRY(kr_alloc(std::max(km, 1), st));
    const int n = lv[0].n;
    const size_t nB = (size_t)n * Bn;
    const double2* f = reinterpret_cast<const double2*>(fd);
    double2* u = reinterpret_cast<double2*>(ud);
    cx<T>* w = reinterpret_cast<cx<T>*>(Kin);           // the cycle's working copy (double2 here)
    const dim3 rg(rows_grid(n));
    hipLaunchKernelGGL(k_fx_resid, rg, dim3(256), 0, st, A64, Bn, lb, f, (const double2*)nullptr, KW);
    H_LAUNCH();
    H_TRY(kr_dot(0, KW, Bn, Kh1, nullptr, st));
    hipLaunchKernelGGL(k_fx_start, dim3(1), dim3(256), 0, st, S, Bn, km, (const double2*)Kh1, rtol, max_cycles, 1);
    H_LAUNCH();
    hipLaunchKernelGGL(k_fx_resid, rg, dim3(256), 0, st, A64, Bn, lb, f, (const double2*)u, KW);
    H_LAUNCH();
    H_TRY(kr_dot(0, KW, Bn, Kh1, nullptr, st));
    hipLaunchKernelGGL(k_hz_solve_check, dim3(1), dim3(256), 0, st, S, Bn, (const double2*)Kh1, rtol, 1);
    H_LAUNCH();
    int cnt = 0;
    H_TRY(read_cnt(&cnt, st));
    for (int c = 1; c <= max_cycles && cnt > 0; ++c) {
      hipLaunchKernelGGL((k_hz_copy<T>), dim3(lin_grid(nB)), dim3(256), 0, st, nB,
                         reinterpret_cast<const cx<T>*>(u), w);
      H_LAUNCH();
      H_TRY(cycle(0, reinterpret_cast<const cx<T>*>(f), w, st));
      hipLaunchKernelGGL(k_hz_take, rg, dim3(256), 0, st, n, Bn, lb, (const int*)S.act,
                         reinterpret_cast<const double2*>(w), u);
      H_LAUNCH();
      hipLaunchKernelGGL(k_fx_resid, rg, dim3(256), 0, st, A64, Bn, lb, f, (const double2*)u, KW);
      H_LAUNCH();
      H_TRY(kr_dot(0, KW, Bn, Kh1, nullptr, st));
      hipLaunchKernelGGL(k_hz_solve_check, dim3(1), dim3(256), 0, st, S, Bn, (const double2*)Kh1, rtol, 0);
      H_LAUNCH();
      if (c % check_every == 0 || c == max_cycles) H_TRY(read_cnt(&cnt, st));
    }
    return report(info, st);
  }

  mg_status fgmres(const double* fd, double* xd, const mg_krylov_options* o, mg_rhs_info* info,
                   hipStream_t st) override {
    if (!fd || !xd || !o) return hfail(MG_ERR_INVALID_ARG, "null argument");
    if (o->restart < 1 || o->restart > 63 || o->max_iter < 1 || !(o->rtol >= 0.0) ||
        o->precond < MG_PC_NONE || o->precond > MG_PC_FMG)
      return hfail(MG_ERR_INVALID_ARG, "bad Krylov options");
    const int m = o->restart, n = lv[0].n;
    H_TRY(kr_alloc(m, st));
    const int mp1 = km + 1;
    const size_t nB = (size_t)n * Bn;
    const double2* f = reinterpret_cast<const double2*>(fd);
    double2* x = reinterpret_cast<double2*>(xd);
    const dim3 rg(rows_grid(n));
    // ||f||
    hipLaunchKernelGGL(k_fx_resid, rg, dim3(256), 0, st, A64, Bn, lb, f, (const double2*)nullptr, KW);
    H_LAUNCH();
    H_TRY(kr_dot(0, KW, Bn, Kh1, nullptr, st));
    hipLaunchKernelGGL(k_fx_start, dim3(1), dim3(256), 0, st, S, Bn, m, (const double2*)Kh1, o->rtol, o->max_iter, 1);
    H_LAUNCH();
    const double thr2 = o->reorth * o->reorth;
    int cnt = 0;
    for (;;) {
      hipLaunchKernelGGL(k_fx_resid, rg, dim3(256), 0, st, A64, Bn, lb, f, (const double2*)x, KW);
      H_LAUNCH();
      H_TRY(kr_dot(0, KW, Bn, Kh1, nullptr, st));
      hipLaunchKernelGGL(k_fx_start, dim3(1), dim3(256), 0, st, S, Bn, m, (const double2*)Kh1, o->rtol,
                         o->max_iter, 0);
      H_LAUNCH();
      H_TRY(read_cnt(&cnt, st));
      if (cnt == 0) break;
      hipLaunchKernelGGL((k_fx_scale<T>), rg, dim3(256), 0, st, n, Bn, lb, (const double*)S.sig,
                         (const double2*)KW, (long)Bn, KV, (long)mp1 * Bn, Kin);
      H_LAUNCH();
      for (int j = 0; j < m; ++j) {
        cx<T>* zj = KZ + (size_t)j * nB;
        switch (o->precond) {
          case MG_PC_NONE:
            hipLaunchKernelGGL((k_hz_copy<T>), dim3(lin_grid(nB)), dim3(256), 0, st, nB, (const cx<T>*)Kin, zj);
            H_LAUNCH();
            break;
          case MG_PC_VCYCLE:
            H_TRY(zero(zj, n, st));
            H_TRY(cycle(0, Kin, zj, st));
            break;
          default:
            H_TRY(fmg_(Kin, zj, st));
            break;
        }
        hipLaunchKernelGGL((k_fx_amul<T>), rg, dim3(256), 0, st, A64, Bn, lb, (const cx<T>*)zj, KW);
        H_LAUNCH();
        const int nv = j + 1;
        double2* vn = KV + (size_t)(j + 1) * Bn;
        const long vrs = (long)mp1 * Bn;
        H_TRY(kr_dot(nv, KW, Bn, Kh1, nullptr, st));
        H_TRY(kr_upd(nv, Kh1, KW, Bn, vn, vrs, Kn2, nullptr, st));
        hipLaunchKernelGGL(k_fx_flag, dim3(1), dim3(256), 0, st, S, Bn, (const double2*)(Kh1 + (size_t)nv * Bn),
                           (const double2*)Kn2, thr2);
        H_LAUNCH();
        H_TRY(kr_dot(nv, vn, vrs, Kh2, S.flag, st));
        H_TRY(kr_upd(nv, Kh2, vn, vrs, vn, vrs, Kn4, S.flag, st));
        hipLaunchKernelGGL(k_fx_givens, dim3(1), dim3(256), 0, st, S, Bn, m, j, (const double2*)Kh1,
                           (const double2*)Kh2, (const double2*)Kn2, (const double2*)Kn4, o->rtol, o->max_iter);
        H_LAUNCH();
        hipLaunchKernelGGL((k_fx_scale<T>), rg, dim3(256), 0, st, n, Bn, lb, (const double*)S.sig,
                           (const double2*)vn, vrs, vn, vrs, Kin);
        H_LAUNCH();
        H_TRY(read_cnt(&cnt, st));
        if (cnt == 0) break;
      }
      hipLaunchKernelGGL(k_fx_lsq, dim3(1), dim3(256), 0, st, S, Bn, m);
      H_LAUNCH();
      hipLaunchKernelGGL((k_fx_xupd<T>), rg, dim3(256), 0, st, n, Bn, lb, (const int*)S.jd, (const double2*)S.y,
                         (const cx<T>*)KZ, nB, x);
      H_LAUNCH();
    }
    std::vector<int> hs(Bn), hi(Bn);
    std::vector<double> hb(Bn), hf(Bn);
    H_HIP(hipMemcpyAsync(hs.data(), S.status, Bn * sizeof(int), hipMemcpyDeviceToHost, st));
    H_HIP(hipMemcpyAsync(hi.data(), S.iters, Bn * sizeof(int), hipMemcpyDeviceToHost, st));
    H_HIP(hipMemcpyAsync(hb.data(), S.beta, Bn * sizeof(double), hipMemcpyDeviceToHost, st));
    H_HIP(hipMemcpyAsync(hf.data(), S.fnorm, Bn * sizeof(double), hipMemcpyDeviceToHost, st));
    H_HIP(hipStreamSynchronize(st));
    mg_status ret = MG_OK;
    for (int b = 0; b < Bn; ++b) {
      if (info) {
        info[b].iters = hi[b];
        info[b].status = hs[b];
        info[b].relres = hf[b] > 0 ? hb[b] / hf[b] : hb[b];
      }
      if (hs[b] == MG_ERR_DIVERGED) ret = MG_ERR_DIVERGED;
      else if (hs[b] != MG_OK && ret == MG_OK) ret = MG_ERR_NOT_CONVERGED;
    }
    if (ret != MG_OK) h_err = ret == MG_ERR_DIVERGED ? "a column's residual is not finite" : "a column did not converge";
    return ret;
  }

  // ------------------------------------------------------------ setup
  mg_status setup(const mgh_hierarchy* h, const mgh_params* p, const mgh_options* o, hipStream_t st) {
    J = h->nlevels;
    Bn = o->nrhs;
    while ((1 << lb) < Bn) ++lb;
    KB = p->KB;
    KR = p->KR;
    KP = p->KP;
    v = p->gmres_steps;
    lv.assign(J, Lv{});
    sizes.assign(J, 0);
    for (int l = 0; l < J; ++l) sizes[l] = h->A[l].nrows;
    for (int l = 0; l < J - 1; ++l) {
      lv[l].kind = p->smoother[l];
      lv[l].pre = p->nu_pre[l];
      lv[l].post = p->nu_post[l];
    }
    H_TRY(set_params(p->values, st));
    for (int l = 0; l < J; ++l) {
      const mgh_ccsr& A = h->A[l];
      Lv& L = lv[l];
      const int n = A.nrows;
      L.n = n;
      // complex ELL of A (diagonal included), graph ELL, inverse degrees and diagonals
      int w = 0, wg = 0;
      for (int i = 0; i < n; ++i) {
        w = std::max(w, A.rowptr[i + 1] - A.rowptr[i]);
        int dg = 0;
        for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
          if (A.col[k] != i && (A.re[k] != 0.0 || A.im[k] != 0.0)) ++dg;
        wg = std::max(wg, dg);
      }
      std::vector<int> col((size_t)w * n), gcol((size_t)std::max(wg, 1) * n);
      std::vector<cx<T>> val((size_t)w * n);
      std::vector<double2> val64(l == 0 ? (size_t)w * n : 0);
      std::vector<T> invdeg(n);
      std::vector<cx<T>> dinv(n);
      for (int i = 0; i < n; ++i) {
        int s = 0, q = 0;
        zd dg(0.0, 0.0);
        for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k, ++s) {
          col[(size_t)s * n + i] = A.col[k];
          cx<T> c;
          c.x = (T)A.re[k];
          c.y = (T)A.im[k];
          val[(size_t)s * n + i] = c;
          if (l == 0) val64[(size_t)s * n + i] = make_double2(A.re[k], A.im[k]);
          if (A.col[k] == i) dg = zd(A.re[k], A.im[k]);
          else if (A.re[k] != 0.0 || A.im[k] != 0.0) gcol[(size_t)q++ * n + i] = A.col[k];
        }
        for (; s < w; ++s) {
          col[(size_t)s * n + i] = i;
          cx<T> z;
          z.x = 0;
          z.y = 0;
          val[(size_t)s * n + i] = z;
          if (l == 0) val64[(size_t)s * n + i] = make_double2(0.0, 0.0);
        }
        invdeg[i] = q > 0 ? (T)(1.0 / q) : (T)0;
        for (; q < std::max(wg, 1); ++q) gcol[(size_t)q * n + i] = i;
        if (l < J - 1 && lv[l].kind == MGH_JACOBI && dg == zd(0.0, 0.0))
          return hfail(MG_ERR_SHAPE, "zero diagonal on a Jacobi level");
        const zd di = dg == zd(0.0, 0.0) ? zd(0.0, 0.0) : 1.0 / dg;
        cx<T> c;
        c.x = (T)di.real();
        c.y = (T)di.imag();
        dinv[i] = c;
      }
      int* dcol;
      cx<T>* dval;
      H_TRY(mem.upload(&dcol, col, st));
      H_TRY(mem.upload(&dval, val, st));
      L.A = CEll<T>{n, w, dcol, dval};
      int* dg;
      H_TRY(mem.upload(&dg, gcol, st));
      L.G = GEll{n, wg, dg};
      T* did;
      H_TRY(mem.upload(&did, invdeg, st));
      L.invdeg = did;
      cx<T>* ddi;
      H_TRY(mem.upload(&ddi, dinv, st));
      L.dinv = ddi;
      if (l == 0) {
        double2* dv64;
        H_TRY(mem.upload(&dv64, val64, st));
        A64 = CEll<double>{n, w, dcol, dv64};
      }
      const size_t nB = (size_t)n * Bn;
      if (l > 0) {
        H_TRY(mem.alloc(&L.F, nB));
        H_TRY(mem.alloc(&L.U, nB));
      }
      if (l < J - 1) {
        H_TRY(mem.alloc(&L.Rb, nB));
        H_TRY(mem.alloc(&L.D, nB));
        H_TRY(mem.alloc(&L.Y0, nB));
        H_TRY(mem.alloc(&L.Y1, nB));
        H_TRY(mem.alloc(&L.Tb, nB));
        if (L.kind == MGH_GMRES) {
          const size_t all = (size_t)hz_slots(v) * n * sizeof(cx<T>), basis = (size_t)v * n * sizeof(cx<T>);
          if (all <= (size_t)kGmresLds) {
            L.gmode = 1;
            L.lds = all;
          } else if (v >= 3 && basis <= (size_t)kGmresLds) {
            L.gmode = 2;
            L.lds = basis;
            H_TRY(mem.alloc(&L.scr, nB * 3));
          } else {
            L.gmode = 0;
            L.lds = 0;
            H_TRY(mem.alloc(&L.scr, nB * (size_t)hz_slots(v)));
          }
        }
      }
    }
    // transfers
    for (int l = 0; l < J - 1; ++l) {
      auto ell = [&](const mg_csr& M, bool transpose, REll<T>& out) -> mg_status {
        // rows of the operator: M itself, or M^T (R = P^T)
        const int nr = transpose ? M.ncols : M.nrows;
        std::vector<std::vector<std::pair<int, double>>> rows(nr);
        for (int i = 0; i < M.nrows; ++i)
          for (int k = M.rowptr[i]; k < M.rowptr[i + 1]; ++k) {
            if (transpose) rows[M.col[k]].push_back({i, M.val[k]});
            else rows[i].push_back({M.col[k], M.val[k]});
          }
        int w = 1;
        for (auto& r : rows) w = std::max(w, (int)r.size());
        // padding slots: weight 0, pointing at a column the row already reads
        // (not all at column 0, which every row's padding would load)
        const int ncol = transpose ? M.nrows : M.ncols;
        std::vector<int> col((size_t)w * nr, 0);
        std::vector<T> val((size_t)w * nr, (T)0);
        for (int i = 0; i < nr; ++i) {
          for (size_t s = 0; s < rows[i].size(); ++s) {
            col[s * nr + i] = rows[i][s].first;
            val[s * nr + i] = (T)rows[i][s].second;
          }
          const int pc = rows[i].empty() ? (int)std::min<long>((long)i * ncol / nr, (long)ncol - 1)
                                         : rows[i][0].first;
          for (size_t s = rows[i].size(); s < (size_t)w; ++s) col[s * nr + i] = pc;
        }
        int* dc;
        T* dv;
        H_TRY(mem.upload(&dc, col, st));
        H_TRY(mem.upload(&dv, val, st));
        out = REll<T>{nr, w, dc, dv};
        return MG_OK;
      };
      H_TRY(ell(h->P[l], false, lv[l].P));
      if (h->R) H_TRY(ell(h->R[l], false, lv[l].R));
      else H_TRY(ell(h->P[l], true, lv[l].R));
    }
    // coarsest inverse: complex Gauss-Jordan with partial pivoting
    {
      const mgh_ccsr& A = h->A[J - 1];
      nc = A.nrows;
      std::vector<zd> M((size_t)nc * nc, zd(0.0, 0.0)), I((size_t)nc * nc, zd(0.0, 0.0));
      for (int i = 0; i < nc; ++i) {
        I[(size_t)i * nc + i] = 1.0;
        for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) M[(size_t)i * nc + A.col[k]] = zd(A.re[k], A.im[k]);
      }
      for (int c = 0; c < nc; ++c) {
        int pr = c;
        for (int r = c + 1; r < nc; ++r)
          if (std::abs(M[(size_t)r * nc + c]) > std::abs(M[(size_t)pr * nc + c])) pr = r;
        if (std::abs(M[(size_t)pr * nc + c]) == 0.0) return hfail(MG_ERR_SHAPE, "coarsest matrix is singular");
        if (pr != c)
          for (int k = 0; k < nc; ++k) {
            std::swap(M[(size_t)pr * nc + k], M[(size_t)c * nc + k]);
            std::swap(I[(size_t)pr * nc + k], I[(size_t)c * nc + k]);
          }
        const zd piv = M[(size_t)c * nc + c];
        for (int k = 0; k < nc; ++k) {
          M[(size_t)c * nc + k] /= piv;
          I[(size_t)c * nc + k] /= piv;
        }
        for (int r = 0; r < nc; ++r) {
          if (r == c) continue;
          const zd fct = M[(size_t)r * nc + c];
          if (fct == zd(0.0, 0.0)) continue;
          for (int k = 0; k < nc; ++k) {
            M[(size_t)r * nc + k] -= fct * M[(size_t)c * nc + k];
            I[(size_t)r * nc + k] -= fct * I[(size_t)c * nc + k];
          }
        }
      }
      std::vector<double2> inv((size_t)nc * nc);
      for (size_t k = 0; k < inv.size(); ++k) inv[k] = make_double2(I[k].real(), I[k].imag());
      H_TRY(mem.upload(&Ainv, inv, st));
    }
    H_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hz_gmres<T, 1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kGmresLds));
    H_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hz_gmres<T, 2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kGmresLds));
    H_HIP(hipHostMalloc((void**)&hcnt, sizeof(int)));
    H_HIP(hipStreamSynchronize(st));
    return MG_OK;
  }
};

mg_status check_setup(const mgh_hierarchy* h, const mgh_params* p, const mgh_options* o) {
  if (!h || !p || !o || !h->A || !h->P || !p->values || !p->smoother || !p->nu_pre || !p->nu_post)
    return hfail(MG_ERR_INVALID_ARG, "null argument");
  const int J = h->nlevels;
  if (J < 2) return hfail(MG_ERR_INVALID_ARG, "need at least two levels");
  if (o->precision != MG_FP64 && o->precision != MG_FP32) return hfail(MG_ERR_INVALID_ARG, "precision must be FP64 or FP32");
  if (o->nrhs < 1 || o->nrhs > kMaxB) return hfail(MG_ERR_INVALID_ARG, "nrhs must be 1..256");
  for (int K : {p->KB, p->KR, p->KP})
    if (K < 0 || K > kMaxK) return hfail(MG_ERR_INVALID_ARG, "convolution order must be 0..8");
  if (p->gmres_steps < 1 || p->gmres_steps > kMaxV) return hfail(MG_ERR_INVALID_ARG, "gmres_steps must be 1..8");
  for (int l = 0; l < J - 1; ++l) {
    if (p->smoother[l] != MGH_JACOBI && p->smoother[l] != MGH_GMRES) return hfail(MG_ERR_INVALID_ARG, "bad smoother kind");
    if (p->nu_pre[l] < 0 || p->nu_pre[l] > kMaxNu || p->nu_post[l] < 0 || p->nu_post[l] > kMaxNu)
      return hfail(MG_ERR_INVALID_ARG, "smoothing steps must be 0..8");
  }
  for (int l = 0; l < J; ++l) {
    const mgh_ccsr& A = h->A[l];
    if (A.nrows != A.ncols) return hfail(MG_ERR_SHAPE, "A_" + std::to_string(l) + " is not square");
    if (!A.re || !A.im) return hfail(MG_ERR_INVALID_ARG, "null matrix values");
    H_TRY(check_csr(A.nrows, A.ncols, A.nnz, A.rowptr, A.col, ("A_" + std::to_string(l)).c_str()));
  }
  if (h->A[J - 1].nrows > 4096) return hfail(MG_ERR_UNSUPPORTED, "coarsest level larger than 4096 rows");
  for (int l = 0; l < J - 1; ++l) {
    const mg_csr& P = h->P[l];
    if (P.nrows != h->A[l].nrows || P.ncols != h->A[l + 1].nrows || !P.val)
      return hfail(MG_ERR_SHAPE, "P_" + std::to_string(l) + " has the wrong shape");
    H_TRY(check_csr(P.nrows, P.ncols, P.nnz, P.rowptr, P.col, ("P_" + std::to_string(l)).c_str()));
    if (h->R) {
      const mg_csr& R = h->R[l];
      if (R.nrows != h->A[l + 1].nrows || R.ncols != h->A[l].nrows || !R.val)
        return hfail(MG_ERR_SHAPE, "R_" + std::to_string(l) + " has the wrong shape");
      H_TRY(check_csr(R.nrows, R.ncols, R.nnz, R.rowptr, R.col, ("R_" + std::to_string(l)).c_str()));
    }
  }
  return MG_OK;
}

}  // namespace

extern "C" {

int64_t mgh_num_params(int32_t J, int32_t KB, int32_t KR, int32_t KP) {
  if (J < 2 || KB < 0 || KR < 0 || KP < 0) return -1;
  return (int64_t)(J - 1) * (2 + 4 * (KB + 1)) + 4 * (KR + 1) + 4 * (KP + 1);
}

mg_status mgh_setup(const mgh_hierarchy* h, const mgh_params* p, const mgh_options* o, void* stream,
                    mgh_ctx** out) {
  h_err.clear();
  if (!out) return hfail(MG_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  H_TRY(check_setup(h, p, o));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::unique_ptr<mgh_ctx> c;
  mg_status s;
  if (o->precision == MG_FP64) {
    auto e = std::make_unique<HzEngine<double>>();
    s = e->setup(h, p, o, st);
    c = std::move(e);
  } else {
    auto e = std::make_unique<HzEngine<float>>();
    s = e->setup(h, p, o, st);
    c = std::move(e);
  }
  if (s != MG_OK) return s;
  *out = c.release();
  return MG_OK;
}

mg_status mgh_set_params(mgh_ctx* c, const double* values, void* stream) {
  if (!c) return hfail(MG_ERR_INVALID_ARG, "null context");
  return c->set_params(values, static_cast<hipStream_t>(stream));
}

mg_status mgh_vcycle(mgh_ctx* c, const void* f, void* u, void* stream) {
  if (!c) return hfail(MG_ERR_INVALID_ARG, "null context");
  return c->vcycle(f, u, static_cast<hipStream_t>(stream));
}

mg_status mgh_fmg(mgh_ctx* c, const void* f, void* u, void* stream) {
  if (!c) return hfail(MG_ERR_INVALID_ARG, "null context");
  return c->fmg(f, u, static_cast<hipStream_t>(stream));
}

mg_status mgh_residual(mgh_ctx* c, const double* f, const double* u, double* r, double* norms, void* stream) {
  if (!c) return hfail(MG_ERR_INVALID_ARG, "null context");
  return c->residual(f, u, r, norms, static_cast<hipStream_t>(stream));
}

mg_status mgh_fgmres(mgh_ctx* c, const double* f, double* u, const mg_krylov_options* o, mg_rhs_info* info,
                     void* stream) {
  if (!c) return hfail(MG_ERR_INVALID_ARG, "null context");
  return c->fgmres(f, u, o, info, static_cast<hipStream_t>(stream));
}

mg_status mgh_solve(mgh_ctx* c, const double* f, double* u, double rtol, int32_t max_cycles, int32_t check_every,
                    mg_rhs_info* info, void* stream) {
  if (!c) return hfail(MG_ERR_INVALID_ARG, "null context");
  return c->solve(f, u, rtol, max_cycles, check_every, info, static_cast<hipStream_t>(stream));
}

mg_status mgh_level_info(const mgh_ctx* c, int64_t* n) {
  if (!c || !n) return hfail(MG_ERR_INVALID_ARG, "null argument");
  for (size_t l = 0; l < c->sizes.size(); ++l) n[l] = c->sizes[l];
  return MG_OK;
}

void mgh_destroy(mgh_ctx* c) { delete c; }

const char* mgh_last_error(void) { return h_err.c_str(); }

}  // extern "C"
