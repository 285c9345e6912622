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

#include <type_traits>

#include "chebtab.hpp"

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

// Level operator in ELL form.  Off-diagonal slots are slot-major (entry
// (k, i) at k*ld + i); a padding slot has col == i and val == 0.  Rows
// [n, ld) of every slot and of the per-row arrays are padding with a valid
// column (n - 1) and zero values, so four consecutive rows starting at a
// multiple of 4 can always be read as one 16-byte vector.
template <class C> struct Lvl {
  int n;
  int ld;                   // slot stride of the ELL arrays: n rounded up to a multiple of 4
  int w;                    // off-diagonal ELL width of A
  const int* col;
  const C* val;
  const C* diag;
  const C* invdiag;
  int wg;                   // ELL width of the graph
  const int* gcol;          // graph neighbours (padding col == i)
  const C* invdeg;          // row scale r_i of the aggregation: 1/|N(i)| (0 for an isolated
                            // node) for the mean, 1/sum_j w_ij for weighted, 1 for symmetric
  const C* gval;            // edge weights w_ij in the graph's slots (padding 0), or null
                            // for the unweighted mean
  int vs;                   // 0: val, diag, invdiag shared by all columns; else per-column
                            // operators: entry (k, i) of column c at (k*ld + i) * vs + c, and
                            // diag / invdiag of row i at i * vs + c
  const int* vmap;          // per-column operators with a compacted cycle: the operator column
                            // of vector column b is vmap[b] (null: b)
};

// operator column of vector column b (per-column operators)
template <class C>
__device__ __forceinline__ int vcol(const Lvl<C>& L, int b) {
  return L.vmap ? L.vmap[b] : b;
}

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

// Values that are the same in every lane of a wavefront: WIDE kernels (64
// lanes per row, B >= 64) broadcast them from the first lane so the compiler
// keeps them in scalar registers and loads their operands with scalar loads.
template <bool W> __device__ __forceinline__ int uni(int v) { return W ? __builtin_amdgcn_readfirstlane(v) : v; }
template <bool W> __device__ __forceinline__ float uni(float v) {
  return W ? __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))) : v;
}
template <bool W> __device__ __forceinline__ double uni(double v) {
  if (!W) return v;
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row tiles: a block of 256 work-items covers ROWS * (256 >> lbs) rows.
//  - WIDE (lbs == 6): wavefront g handles the ROWS consecutive rows
//    base + g * ROWS + r; rows are wave-uniform.
//  - otherwise the work-items of row group g handle rows base + r * (256 >> lbs) + g,
//    so the lane groups of a wavefront cover consecutive rows (coalesced).
// All index loads of a tile are issued before its value loads, so every
// wavefront keeps ROWS * 4 independent loads in flight per phase.  Rows past
// the end are clamped to n - 1 for loads and skipped for stores.
template <int ROWS, bool WIDE>
struct Tile {
  int lane, LB;
  int row0;                 // WIDE: first of the ROWS consecutive rows (a multiple of ROWS)
  bool any;                 // WIDE: row0 < n
  int row[ROWS];
  bool ok[ROWS];
  __device__ __forceinline__ Tile(int n, int lbs) {
    LB = 1 << lbs;
    lane = threadIdx.x & (LB - 1);
    const int rpb = 256 >> lbs;
    const int g = uni<WIDE>((int)(threadIdx.x >> lbs));
    const long base = (long)xcd_block() * rpb * ROWS;
    row0 = (int)(base + (long)g * ROWS);
    any = row0 < n;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const long rr = WIDE ? base + (long)g * ROWS + r : base + (long)r * rpb + g;
      ok[r] = rr < n;
      row[r] = ok[r] ? (int)rr : n - 1;
    }
  }
};

// Four consecutive entries p[0..3] (p 16-byte aligned for 4-byte types).
template <class T> struct V4 { T v[4]; };
__device__ __forceinline__ V4<int> ld4(const int* p) {
  const int4 t = *reinterpret_cast<const int4*>(p);
  return V4<int>{{t.x, t.y, t.z, t.w}};
}
__device__ __forceinline__ V4<float> ld4(const float* p) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  return V4<float>{{t.x, t.y, t.z, t.w}};
}
__device__ __forceinline__ V4<double> ld4(const double* p) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  return V4<double>{{a.x, a.y, b.x, b.y}};
}

// s[r] += sum_k val(k, row_r) * x[col(k, row_r)] over W slots (W multiple of 4).
// CONSEC (WIDE, NR == 4): the rows are row0 .. row0 + 3 and each slot's four
// indices and values are one scalar 16-byte load.
template <bool WIDE, bool CONSEC, int NR, class C, class TX>
__device__ __forceinline__ void ell_dot(int W, int ld, const int* __restrict__ col, const C* __restrict__ val,
                                        const int (&row)[NR], int row0, const TX* __restrict__ x, int B, int b,
                                        C (&s)[NR]) {
  for (int k = 0; k < W; k += 4) {
    int j[NR][4];
    C v[NR][4];
    if constexpr (CONSEC && NR == 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const V4<int> jj = ld4(col + (size_t)(k + q) * ld + row0);
        const V4<C> vv = ld4(val + (size_t)(k + q) * ld + row0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          j[r][q] = uni<WIDE>(jj.v[r]);
          v[r][q] = uni<WIDE>(vv.v[r]);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const size_t o = (size_t)(k + q) * ld + row[r];
          j[r][q] = uni<WIDE>(col[o]);
          v[r][q] = uni<WIDE>(val[o]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) s[r] += v[r][q] * ldc<C>(x + (size_t)j[r][q] * B + b);
  }
}

// ell_dot with per-column operator values (Lvl::vs): the values of operator
// column vb; indices as in ell_dot, same sums in the same order
template <bool WIDE, int NR, class C, class TX>
__device__ __forceinline__ void ell_dot_v(int W, int ld, int vs, int vb, const int* __restrict__ col,
                                          const C* __restrict__ val, const int (&row)[NR],
                                          const TX* __restrict__ x, int B, int b, C (&s)[NR]) {
  for (int k = 0; k < W; k += 4) {
    int j[NR][4];
    C v[NR][4];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t o = (size_t)(k + q) * ld + row[r];
        j[r][q] = uni<WIDE>(col[o]);
        v[r][q] = val[o * vs + vb];
      }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) s[r] += v[r][q] * ldc<C>(x + (size_t)j[r][q] * B + b);
  }
}

// As ell_dot on the iterate v = u + e of one column (u: that column's entries
// at stride su, e: at stride se), each neighbour's sum formed in FP64 as it is
// read (the FP64 outer residual of the solver's fused update).
template <bool WIDE, bool CONSEC, int NR, class TE>
__device__ __forceinline__ void ell_dot_upd(int W, int ld, const int* __restrict__ col,
                                            const double* __restrict__ val, const int (&row)[NR], int row0,
                                            const double* __restrict__ u, int su, const TE* __restrict__ e, int se,
                                            double (&s)[NR], int vs = 0, int vb = 0) {
  for (int k = 0; k < W; k += 4) {
    int j[NR][4];
    double v[NR][4];
    if (vs) {   // per-column operator values
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const size_t o = (size_t)(k + q) * ld + row[r];
          j[r][q] = uni<WIDE>(col[o]);
          v[r][q] = val[o * vs + vb];
        }
    } else if constexpr (CONSEC && NR == 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const V4<int> jj = ld4(col + (size_t)(k + q) * ld + row0);
        const V4<double> vv = ld4(val + (size_t)(k + q) * ld + row0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          j[r][q] = uni<WIDE>(jj.v[r]);
          v[r][q] = uni<WIDE>(vv.v[r]);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const size_t o = (size_t)(k + q) * ld + row[r];
          j[r][q] = uni<WIDE>(col[o]);
          v[r][q] = uni<WIDE>(val[o]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        s[r] += v[r][q] * (u[(size_t)j[r][q] * su] + (double)e[(size_t)j[r][q] * se]);
  }
}

// Neighbour sums over the graph (W multiple of 4, padding col == row):
//   TRANS = false: s[r] += sum_{j in N(row)} [w_{row,j}] y_j         ((G y) = r_row * s)
//   TRANS = true:  s[r] += sum_{j in N(row)} [w_{row,j}] r_j y_j     ((G^T y) = s, symmetric
//                                                                       pattern and weights)
// with r the row scale (Lvl::invdeg) and the edge weights w (Lvl::gval) when
// WG.  The padding test uses the unclamped row (row0 + r under CONSEC).
template <bool WIDE, bool CONSEC, int NR, bool TRANS, bool WG, class C, class TY>
__device__ __forceinline__ void graph_sum(const Lvl<C>& L, const int (&row)[NR], int row0, const TY* __restrict__ y,
                                          int B, int b, C (&s)[NR]) {
#pragma clang fp contract(off)
  for (int k = 0; k < L.wg; k += 4) {
    int j[NR][4];
    C ew[NR][4];
    if constexpr (CONSEC && NR == 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const V4<int> jj = ld4(L.gcol + (size_t)(k + q) * L.ld + row0);
#pragma unroll
        for (int r = 0; r < 4; ++r) j[r][q] = uni<WIDE>(jj.v[r]);
        if constexpr (WG) {
          const V4<C> ww = ld4(L.gval + (size_t)(k + q) * L.ld + row0);
#pragma unroll
          for (int r = 0; r < 4; ++r) ew[r][q] = uni<WIDE>(ww.v[r]);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          j[r][q] = uni<WIDE>(L.gcol[(size_t)(k + q) * L.ld + row[r]]);
          if constexpr (WG) ew[r][q] = uni<WIDE>(L.gval[(size_t)(k + q) * L.ld + row[r]]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int self = (CONSEC && NR == 4) ? row0 + r : row[r];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        C v = ldc<C>(y + (size_t)j[r][q] * B + b);
        if (TRANS) v *= uni<WIDE>(L.invdeg[j[r][q]]);
        if constexpr (WG) v *= ew[r][q];
        s[r] += (j[r][q] != self) ? v : C(0);
      }
    }
  }
}

// per-row scalar p[row_r] for the rows of a tile (one 16-byte load under CONSEC)
template <bool WIDE, bool CONSEC, int NR, class C>
__device__ __forceinline__ void row_vals(const C* __restrict__ p, const int (&row)[NR], int row0, C (&out)[NR]) {
  if constexpr (CONSEC && NR == 4) {
    const V4<C> t = ld4(p + row0);
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = uni<WIDE>(t.v[r]);
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r] = uni<WIDE>(p[row[r]]);
  }
}

// out = [invdiag *] (f - A u); uz: u is identically zero.
// FINE only tags finest-level launches with their own kernel symbol (for
// per-level profiles); the code is the same.
// PCV: per-column operators (Lvl::vs), the diagonal and values of each column's own operator.
template <int ROWS, bool WIDE, bool FINE, bool PCV, class C, class TU, class TO>
__global__ __launch_bounds__(256) void k_resid(Lvl<C> L, int B, int lbs, const TU* __restrict__ f,
                                               const TU* __restrict__ u, int uz, int jacobi,
                                               TO* __restrict__ out) {
  constexpr bool CS = WIDE && ROWS == 4 && !PCV;
  const Tile<ROWS, WIDE> t(L.n, lbs);
  if (WIDE && !t.any) return;
  C dinv[ROWS];
  if (!PCV && jacobi) row_vals<WIDE, CS>(L.invdiag, t.row, t.row0, dinv);
  if (uz) {
    for (int b = t.lane; b < B; b += t.LB) {
      const int vb = PCV ? vcol(L, b) : 0;
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (!t.ok[r]) continue;
        C v = ldc<C>(f + (size_t)t.row[r] * B + b);
        if (jacobi) v *= PCV ? L.invdiag[(size_t)t.row[r] * L.vs + vb] : dinv[r];
        put(out + (size_t)t.row[r] * B + b, v);
      }
    }
    return;
  }
  C dg[ROWS];
  if (!PCV) row_vals<WIDE, CS>(L.diag, t.row, t.row0, dg);
  for (int b = t.lane; b < B; b += t.LB) {
    // the row's own f and u are loaded first but consumed only at the end, so
    // their loads overlap the index loads and the off-diagonal gathers
    C fv[ROWS], uv[ROWS], s[ROWS];
    const int vb = PCV ? vcol(L, b) : 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      fv[r] = ldc<C>(f + (size_t)t.row[r] * B + b);
      uv[r] = ldc<C>(u + (size_t)t.row[r] * B + b);
      s[r] = C(0);
      if constexpr (PCV) {
        dg[r] = L.diag[(size_t)t.row[r] * L.vs + vb];
        if (jacobi) dinv[r] = L.invdiag[(size_t)t.row[r] * L.vs + vb];
      }
    }
    if constexpr (PCV) ell_dot_v<WIDE>(L.w, L.ld, L.vs, vb, L.col, L.val, t.row, u, B, b, s);
    else ell_dot<WIDE, CS>(L.w, L.ld, L.col, L.val, t.row, t.row0, u, B, b, s);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (!t.ok[r]) continue;
      C v = fv[r] - (s[r] + dg[r] * uv[r]);
      if (jacobi) v *= dinv[r];
      put(out + (size_t)t.row[r] * B + b, v);
    }
  }
}

// Arithmetic of one Horner hop at one node and column, with the roundings
// fixed (no contraction left to the compiler), so that the per-hop sweeps
// and the fused tile kernel give the same bits:
//   hop_value:  v = fma(c, x, a * (r * s))     (s the neighbour sum, r the row scale)
//   hop_value1: the same with a == 1 (a * t == t exactly, so the product is skipped)
//   hop_update: u + scale * v = fma(scale, v, u)
__device__ __forceinline__ float hop_value(float a, float r, float s, float c, float x) {
  return __builtin_fmaf(c, x, __fmul_rn(a, __fmul_rn(r, s)));
}
__device__ __forceinline__ double hop_value(double a, double r, double s, double c, double x) {
  return __builtin_fma(c, x, __dmul_rn(a, __dmul_rn(r, s)));
}
__device__ __forceinline__ float hop_value1(float r, float s, float c, float x) {
  return __builtin_fmaf(c, x, __fmul_rn(r, s));
}
__device__ __forceinline__ float hop_update(float u, float scale, float v) { return __builtin_fmaf(scale, v, u); }
__device__ __forceinline__ double hop_update(double u, double scale, double v) { return __builtin_fma(scale, v, u); }

// Horner hop v = a * (M yin)_i + c * x_i.
//   mode 0: out = v (type TO)
//   mode 1: out = (oz ? 0 : out) + scale * v
template <int ROWS, bool WIDE, bool FINE, bool WG, class C, class TY, class TX, class TO>
__global__ __launch_bounds__(256) void k_hop(Lvl<C> L, int B, int lbs, const TY* __restrict__ yin, C a,
                                             const TX* __restrict__ x, C c, TO* __restrict__ out, int mode, C scale,
                                             int oz) {
  constexpr bool CS = WIDE && ROWS == 4;
  const Tile<ROWS, WIDE> t(L.n, lbs);
  if (WIDE && !t.any) return;
  C idg[ROWS];
  row_vals<WIDE, CS>(L.invdeg, t.row, t.row0, idg);
  for (int b = t.lane; b < B; b += t.LB) {
    C xv[ROWS], ov[ROWS], s[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const size_t o = (size_t)t.row[r] * B + b;
      xv[r] = ldc<C>(x + o);
      ov[r] = (mode == 1 && !oz) ? ldc<C>(out + o) : C(0);
      s[r] = C(0);
    }
    graph_sum<WIDE, CS, ROWS, false, WG>(L, t.row, t.row0, yin, B, b, s);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (!t.ok[r]) continue;
      const C v = hop_value(a, idg[r], s[r], c, xv[r]);
      put(out + (size_t)t.row[r] * B + b, mode == 0 ? v : hop_update(ov[r], scale, v));
    }
  }
}

// ---------------------------------------------------------------- fused K-hop convolution over tiles
// One workgroup computes all K Horner hops of Phi(x) = sum_k c_k M^k x for
// the own nodes of a tile and kTileCols of the B columns, with the input on
// the tile's K-hop neighbourhood and the intermediate hops in LDS (node
// lists and local graph columns are built on the host).  Per launch the
// input is read once (halo rows mostly from the L2) and the output written
// once; a chain of K separate hops moves about 3K vectors.
//
// The kernel is persistent: each XCD takes a contiguous range of the
// (tile, column group) items and its workgroups walk that range with a
// stride, so neighbouring tiles (whose halos overlap) are processed close in
// time on one L2.  Loads are software-pipelined in registers: while the
// hops of one item run out of LDS, the input rows, outputs, local columns
// and row scales of the next item and the node ids of the one after are in
// flight.
#ifndef MGL_TILE_THREADS
#define MGL_TILE_THREADS 512
#endif
#ifndef MGL_TILE_ROWS
#define MGL_TILE_ROWS 4
#endif
#ifndef MGL_TILE_OWN_PER_THREAD
#define MGL_TILE_OWN_PER_THREAD 2
#endif
#ifndef MGL_TILE_COLS
#define MGL_TILE_COLS 16
#endif
constexpr int kTileMaxK = 8;
constexpr int kTileCols = MGL_TILE_COLS;  // columns per item (4 per work-item)
constexpr int kTileQ = kTileCols / 4;     // work-items (float4 slots) per node
constexpr int kTileThreads = MGL_TILE_THREADS;
constexpr int kTileNp = kTileThreads / kTileQ;             // nodes per pass
constexpr int kTileRows = MGL_TILE_ROWS;                   // input rows per item <= kTileRows * kTileNp
constexpr int kTileOwnPerThread = MGL_TILE_OWN_PER_THREAD; // own rows per item <= this * kTileNp
constexpr int kTileMeta = 2;   // column chunks (4 slots) and row scales per item <= kTileMeta * kTileThreads

struct TileDev {
  int ntiles;
  int KM;                   // halo depth of the node lists
  int wg;                   // graph ELL width (multiple of 4)
  int ngroups;              // B / kTileCols
  const int* toff;          // ntiles + 1
  const int* node;          // per tile: own nodes, then by distance
  const int* cnt;           // ntiles x (KM + 1): nodes at distance <= d
  const int* goff;          // ntiles + 1; goff / wg indexes the per-row arrays below
  const uint16_t* lcol;     // local graph columns of the rows at distance <= KM - 1: (index + 1) x the
                            // LDS row size in bytes (0: padding, the row of zeros)
  const float* lidg;        // row scale of the aggregation (invdeg) of those rows
  const float* lgw;         // edge weights in their slots (weighted / symmetric aggregation), or null
};
struct TileCoef {
  float c[kTileMaxK + 1];
};
// LDS layout of one workgroup, in float4 units
struct TileLds {
  int xs;                   // input rows
  int y0, y1;               // hop buffers (each of the three preceded by a row of zeros)
  int col;                  // local columns of the rows at distance <= K - 1 as byte offsets (uint16)
  int idg;                  // their row scales (float)
};

__device__ __forceinline__ void ld4v(const float* p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4v(const bf16_t* p, float (&v)[4]) {
  const uint2 t = *reinterpret_cast<const uint2*>(p);
  v[0] = __uint_as_float(t.x << 16); v[1] = __uint_as_float(t.x & 0xffff0000u);
  v[2] = __uint_as_float(t.y << 16); v[3] = __uint_as_float(t.y & 0xffff0000u);
}
__device__ __forceinline__ void st4v(float* p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4v(bf16_t* p, const float (&v)[4]) {
  uint2 t;
  t.x = (uint32_t)f2bf(v[0]).bits | ((uint32_t)f2bf(v[1]).bits << 16);
  t.y = (uint32_t)f2bf(v[2]).bits | ((uint32_t)f2bf(v[3]).bits << 16);
  *reinterpret_cast<uint2*>(p) = t;
}

// A read of memory that no kernel of the launch writes (the tile metadata),
// through the constant address space: wave-uniform addresses become scalar
// loads, which are waited on apart from the vector loads in flight (those
// complete in order, so any wait on a vector load would also wait for every
// prefetch issued before it).
__device__ __forceinline__ int ld_const(const int* p) {
  return *(const __attribute__((address_space(4))) int*)p;
}

// s += sum over the graph slots of a local row of [w] y_j; columns from LDS as
// byte offsets ((local index + 1) x row size) from y0, the row of zeros before
// the LDS buffer, weights (WG) from the tile's slot array in global memory.  A
// padding slot (offset 0) reads that zero row and adds +0, as the per-hop sweep
// adds +0 for it (same sums, same order, no selection); weighted terms are
// rounded before they are added (no fused multiply-add).
template <bool WG>
__device__ __forceinline__ void tile_gather(int wg, const uint16_t* lc, const float* __restrict__ gw,
                                            const float4* y0, int q, float (&s)[4]) {
#pragma clang fp contract(off)
  const char* yb = reinterpret_cast<const char*>(y0 + q);
  for (int k = 0; k < wg; k += 4) {
    const ushort4 jj = *reinterpret_cast<const ushort4*>(lc + k);
    const int j[4] = {jj.x, jj.y, jj.z, jj.w};
    float ew[4];
    if constexpr (WG) {
      const float4 w4 = *reinterpret_cast<const float4*>(gw + k);
      ew[0] = w4.x; ew[1] = w4.y; ew[2] = w4.z; ew[3] = w4.w;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float4 t = *reinterpret_cast<const float4*>(yb + j[e]);
      float v[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (WG) v[c] *= ew[e];
        s[c] += v[c];
      }
    }
  }
}

// Item scalars and node ids (fetched two items ahead)
struct TileHead {
  int t, g, cK, rows1, own, base, m0;
  int nd[kTileRows];
};
// Item data in registers (fetched one item ahead)
struct TileBody {
  float xv[kTileRows][4];
  float xs[kTileRows];      // row scales of the input (xsc)
  float ov[kTileOwnPerThread][4];
  uint2 lc[kTileMeta];
  float li[kTileMeta];
};

//   mode 0: out = Phi(x)      mode 1: out = (oz ? 0 : out) + scale * Phi(x)
// With xsc the input is x_i xsc_i (the Jacobi-scaled residual of a zero iterate,
// f_i / a_ii, formed as the rows enter LDS: one sweep less per cycle level).
// Arithmetic per node and column as in k_hop (same order of the sums).
// Grid: a multiple of 8 blocks of kTileThreads; out must not alias x.  FINE
// only tags finest-level launches with their own symbol (same code).
template <bool FINE, bool WG, class TX, class TO>
__global__ __launch_bounds__(kTileThreads) void k_conv_tile(TileDev T, int B, int K, TileCoef cf,
                                                           const TX* __restrict__ x, TO* __restrict__ out, int mode,
                                                           float scale, int oz, TileLds lo,
                                                           const float* __restrict__ xsc) {
  extern __shared__ __align__(16) float4 conv_smem[];
  const int per = gridDim.x >> 3;             // workgroups per XCD
  const int xc = blockIdx.x & 7;              // blocks are dispatched round-robin over the XCDs
  const int W = T.ntiles * T.ngroups;
  const int i1 = (int)((long long)W * (xc + 1) / 8);
  int it = (int)((long long)W * xc / 8) + (blockIdx.x >> 3);
  if (it >= i1) return;
  const int q = threadIdx.x % kTileQ;
  const int p0 = threadIdx.x / kTileQ;
  const int KM = T.KM, wg = T.wg;
  float4* S = conv_smem + lo.xs;
  // the rows of zeros before the three buffers (never written again; the
  // first barrier below orders them before any read)
  for (int z = threadIdx.x; z < 3 * kTileQ; z += blockDim.x) {
    const int base = z < kTileQ ? lo.xs : (z < 2 * kTileQ ? lo.y0 : lo.y1);
    conv_smem[base - kTileQ + z % kTileQ] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  uint2* LC2 = reinterpret_cast<uint2*>(conv_smem + lo.col);
  const uint16_t* LC = reinterpret_cast<const uint16_t*>(conv_smem + lo.col);
  float* LI = reinterpret_cast<float*>(conv_smem + lo.idg);
  const bool rd_out = mode == 1 && !oz;

  auto head = [&](int i, TileHead& h) {
    h.t = i / T.ngroups;
    h.g = i - h.t * T.ngroups;
    const int* cn = T.cnt + (size_t)h.t * (KM + 1);
    h.cK = ld_const(cn + K);
    h.rows1 = ld_const(cn + K - 1);
    h.own = ld_const(cn);
    h.base = ld_const(T.toff + h.t);
    h.m0 = ld_const(T.goff + h.t);
#pragma unroll
    for (int e = 0; e < kTileRows; ++e) h.nd[e] = T.node[h.base + min(p0 + e * kTileNp, h.cK - 1)];
  };
  auto body = [&](const TileHead& h, TileBody& b) {
    const int col = h.g * kTileCols + q * 4;
#pragma unroll
    for (int e = 0; e < kTileRows; ++e) {
      ld4v(x + (size_t)h.nd[e] * B + col, b.xv[e]);
      if (xsc) b.xs[e] = xsc[h.nd[e]];
    }
#pragma unroll
    for (int e = 0; e < kTileOwnPerThread; ++e) {
#pragma unroll
      for (int c = 0; c < 4; ++c) b.ov[e][c] = 0.f;
      if (rd_out && p0 + e * kTileNp < h.own) ld4v(out + (size_t)h.nd[e] * B + col, b.ov[e]);
    }
    const uint2* src = reinterpret_cast<const uint2*>(T.lcol + h.m0);
    const float* ls = T.lidg + h.m0 / wg;
    const int nch = h.rows1 * wg / 4;
#pragma unroll
    for (int e = 0; e < kTileMeta; ++e) {
      const int c = threadIdx.x + e * kTileThreads;
      if (c < nch) b.lc[e] = src[c];
      if (c < h.rows1) b.li[e] = ls[c];
    }
  };

  TileHead hc, hn;
  TileBody bc;
  head(it, hc);
  body(hc, bc);
  int itn = it + per;
  if (itn < i1) head(itn, hn);
  while (true) {
    // item `it` into LDS
#pragma unroll
    for (int e = 0; e < kTileRows; ++e) {
      const int r = p0 + e * kTileNp;
      if (xsc) {
#pragma unroll
        for (int c = 0; c < 4; ++c) bc.xv[e][c] *= bc.xs[e];
      }
      if (r < hc.cK) S[r * kTileQ + q] = make_float4(bc.xv[e][0], bc.xv[e][1], bc.xv[e][2], bc.xv[e][3]);
    }
    {
      const int nch = hc.rows1 * wg / 4;
#pragma unroll
      for (int e = 0; e < kTileMeta; ++e) {
        const int c = threadIdx.x + e * kTileThreads;
        if (c < nch) LC2[c] = bc.lc[e];
        if (c < hc.rows1) LI[c] = bc.li[e];
      }
    }
    const TileHead h = hc;
    float ov[kTileOwnPerThread][4];
#pragma unroll
    for (int e = 0; e < kTileOwnPerThread; ++e)
#pragma unroll
      for (int c = 0; c < 4; ++c) ov[e][c] = bc.ov[e][c];
    __syncthreads();
    // next item's data and the one after's node ids, in flight during the hops
    const bool more = itn < i1;
    if (more) {
      body(hn, bc);
      hc = hn;
    }
    const int itnn = itn + per;
    if (itnn < i1) head(itnn, hn);
    const int* cn = T.cnt + (size_t)h.t * (KM + 1);
    const float* gw = WG ? T.lgw + h.m0 : nullptr;
    // hops 1 .. K-1 on the nodes at distance <= K - hop; the first applies c_K, the
    // others continue Horner's rule with factor 1 (hop_value1, a == 1 exactly).
    // yin points at the row of zeros before the hop's input buffer.
    const float4* yin = S - kTileQ;
    auto hop_pass = [&](auto scaled, int hp) {
      const int rows = ld_const(cn + K - hp);
      const float cc = cf.c[K - hp];
      float4* yo = conv_smem + ((hp & 1) ? lo.y0 : lo.y1);
      for (int r = p0; r < rows; r += kTileNp) {
        float s[4] = {0.f, 0.f, 0.f, 0.f};
        tile_gather<WG>(wg, LC + r * wg, WG ? gw + (size_t)r * wg : nullptr, yin, q, s);
        const float idg = LI[r];
        const float4 xv = S[r * kTileQ + q];
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
        float o[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if constexpr (decltype(scaled)::value) o[c] = hop_value(cf.c[K], idg, s[c], cc, xs[c]);
          else o[c] = hop_value1(idg, s[c], cc, xs[c]);
        }
        yo[r * kTileQ + q] = make_float4(o[0], o[1], o[2], o[3]);
      }
      __syncthreads();
      yin = yo - kTileQ;
    };
    hop_pass(std::true_type{}, 1);
    for (int hp = 2; hp < K; ++hp) hop_pass(std::false_type{}, hp);
    // last hop on the own nodes, fused with the output update (factor 1: K >= 2)
    const float c0 = cf.c[0];
    const int col = h.g * kTileCols + q * 4;
#pragma unroll
    for (int e = 0; e < kTileOwnPerThread; ++e) {
      const int r = p0 + e * kTileNp;
      if (r < h.own) {
        float s[4] = {0.f, 0.f, 0.f, 0.f};
        tile_gather<WG>(wg, LC + r * wg, WG ? gw + (size_t)r * wg : nullptr, yin, q, s);
        const float idg = LI[r];
        const float4 xv = S[r * kTileQ + q];
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
        float v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float w = hop_value1(idg, s[c], c0, xs[c]);
          v[c] = mode == 0 ? w : hop_update(ov[e][c], scale, w);
        }
        st4v(out + (size_t)h.nd[e] * B + col, v);
      }
    }
    __syncthreads();
    if (!more) break;
    it = itn;
    itn = itnn;
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
// R's ELL width is a multiple of 4 (padding val == 0); the four fine rows of
// a slot chunk are processed together.
template <bool WIDE, bool WG, class C, class TU, class TY, class TX>
__global__ __launch_bounds__(256) void k_restrict(Xfer<C> R, Lvl<C> L, int B, int lbs, int mode,
                                                  const TY* __restrict__ y, C a, const TX* __restrict__ x,
                                                  C c, const TU* __restrict__ f, const TU* __restrict__ u,
                                                  int uz, C scale, TU* __restrict__ rc) {
  const long gt_ = (long)xcd_block() * blockDim.x + threadIdx.x;
  const int i = uni<WIDE>((int)(gt_ >> lbs));
  const int lane = (int)(gt_ & ((1 << lbs) - 1));
  if (i >= R.n) return;
  if (mode == 0 && R.w <= 8) {
    // plain restriction of y: every slot's index and weight, then every gather,
    // issued before the sums (one round trip each instead of one per chunk);
    // slots past R.w repeat slot 0's index and are not summed
    int jr[8];
    C wr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int kk = k < R.w ? k : 0;
      jr[k] = uni<WIDE>(R.col[(size_t)kk * R.n + i]);
      wr[k] = uni<WIDE>(R.val[(size_t)kk * R.n + i]);
    }
    for (int b = lane; b < B; b += (1 << lbs)) {
      C v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = ldc<C>(y + (size_t)jr[k] * B + b);
      C acc = C(0);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < R.w) acc += (wr[k] != C(0)) ? wr[k] * v[k] : C(0);
      put(rc + (size_t)i * B + b, scale * acc);
    }
    return;
  }
  for (int b = lane; b < B; b += (1 << lbs)) {
    C acc = C(0);
    for (int k = 0; k < R.w; k += 4) {
      int jr[4];
      C wr[4], v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        jr[q] = uni<WIDE>(R.col[(size_t)(k + q) * R.n + i]);
        wr[q] = uni<WIDE>(R.val[(size_t)(k + q) * R.n + i]);
      }
      if (mode == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = ldc<C>(y + (size_t)jr[q] * B + b);
      } else if (mode == 1) {
        C sm[4] = {C(0), C(0), C(0), C(0)}, xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[q] = ldc<C>(x + (size_t)jr[q] * B + b);
        graph_sum<WIDE, false, 4, false, WG>(L, jr, 0, y, B, b, sm);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = hop_value(a, uni<WIDE>(L.invdeg[jr[q]]), sm[q], c, xv[q]);
      } else {
        C fv[4], sa[4];
        const int vb = L.vs ? vcol(L, b) : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          fv[q] = ldc<C>(f + (size_t)jr[q] * B + b);
          const C dq = L.vs ? L.diag[(size_t)jr[q] * L.vs + vb] : uni<WIDE>(L.diag[jr[q]]);
          sa[q] = uz ? C(0) : dq * ldc<C>(u + (size_t)jr[q] * B + b);
        }
        if (!uz) {
          if (L.vs) ell_dot_v<WIDE>(L.w, L.ld, L.vs, vb, L.col, L.val, jr, u, B, b, sa);
          else ell_dot<WIDE, false>(L.w, L.ld, L.col, L.val, jr, 0, u, B, b, sa);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = fv[q] - sa[q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc += (wr[q] != C(0)) ? wr[q] * v[q] : C(0);
    }
    put(rc + (size_t)i * B + b, scale * acc);
  }
}

// Prolongation (or any ELL transfer applied to a coarse vector); even width:
//   mode 0: out = scale * (P ec)     mode 1: out = (oz ? 0 : out) + scale * (P ec)
template <int ROWS, bool WIDE, class C, class TU, class TO>
__global__ __launch_bounds__(256) void k_prolong(Xfer<C> P, int B, int lbs, const TU* __restrict__ ec,
                                                 TO* __restrict__ out, int mode, C scale, int oz) {
  const Tile<ROWS, WIDE> t(P.n, lbs);
  for (int b = t.lane; b < B; b += t.LB) {
    C acc[ROWS], ov[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      acc[r] = C(0);
      ov[r] = (mode == 1 && !oz) ? ldc<C>(out + (size_t)t.row[r] * B + b) : C(0);
    }
    for (int k = 0; k < P.w; k += 2) {
      int j[ROWS][2];
      C w[ROWS][2];
#pragma unroll
      for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const size_t o = (size_t)(k + q) * P.n + t.row[r];
          j[r][q] = uni<WIDE>(P.col[o]);
          w[r][q] = uni<WIDE>(P.val[o]);
        }
      // every gather of the chunk issued before the sums use them
      C v[ROWS][2];
#pragma unroll
      for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) v[r][q] = ldc<C>(ec + (size_t)j[r][q] * B + b);
#pragma unroll
      for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[r] += w[r][q] * v[r][q];
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (!t.ok[r]) continue;
      put(out + (size_t)t.row[r] * B + b, mode == 0 ? scale * acc[r] : ov[r] + scale * acc[r]);
    }
  }
}

// Coarsest level: u = Ainv f (or Ainv^T f), Ainv dense row-major FP64.
template <class TU>
__global__ __launch_bounds__(256) void k_coarse(int n, int B, const double* __restrict__ Ainv,
                                                const TU* __restrict__ f, TU* __restrict__ u, int trans,
                                                int pcv, const int* __restrict__ vmap) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * B) return;
  const int i = (int)(t / B), b = (int)(t % B);
  // per-column operators: column b's own inverse
  if (pcv) Ainv += (size_t)(vmap ? vmap[b] : b) * n * n;
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
// Block b (XCD-remapped) owns the contiguous rows [b*chunk, (b+1)*chunk) and
// walks them four rows per work-item at a time, so neighbour rows are reused
// from L2; the summation order is fixed (deterministic).  B <= 256.
//
// UPD (the solver's update fused into the next residual): the iterate is
// v = u + e in the columns with act[b] != 0 and v = u in the others, formed on
// the fly for the row and its neighbours (the same FP64 sum for every
// reader, so the same bits as storing it first); v is written to uo (which
// must not alias u: neighbours still read u) and the residual is f - A v.
template <bool WIDE, bool UPD, bool PCV, class TR, class TE>
__global__ __launch_bounds__(256) void k_outer_resid(Lvl<double> L, int B, int lbs, int chunk,
                                                     const double* __restrict__ f, const double* __restrict__ u,
                                                     double* __restrict__ r64, TR* __restrict__ rc,
                                                     double* __restrict__ part, const TE* __restrict__ e,
                                                     const int* __restrict__ act, double* __restrict__ uo, int Bc,
                                                     const int* __restrict__ cmap) {
  __shared__ double red[256 * 4];
  const int LB = 1 << lbs, rpb = 256 >> lbs;
  const int lane = threadIdx.x & (LB - 1), rg = uni<WIDE>((int)(threadIdx.x >> lbs));
  const int blk = xcd_block();
  const long lo = (long)blk * chunk, hi = lo + chunk < L.n ? lo + chunk : L.n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i0 = lo + (long)rg * 4; i0 < hi; i0 += 4L * rpb) {
    int row[4];
    bool ok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long rr = i0 + r;
      ok[r] = rr < hi;
      row[r] = ok[r] ? (int)rr : (int)(hi - 1);
    }
    // WIDE: the four rows are i0 .. i0+3 (i0 a multiple of 4, rows past the
    // chunk computed but not stored), so each slot's indices and values and
    // the diagonal are one 16-byte scalar load per row quadruple
    const int r0 = uni<WIDE>((int)i0);
    double dg[4];
    if (!PCV) row_vals<WIDE, WIDE>(L.diag, row, r0, dg);
    int q = 0;
    for (int b = lane; b < B; b += LB, ++q) {
      // UPD: a stopped column is not touched (its iterate stays where it was last written)
      if (UPD && act[b] == 0) continue;
      // the cycle-type vectors (rc, e) may hold only the columns still iterating: column b
      // at slot cmap[b] of Bc
      const int sb = cmap ? cmap[b] : b;
      // own f and u loaded first, consumed after the off-diagonal gathers
      double fv[4], uv[4], s[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        fv[r] = f[(size_t)row[r] * B + b];
        uv[r] = u[(size_t)row[r] * B + b];
        if constexpr (UPD) uv[r] += (double)e[(size_t)row[r] * Bc + sb];
        if constexpr (PCV) dg[r] = L.diag[(size_t)row[r] * L.vs + b];
        s[r] = 0.0;
      }
      if constexpr (UPD)
        ell_dot_upd<WIDE, WIDE && !PCV>(L.w, L.ld, L.col, L.val, row, r0, u + b, B, e + sb, Bc, s, PCV ? L.vs : 0, b);
      else if constexpr (PCV) ell_dot_v<WIDE>(L.w, L.ld, L.vs, b, L.col, L.val, row, u, B, b, s);
      else ell_dot<WIDE, WIDE>(L.w, L.ld, L.col, L.val, row, r0, u, B, b, s);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!ok[r]) continue;
        const size_t o = (size_t)row[r] * B + b;
        const double v = fv[r] - (s[r] + dg[r] * uv[r]);
        if constexpr (UPD) uo[o] = uv[r];
        if (r64) r64[o] = v;
        if (rc) put(rc + (size_t)row[r] * Bc + sb, v);
        acc[q] += v * v;
      }
    }
  }
  for (int q = 0; q < 4; ++q) red[q * 256 + threadIdx.x] = acc[q];
  __syncthreads();
  if (threadIdx.x < LB) {
    int q = 0;
    for (int b = lane; b < B; b += LB, ++q) {
      double s = 0.0;
      for (int g = 0; g < rpb; ++g) s += red[q * 256 + g * LB + lane];
      part[(size_t)blk * B + b] = s;
    }
  }
}

// norms[b] = sqrt(sum over blocks of part[block][b]); one block per column,
// fixed strided order and fixed tree (deterministic).
__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ part, int nblk, int B,
                                                    double* __restrict__ norms, const int* __restrict__ act) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  if (act && act[b] == 0) return;   // a stopped column keeps its last norm
  double s = 0.0;
  for (int g = threadIdx.x; g < nblk; g += 256) s += part[(size_t)g * B + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[b] = sqrt(red[0]);
}

// ------------------------------------------------------------------ residual loss (Alg. 3)
// Per-block, per-column partial sums of x^2 over the outer residual's row
// chunks (block b owns rows [b*chunk, (b+1)*chunk)), fixed order.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_colsq(int n, int B, int lbs, int chunk, const double* __restrict__ x,
                                               double* __restrict__ part) {
  __shared__ double red[256 * 4];
  const int LB = 1 << lbs, rpb = 256 >> lbs;
  const int lane = threadIdx.x & (LB - 1), rg = uni<WIDE>((int)(threadIdx.x >> lbs));
  const int blk = xcd_block();
  const long lo = (long)blk * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i0 = lo + (long)rg * 4; i0 < hi; i0 += 4L * rpb) {
    int q = 0;
    for (int b = lane; b < B; b += LB, ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (i0 + r < hi) {
          const double v = x[(size_t)(i0 + r) * B + b];
          acc[q] += v * v;
        }
  }
  for (int q = 0; q < 4; ++q) red[q * 256 + threadIdx.x] = acc[q];
  __syncthreads();
  if (threadIdx.x < LB) {
    int q = 0;
    for (int b = lane; b < B; b += LB, ++q) {
      double s = 0.0;
      for (int g = 0; g < rpb; ++g) s += red[q * 256 + g * LB + lane];
      part[(size_t)blk * B + b] = s;
    }
  }
}

// Loss and per-column gradient coefficients from the column norms rn = ||r_b||,
// fn = ||f_b|| (one block of 256 work-items, B <= 256, fixed summation tree):
//   kind 0: L = (1/B) sum_b rn_b^2 / fn_b^2,  alpha_b = 2 g / (B fn_b^2),
//           beta_b = 2 g rn_b^2 / (B fn_b^4); a column with fn_b = 0 adds 0
//           and gets alpha_b = beta_b = 0
//   kind 1: L = sum_b rn_b,  alpha_b = g / rn_b (0 when rn_b = 0),  beta_b = 0
// so that dL/du_b = -alpha_b A^T r_b and dL/df_b = alpha_b r_b - beta_b f_b,
// scaled by the incoming cotangent g = *gseed (1 when gseed is null).
__global__ __launch_bounds__(256) void k_loss_coef(const double* __restrict__ rn, const double* __restrict__ fn,
                                                   int B, int kind, const double* __restrict__ gseed,
                                                   double* __restrict__ alpha, double* __restrict__ beta,
                                                   double* __restrict__ loss) {
  __shared__ double red[256];
  const int b = threadIdx.x;
  const double g = gseed ? gseed[0] : 1.0;
  double term = 0.0;
  if (b < B) {
    const double r = rn[b], q = fn[b];
    double a = 0.0, c = 0.0;
    if (kind == 0) {
      if (q > 0.0) {
        const double q2 = q * q;
        term = r * r / q2;
        a = 2.0 * g / ((double)B * q2);
        c = a * term;
      }
    } else {
      term = r;
      a = r > 0.0 ? g / r : 0.0;
    }
    if (alpha) alpha[b] = a;
    if (beta) beta[b] = c;
  }
  red[threadIdx.x] = term;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = kind == 0 ? red[0] / (double)B : red[0];
}

// gu_b = -alpha_b (A r_b)  (A symmetric, so A^T r = A r),  gf_b = alpha_b r_b - beta_b f_b;
// either output may be null.
template <int ROWS, bool WIDE>
__global__ __launch_bounds__(256) void k_loss_grad(Lvl<double> L, int B, int lbs, const double* __restrict__ r,
                                                   const double* __restrict__ f, const double* __restrict__ alpha,
                                                   const double* __restrict__ beta, double* __restrict__ gu,
                                                   double* __restrict__ gf) {
  const Tile<ROWS, WIDE> t(L.n, lbs);
  if (WIDE && !t.any) return;
  for (int b = t.lane; b < B; b += t.LB) {
    const double a = alpha[b];
    double rv[ROWS], s[ROWS];
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
      rv[q] = r[(size_t)t.row[q] * B + b];
      s[q] = 0.0;
    }
    if (gu) ell_dot<WIDE, false>(L.w, L.ld, L.col, L.val, t.row, t.row0, r, B, b, s);
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
      if (!t.ok[q]) continue;
      const size_t o = (size_t)t.row[q] * B + b;
      if (gu) gu[o] = -a * (s[q] + uni<WIDE>(L.diag[t.row[q]]) * rv[q]);
      if (gf) gf[o] = a * rv[q] - beta[b] * f[o];
    }
  }
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

// dst[i][s] = src[i][from[s]] (0 where from[s] < 0): columns of an [n][Bo]
// array gathered into an [n][Bn] one (the solver's active-column compaction)
template <class T>
__global__ __launch_bounds__(256) void k_repack(int n, int Bo, int Bn, const int* __restrict__ from,
                                                const T* __restrict__ src, T* __restrict__ dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * Bn) return;
  const long i = t / Bn;
  const int c = (int)(t - i * Bn);
  const int k = from[c];
  dst[t] = k >= 0 ? src[i * Bo + k] : T(0);
}

// Column b of a level's per-column operator arrays from one column's FP64
// arrays (off: [w][ld] slot values, dg: [ld] diagonal): values, diagonal and
// inverse diagonal in the cycle type, and (val64 / diag64 non-null) the FP64
// copies of the finest level.  Rows [n, ld) are padding (inverse diagonal 0).
template <class C>
__global__ __launch_bounds__(256) void k_put_column(int w, int ld, int n, int nv, int b, const double* __restrict__ off,
                                                    const double* __restrict__ dg, C* val, C* diag, C* invdiag,
                                                    double* val64, double* diag64) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long)w * ld) {
    val[t * nv + b] = (C)off[t];
    if (val64) val64[t * nv + b] = off[t];
  }
  if (t < ld) {
    diag[t * nv + b] = (C)dg[t];
    invdiag[t * nv + b] = t < n ? (C)(1.0 / dg[t]) : C(0);
    if (diag64) diag64[t * nv + b] = dg[t];
  }
}

// u[i][b] = w[i][b] for the columns whose update count iters[b] is odd (the
// solver alternates the iterate between u and w, one buffer per update)
__global__ __launch_bounds__(256) void k_copy_odd(int n, int B, int lbs, const int* __restrict__ iters,
                                                  const double* __restrict__ w, double* __restrict__ u) {
  MGL_ROW_LANE(n)
  for (int b = lane; b < B; b += (1 << lbs))
    if (iters[b] & 1) u[(size_t)i * B + b] = w[(size_t)i * B + b];
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

// ------------------------------------------------------------------ coarse tail in LDS
// Levels lt .. J-1 of one V-cycle for CPB right-hand-side columns per
// workgroup, with every vector of those levels in LDS (the operators are read
// from global memory and stay in L2).  Columns are independent, so
// workgroups never synchronise with each other; inside a workgroup the sweeps
// are separated by barriers.  LDS layout (units of C, column-minor:
// element (i, c) of a vector at off + i * CPB + c): per tail level u and f,
// plus four scratch vectors of the largest tail level.
constexpr int kTailMaxLevels = 12;
template <class C>
struct TailLevel {
  Lvl<C> L;
  Xfer<C> P;                // n_l x n_{l+1} (levels below the coarsest)
  Xfer<C> R;                // n_{l+1} x n_l
  int off_u, off_f;
};
template <class C>
struct TailArgs {
  int nl;                   // number of tail levels (the last one is the coarsest)
  TailLevel<C> lv[kTailMaxLevels];
  int off_s, off_ya, off_yb, off_t;
  int KB, KR, KP, nu_pre, nu_post, per;
  const double* prm;        // flat parameters, row `per` per level, first tail level first
  const double* Ainv;       // coarsest inverse (row-major)
  int nJ;
  int lt;                   // global index of the first tail level
};

// The tail's operators stay in global memory (L2-resident) while its vectors
// live in LDS.  Rows of width 1 .. kTailW load all their slots' indices (and
// values) at once, so a sweep costs one global round trip rather than one per
// slot; slots past the width repeat slot 0 and are not summed (same sums, same
// order, as the slot loop).
constexpr int kTailW = 8;

// One work-item's row of a tail level, held in registers for the sweeps of a
// level visit when every row has its own work-item (n * CPB <= blockDim.x) and
// the widths are 1 .. kTailW: the sweeps then read only LDS.
template <class C, bool WG>
struct TRow {
  int ac[kTailW], gc[kTailW];
  C av[kTailW], gw[WG ? kTailW : 1];
  C dg, ida, idg;
};
template <int CPB, bool WG, class C>
__device__ __forceinline__ bool tl_cacheable(const Lvl<C>& L) {
  return L.n * CPB <= (int)blockDim.x && L.w >= 1 && L.w <= kTailW && L.wg >= 1 && L.wg <= kTailW;
}
template <int CPB, bool WG, class C>
__device__ __forceinline__ void tl_load_row(const Lvl<C>& L, TRow<C, WG>& R) {
  const int e = threadIdx.x;
  if (e >= L.n * CPB) return;
  const int i = e / CPB;
  // per-column operators (one column per workgroup): the operator column of this workgroup's column
  const int vs = L.vs, vb = vs ? vcol(L, (int)blockIdx.x) : 0;
#pragma unroll
  for (int k = 0; k < kTailW; ++k) {
    const size_t o = (size_t)(k < L.w ? k : 0) * L.ld + i;
    const size_t og = (size_t)(k < L.wg ? k : 0) * L.ld + i;
    R.ac[k] = L.col[o];
    R.av[k] = vs ? L.val[o * vs + vb] : L.val[o];
    R.gc[k] = L.gcol[og];
    if constexpr (WG) R.gw[k] = L.gval[og];
  }
  R.dg = vs ? L.diag[(size_t)i * vs + vb] : L.diag[i];
  R.ida = vs ? L.invdiag[(size_t)i * vs + vb] : L.invdiag[i];
  R.idg = L.invdeg[i];
}

template <int CPB, class C, bool WG>
__device__ __forceinline__ void tl_resid(const Lvl<C>& L, const C* f, const C* u, int uz, int jacobi, C* out,
                                         const TRow<C, WG>& rc, bool cached) {
  if (cached) {   // the row in registers (one row per work-item)
    const int e = threadIdx.x;
    if (e < L.n * CPB) {
      const int c = e % CPB;
      C v = f[e];
      if (!uz) {
        C au = rc.dg * u[e];
#pragma unroll
        for (int k = 0; k < kTailW; ++k)
          if (k < L.w) au += rc.av[k] * u[rc.ac[k] * CPB + c];
        v -= au;
      }
      if (jacobi) v *= rc.ida;
      out[e] = v;
    }
    __syncthreads();
    return;
  }
  // per-column operators (one column per workgroup, CPB == 1): value (o) of the workgroup's column
  const int vs = L.vs, vb = vs ? vcol(L, (int)blockIdx.x) : 0;
  auto vi = [&](size_t o) { return vs ? o * vs + vb : o; };
  for (int e = threadIdx.x; e < L.n * CPB; e += blockDim.x) {
    const int i = e / CPB, c = e - i * CPB;
    C v = f[e];
    if (!uz) {
      C au = L.diag[vi(i)] * u[e];
      if (L.w >= 1 && L.w <= kTailW) {
        int jj[kTailW];
        C vv[kTailW];
#pragma unroll
        for (int k = 0; k < kTailW; ++k) {
          const size_t o = (size_t)(k < L.w ? k : 0) * L.ld + i;
          jj[k] = L.col[o];
          vv[k] = L.val[vi(o)];
        }
#pragma unroll
        for (int k = 0; k < kTailW; ++k)
          if (k < L.w) au += vv[k] * u[jj[k] * CPB + c];
      } else {
        for (int k = 0; k < L.w; ++k)
          au += L.val[vi((size_t)k * L.ld + i)] * u[L.col[(size_t)k * L.ld + i] * CPB + c];
      }
      v -= au;
    }
    if (jacobi) v *= L.invdiag[vi(i)];
    out[e] = v;
  }
  __syncthreads();
}

// out = a (M yin) + c x   (mode 0)   |   out = (oz ? 0 : out) + scale (a (M yin) + c x)   (mode 1)
template <int CPB, bool WG, class C>
__device__ __forceinline__ void tl_hop(const Lvl<C>& L, const C* yin, C a, const C* x, C cc, C* out, int mode,
                                       C scale, int oz, const TRow<C, WG>& rc, bool cached) {
  if (cached) {   // the row in registers (one row per work-item)
    const int e = threadIdx.x;
    if (e < L.n * CPB) {
      const int i = e / CPB, c = e - i * CPB;
      C sm = C(0);
#pragma unroll
      for (int k = 0; k < kTailW; ++k) {
        if (k >= L.wg) continue;
        C v = yin[rc.gc[k] * CPB + c];
        if constexpr (WG) v *= rc.gw[k];
        if (rc.gc[k] != i) sm += v;
      }
      const C v = hop_value(a, rc.idg, sm, cc, x[e]);
      out[e] = mode == 0 ? v : hop_update(oz ? C(0) : out[e], scale, v);
    }
    __syncthreads();
    return;
  }
  for (int e = threadIdx.x; e < L.n * CPB; e += blockDim.x) {
    const int i = e / CPB, c = e - i * CPB;
    C sm = C(0);
    if (L.wg >= 1 && L.wg <= kTailW) {
      int jj[kTailW];
      C ww[kTailW];
#pragma unroll
      for (int k = 0; k < kTailW; ++k) {
        const size_t o = (size_t)(k < L.wg ? k : 0) * L.ld + i;
        jj[k] = L.gcol[o];
        if constexpr (WG) ww[k] = L.gval[o];
      }
#pragma unroll
      for (int k = 0; k < kTailW; ++k) {
        if (k >= L.wg) continue;
        C v = yin[jj[k] * CPB + c];
        if constexpr (WG) v *= ww[k];
        if (jj[k] != i) sm += v;
      }
    } else {
      for (int k = 0; k < L.wg; ++k) {
        const int j = L.gcol[(size_t)k * L.ld + i];
        C v = yin[j * CPB + c];
        if constexpr (WG) v *= L.gval[(size_t)k * L.ld + i];
        if (j != i) sm += v;
      }
    }
    const C v = hop_value(a, L.invdeg[i], sm, cc, x[e]);
    out[e] = mode == 0 ? v : hop_update(oz ? C(0) : out[e], scale, v);
  }
  __syncthreads();
}

// out = X v  for an ELL transfer X (rows X.n)
template <int CPB, class C>
__device__ __forceinline__ void tl_xfer(const Xfer<C>& X, const C* v, C* out, int add, C scale, int oz) {
  for (int e = threadIdx.x; e < X.n * CPB; e += blockDim.x) {
    const int i = e / CPB, c = e - i * CPB;
    C acc = C(0);
    if (X.w >= 1 && X.w <= kTailW) {
      int jj[kTailW];
      C ww[kTailW];
#pragma unroll
      for (int k = 0; k < kTailW; ++k) {
        const size_t o = (size_t)(k < X.w ? k : 0) * X.n + i;
        jj[k] = X.col[o];
        ww[k] = X.val[o];
      }
#pragma unroll
      for (int k = 0; k < kTailW; ++k)
        if (k < X.w && ww[k] != C(0)) acc += ww[k] * v[jj[k] * CPB + c];
    } else {
      for (int k = 0; k < X.w; ++k) {
        const C w = X.val[(size_t)k * X.n + i];
        if (w != C(0)) acc += w * v[X.col[(size_t)k * X.n + i] * CPB + c];
      }
    }
    out[e] = add ? (oz ? C(0) : out[e]) + scale * acc : scale * acc;
  }
  __syncthreads();
}

// u = (oz ? 0 : u) + scale * sum_k c_k M^k x  (Horner, as the per-level sweeps)
template <int CPB, bool WG, class C>
__device__ __forceinline__ void tl_conv_add(const Lvl<C>& L, const double* c, int K, const C* x, double scale, C* u,
                                            int oz, C* ya, C* yb, const TRow<C, WG>& rc, bool cached) {
  if (K == 0) {
    const C a0 = (C)(scale * c[0]);
    for (int e = threadIdx.x; e < L.n * CPB; e += blockDim.x) u[e] = (oz ? C(0) : u[e]) + a0 * x[e];
    __syncthreads();
    return;
  }
  const C* yin = x;
  C a = (C)c[K];
  C* buf[2] = {ya, yb};
  int cur = 0;
  for (int k = K - 1; k >= 1; --k) {
    tl_hop<CPB, WG>(L, yin, a, x, (C)c[k], buf[cur], 0, C(0), 0, rc, cached);
    yin = buf[cur];
    cur ^= 1;
    a = C(1);
  }
  tl_hop<CPB, WG>(L, yin, a, x, (C)c[0], u, 1, (C)scale, oz, rc, cached);
}

// the coarsest tail level: u = A^{-1} f (FP64 accumulation)
template <int CPB, class C>
__device__ __forceinline__ void tl_coarse(const TailArgs<C>& T, C* sm) {
  const TailLevel<C>& tl = T.lv[T.nl - 1];
  const C* f = sm + tl.off_f;
  C* u = sm + tl.off_u;
  // per-column operators (CPB == 1): the inverse of this workgroup's column
  const Lvl<C>& LJ = tl.L;
  const double* Ai = LJ.vs ? T.Ainv + (size_t)vcol(LJ, (int)blockIdx.x) * T.nJ * T.nJ : T.Ainv;
  for (int e = threadIdx.x; e < T.nJ * CPB; e += blockDim.x) {
    const int i = e / CPB, c = e - i * CPB;
    double acc = 0.0;
    for (int j = 0; j < T.nJ; ++j) acc += Ai[(size_t)i * T.nJ + j] * (double)f[j * CPB + c];
    u[e] = (C)acc;
  }
  __syncthreads();
}

// One learnable cycle over tail levels q0 .. nl-1 in LDS: u_q0 <- LMG(f_q0, u_q0)
// (uz0: u_q0 is logically zero on entry; deeper levels always start from zero).
template <int CPB, bool WG, class C>
__device__ __forceinline__ void tl_cycle(const TailArgs<C>& T, C* sm, int q0, int uz0) {
  C *s = sm + T.off_s, *ya = sm + T.off_ya, *yb = sm + T.off_yb, *t = sm + T.off_t;
  // down: pre-smoothing and restriction
  for (int q = q0; q + 1 < T.nl; ++q) {
    const TailLevel<C>& tl = T.lv[q];
    const double* p = T.prm + (size_t)q * T.per;
    const double *cB = p + 2, *cR = cB + T.KB + 1;
    C* u = sm + tl.off_u;
    const C* f = sm + tl.off_f;
    TRow<C, WG> rc;
    const bool cached = tl_cacheable<CPB, WG>(tl.L);
    if (cached) tl_load_row<CPB, WG>(tl.L, rc);
    int uz = q == q0 ? uz0 : 1;
    for (int j = 0; j < T.nu_pre; ++j) {
      tl_resid<CPB>(tl.L, f, u, uz, 1, s, rc, cached);
      tl_conv_add<CPB, WG>(tl.L, cB, T.KB, s, p[1] * p[0], u, uz, ya, yb, rc, cached);
      uz = 0;
    }
    // r = f - A u (u may still be zero when nu_pre == 0), then y = Phi_R r, f_{l+1} = R y
    tl_resid<CPB>(tl.L, f, u, uz, 0, t, rc, cached);
    if (uz) {  // u is logically zero: materialise it for the prolongation's update
      for (int e = threadIdx.x; e < tl.L.n * CPB; e += blockDim.x) u[e] = C(0);
      __syncthreads();
    }
    tl_conv_add<CPB, WG>(tl.L, cR, T.KR, t, 1.0, s, 1, ya, yb, rc, cached);
    tl_xfer<CPB>(tl.R, s, sm + T.lv[q + 1].off_f, 0, C(1), 0);
  }
  tl_coarse<CPB>(T, sm);
  // up: prolongation with Phi_P and post-smoothing
  for (int q = T.nl - 2; q >= q0; --q) {
    const TailLevel<C>& tl = T.lv[q];
    const double* p = T.prm + (size_t)q * T.per;
    const double *cB = p + 2, *cP = cB + T.KB + 1 + T.KR + 1;
    C* u = sm + tl.off_u;
    const C* f = sm + tl.off_f;
    TRow<C, WG> rc;
    const bool cached = tl_cacheable<CPB, WG>(tl.L);
    if (cached) tl_load_row<CPB, WG>(tl.L, rc);
    tl_xfer<CPB>(tl.P, sm + T.lv[q + 1].off_u, t, 0, C(1), 0);
    tl_conv_add<CPB, WG>(tl.L, cP, T.KP, t, 1.0, u, 0, ya, yb, rc, cached);
    for (int j = 0; j < T.nu_post; ++j) {
      tl_resid<CPB>(tl.L, f, u, 0, 1, s, rc, cached);
      tl_conv_add<CPB, WG>(tl.L, cB, T.KB, s, p[1] * p[0], u, 0, ya, yb, rc, cached);
    }
  }
}

// fmg == 0: e = LMG(A_lt, f, 0) over the tail levels lt .. J-1.
// fmg == 1: e = FMG(f) over the same levels: f_{q+1} = R Phi_R(f_q), exact
//           coarsest solve, then per level u_q = Phi_P(P u_{q+1}) and one cycle.
template <int CPB, bool WG, class C, class TU>
__global__ __launch_bounds__(1024) void k_tail(TailArgs<C> T, int B, const TU* __restrict__ fg,
                                               TU* __restrict__ eg, int fmg) {
  extern __shared__ __align__(16) unsigned char tail_smem[];
  C* sm = reinterpret_cast<C*>(tail_smem);
  const int col0 = blockIdx.x * CPB;
  // load the first tail level's right-hand side for this workgroup's columns
  {
    const TailLevel<C>& t0 = T.lv[0];
    for (int e = threadIdx.x; e < t0.L.n * CPB; e += blockDim.x) {
      const int i = e / CPB, c = e - i * CPB;
      sm[t0.off_f + e] = (col0 + c < B) ? (C)fg[(size_t)i * B + col0 + c] : C(0);
    }
    __syncthreads();
  }
  if (!fmg) {
    tl_cycle<CPB, WG>(T, sm, 0, 1);
  } else {
    C *s = sm + T.off_s, *ya = sm + T.off_ya, *yb = sm + T.off_yb, *t = sm + T.off_t;
    for (int q = 0; q + 1 < T.nl; ++q) {
      const TailLevel<C>& tl = T.lv[q];
      const double* cR = T.prm + (size_t)q * T.per + 2 + T.KB + 1;
      tl_conv_add<CPB, WG>(tl.L, cR, T.KR, sm + tl.off_f, 1.0, s, 1, ya, yb, TRow<C, WG>{}, false);
      tl_xfer<CPB>(tl.R, s, sm + T.lv[q + 1].off_f, 0, C(1), 0);
    }
    tl_coarse<CPB>(T, sm);
    for (int q = T.nl - 2; q >= 0; --q) {
      const TailLevel<C>& tl = T.lv[q];
      const double* cP = T.prm + (size_t)q * T.per + 2 + T.KB + 1 + T.KR + 1;
      tl_xfer<CPB>(tl.P, sm + T.lv[q + 1].off_u, t, 0, C(1), 0);
      tl_conv_add<CPB, WG>(tl.L, cP, T.KP, t, 1.0, sm + tl.off_u, 1, ya, yb, TRow<C, WG>{}, false);
      tl_cycle<CPB, WG>(T, sm, q, 0);
    }
  }
  {
    const TailLevel<C>& t0 = T.lv[0];
    for (int e = threadIdx.x; e < t0.L.n * CPB; e += blockDim.x) {
      const int i = e / CPB, c = e - i * CPB;
      if (col0 + c < B) put(eg + (size_t)i * B + col0 + c, sm[t0.off_u + e]);
    }
  }
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
// Every work-item reaches the block sum (no early return).
template <int ROWS, bool WIDE, bool WG, class C, class TZ, class TS>
__global__ __launch_bounds__(256) void k_hopT(Lvl<C> L, int B, int lbs, const TZ* __restrict__ zin,
                                              const TZ* __restrict__ zsrc, TZ* __restrict__ zout, C c,
                                              TZ* __restrict__ acc, int first, const TS* __restrict__ s,
                                              double* __restrict__ part) {
  __shared__ double red[256];
  const Tile<ROWS, WIDE> t(L.n, lbs);
  double d = 0.0;
  for (int b = t.lane; b < B; b += t.LB) {
    C z[ROWS], av[ROWS], sv[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const size_t o = (size_t)t.row[r] * B + b;
      z[r] = zin ? C(0) : ldc<C>(zsrc + o);
      av[r] = first ? C(0) : ldc<C>(acc + o);
      sv[r] = ldc<C>(s + o);
    }
    if (zin) graph_sum<WIDE, false, ROWS, true, WG>(L, t.row, t.row0, zin, B, b, z);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (!t.ok[r]) continue;
      const size_t o = (size_t)t.row[r] * B + b;
      if (zout) put(zout + o, z[r]);
      put(acc + o, av[r] + c * z[r]);
      d += (double)z[r] * (double)sv[r];
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
template <int ROWS, bool WIDE, class C, class TZ>
__global__ __launch_bounds__(256) void k_sub_Aq(Lvl<C> L, int B, int lbs, const TZ* gin,
                                                const TZ* __restrict__ q, TZ* gout) {
  const Tile<ROWS, WIDE> t(L.n, lbs);
  for (int b = t.lane; b < B; b += t.LB) {
    C gv[ROWS], qv[ROWS], s[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      gv[r] = ldc<C>(gin + (size_t)t.row[r] * B + b);
      qv[r] = ldc<C>(q + (size_t)t.row[r] * B + b);
      s[r] = C(0);
    }
    ell_dot<WIDE, false>(L.w, L.ld, L.col, L.val, t.row, t.row0, q, B, b, s);
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
      if (t.ok[r]) put(gout + (size_t)t.row[r] * B + b, gv[r] - (s[r] + uni<WIDE>(L.diag[t.row[r]]) * qv[r]));
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

// Gradients with respect to Chebyshev coefficients from those with respect to
// the power-series coefficients the cycle ran with:
//   a_m = sum_k c_k (-1)^k T_k[m]   =>   dL/dc_k = (-1)^k sum_m T_k[m] dL/da_m
// for every convolution of every level (one work-item per level).
__global__ void k_cheb_grad(double* __restrict__ g, int L, int per, int KB, int KR, int KP, ChebTab T) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  double* gl = g + (size_t)l * per + 2;
  const int Ks[3] = {KB, KR, KP};
  for (int q = 0; q < 3; ++q) {
    const int K = Ks[q];
    double out[9];
    for (int k = 0; k <= K; ++k) {
      double v = 0.0;
      for (int m = 0; m <= k; ++m) v += T.t[k][m] * gl[m];
      out[k] = (k & 1) ? -v : v;
    }
    for (int k = 0; k <= K; ++k) gl[k] = out[k];
    gl += K + 1;
  }
}

}  // namespace mgl
