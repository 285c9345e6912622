// Host driver and C ABI of the learnable V-cycle (see include/mgl.h).
//
// mg_setup turns the host CSR hierarchy into device ELL structures inside one
// workspace buffer; the V-cycle (paper Alg. 2), the refinement iteration
// u^m = u^{m-1} + B(f - A u^{m-1}) (Sec. 1), the solver loop and the reverse
// sweep used for training (Sec. 3.1) are sequences of the kernels of
// kernels.hpp enqueued on the caller's stream; full multigrid and flexible
// GMRES with the cycle as preconditioner (Sec. 4.2) add the Krylov kernels of
// krylov.hpp.  Three precisions share the code: FP64 throughout; FP32 cycles;
// FP32 cycles with BF16 intermediates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "krylov.hpp"
#include "mgl.h"
#include "plan.hpp"
#include "tiles.hpp"

using namespace mgl;

namespace {

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return fail(MG_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define LAUNCH_OK()                                                                         \
  do {                                                                                      \
    hipError_t e_ = hipGetLastError();                                                      \
    if (e_ != hipSuccess) return fail(MG_ERR_HIP, std::string("kernel launch at line ") +   \
                                                   std::to_string(__LINE__) + ": " + hipGetErrorString(e_)); \
  } while (0)

// launch `...` bracketed by the timing events of kernel family `fam`
#define TIMED(fam, bytes, ...)                   \
  do {                                           \
    MG_TRY(tmark((fam), l, false, 0.0, st));     \
    __VA_ARGS__;                                 \
    LAUNCH_OK();                                 \
    MG_TRY(tmark((fam), l, true, (bytes), st));  \
  } while (0)

#define MGL_UNPAREN(...) __VA_ARGS__
// run `...` with the compile-time flag WGv = (the aggregation uses edge weights)
#define WG_SPLIT(...)                      \
  do {                                     \
    if (wgt()) {                           \
      constexpr bool WGv = true;           \
      __VA_ARGS__;                         \
    } else {                               \
      constexpr bool WGv = false;          \
      __VA_ARGS__;                         \
    }                                      \
  } while (0)
// run `...` with the compile-time flag PCVv = (the columns have their own operator values)
#define PCV_SPLIT(...)                     \
  do {                                     \
    if (pl.nv) {                           \
      constexpr bool PCVv = true;          \
      __VA_ARGS__;                         \
    } else {                               \
      constexpr bool PCVv = false;         \
      __VA_ARGS__;                         \
    }                                      \
  } while (0)
// launch row-tile kernel KERN<ROWS, TARGS...> over the rows of level record D
#define ROWS_LAUNCH(D, KERN, TARGS, ...)                                                                        \
  do {                                                                                                          \
    if (lbs == 6) {                                                                                             \
      if ((D).rows4)                                                                                            \
        hipLaunchKernelGGL((KERN<4, true, MGL_UNPAREN TARGS>), dim3((D).rblocks), dim3(256), 0, st, __VA_ARGS__); \
      else                                                                                                      \
        hipLaunchKernelGGL((KERN<1, true, MGL_UNPAREN TARGS>), dim3((D).rblocks), dim3(256), 0, st, __VA_ARGS__); \
    } else {                                                                                                    \
      if ((D).rows4)                                                                                            \
        hipLaunchKernelGGL((KERN<4, false, MGL_UNPAREN TARGS>), dim3((D).rblocks), dim3(256), 0, st, __VA_ARGS__); \
      else                                                                                                      \
        hipLaunchKernelGGL((KERN<1, false, MGL_UNPAREN TARGS>), dim3((D).rblocks), dim3(256), 0, st, __VA_ARGS__); \
    }                                                                                                           \
  } while (0)
// as ROWS_LAUNCH for kernels with a finest-level tag (FINE = level 0)
#define ROWS_LAUNCH_F(D, FINE, KERN, TARGS, ...)                                                      \
  do {                                                                                                \
    if (FINE) ROWS_LAUNCH(D, KERN, (true, MGL_UNPAREN TARGS), __VA_ARGS__);                           \
    else ROWS_LAUNCH(D, KERN, (false, MGL_UNPAREN TARGS), __VA_ARGS__);                               \
  } while (0)
// restriction sweep (one coarse row per lane group), wave-uniform rows when B >= 64
#define RESTRICT_LAUNCH(GRID, TARGS, ...)                                                                        \
  do {                                                                                                          \
    if (lbs == 6)                                                                                               \
      hipLaunchKernelGGL((k_restrict<true, MGL_UNPAREN TARGS>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__);      \
    else                                                                                                        \
      hipLaunchKernelGGL((k_restrict<false, MGL_UNPAREN TARGS>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__);     \
  } while (0)


// ------------------------------------------------------------------ workspace bump allocator
struct Bump {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

inline int lb_shift(int B) {
  int s = 0;
  while ((1 << s) < B && s < 6) ++s;
  return s;
}
inline unsigned nblocks(long threads) { return (unsigned)((threads + 255) / 256); }

struct EngineBase {
  virtual mg_status vcycle(const void* f, void* u, void* ck, hipStream_t st) = 0;
  virtual mg_status vcycle_bwd(const void* ck, const void* gout, void* gin, void* gf, double* gp, hipStream_t st) = 0;
  virtual mg_status residual(const double* f, const double* u, double* r, double* norms, hipStream_t st) = 0;
  virtual mg_status residual_loss(int kind, const double* f, const double* u, const double* gseed, double* loss,
                                  double* gu, double* gf, hipStream_t st) = 0;
  virtual mg_status refine(const double* f, const double* uin, double* uout, void* ck, hipStream_t st) = 0;
  virtual mg_status refine_bwd(const void* ck, const double* gout, double* gin, double* gf, double* gp, hipStream_t st) = 0;
  virtual mg_status solve(const double* f, double* u, mg_rhs_info* info, hipStream_t st) = 0;
  virtual mg_status fmg_entry(const void* f, void* u, hipStream_t st) = 0;
  virtual mg_status fgmres(const double* f, double* u, const mg_krylov_options* o, void* work, size_t wbytes,
                           mg_rhs_info* info, hipStream_t st) = 0;
  virtual size_t fgmres_bytes(int restart) = 0;
  virtual mg_status set_params(const double* v, hipStream_t st) = 0;
  virtual mg_status load_column(int b, const double* const* vals, hipStream_t st) = 0;
  virtual mg_status setup(void* ws, hipStream_t st) = 0;
  virtual size_t ws_bytes() = 0;
  virtual size_t ck_bytes() = 0;
  HostPlan pl;
  std::vector<int64_t> sizes;
  std::vector<int32_t> widths;

  // ---- launch timing (instrumentation)
  int tfam = MG_KF_NONE;
  int tlevel = -1;               // -1: every level
  std::vector<hipEvent_t> tev;   // start/stop pairs, reused across runs
  size_t tn = 0;                 // pairs recorded
  double tbytes = 0.0;
  virtual ~EngineBase() {
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
  }
  mg_status timing_start(int fam, int level) {
    tfam = fam;
    tlevel = level;
    tn = 0;
    tbytes = 0.0;
    return MG_OK;
  }
  // record one event of the pair for launch family `fam`; returns false when not timed
  mg_status tmark(int fam, int level, bool stop, double bytes, hipStream_t st) {
    // level -2 marks launches that are never timed (their work is data-dependent)
    if (fam != tfam || tfam == MG_KF_NONE || level < -1 || (tlevel >= 0 && level != tlevel)) return MG_OK;
    const size_t k = 2 * tn + (stop ? 1 : 0);
    while (tev.size() <= k) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      tev.push_back(e);
    }
    HIP_TRY(hipEventRecord(tev[k], st));
    if (stop) {
      ++tn;
      tbytes += bytes;
    }
    return MG_OK;
  }
  mg_status timing_read(int64_t* n, double* ms, double* bytes) {
    double tot = 0.0;
    if (tn) HIP_TRY(hipEventSynchronize(tev[2 * tn - 1]));
    for (size_t k = 0; k < tn; ++k) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, tev[2 * k], tev[2 * k + 1]));
      tot += t;
    }
    if (n) *n = (int64_t)tn;
    if (ms) *ms = tot;
    if (bytes) *bytes = tbytes;
    return MG_OK;
  }
};

// ------------------------------------------------------------------ engine
template <class C, class TU, class TH>
struct Engine final : EngineBase {
  struct DL {
    Lvl<C> L{};
    Xfer<C> P{}, R{}, PT{}, RT{};   // P: n_l x n_{l+1}, R: n_{l+1} x n_l, PT = P^T, RT = R^T
    TU *f = nullptr, *u = nullptr;  // levels >= 1
    TH *s = nullptr, *ya = nullptr, *yb = nullptr, *x = nullptr;
    TU* r = nullptr;
    // reverse sweep
    TH* S[2 * kMaxNu] = {};
    TU *Rv = nullptr, *ut = nullptr, *g = nullptr, *za = nullptr, *zb = nullptr, *acc = nullptr, *q = nullptr,
       *gfo = nullptr, *gin = nullptr;
    TH* X = nullptr;
    unsigned blocks = 0;            // one work-item per (row, lane): n * LB / 256
    int rows4 = 0;                  // row-tile sweeps use 4 rows per work-item
    unsigned rblocks = 0;           // blocks of the row-tile sweeps
    TileDev td{};                   // fused convolution tiles (td.ntiles == 0: none)
    TileLds tlo[kTileMaxK + 1] = {};  // LDS layout of a fused convolution of order K
    size_t tlds[kTileMaxK + 1] = {};  // and its size in bytes
    unsigned tgrid[kTileMaxK + 1] = {};  // persistent grid (a multiple of 8 blocks)
    int tocc[kTileMaxK + 1] = {};        // resident workgroups per compute unit
  };
  std::vector<DL> d;
  Lvl<double> L64{};                // level-0 operator in FP64 (outer residual)
  double* Ainv = nullptr;           // coarsest inverse, row-major
  double* gj = nullptr;             // Gauss-Jordan scratch n x 2n
  int* dinfo = nullptr;
  TU *r0 = nullptr, *e0 = nullptr;  // refinement: cycle input / output (level 0)
  double* dbuf = nullptr;           // FP64 level-0 scratch
  double *part = nullptr, *norms = nullptr, *fnorm = nullptr, *init = nullptr;
  double *lalpha = nullptr, *lbeta = nullptr;   // residual-loss gradient coefficients per column
  int* dstat = nullptr;
  double *dots = nullptr, *dpart = nullptr, *dprm = nullptr;
  long* doff = nullptr;
  int *dcnt = nullptr, *ddesc = nullptr;
  int nslots = 0;
  std::vector<long> h_off;
  std::vector<int> h_cnt, h_desc;
  int* hcount = nullptr;            // pinned host
  char* kr_own = nullptr;           // Krylov workspace allocated by the library
  size_t kr_own_bytes = 0;
  char* tile_mem = nullptr;         // tile lists of the fused convolution, allocated by the library
  size_t tile_mem_bytes = 0;
  // coarse tail (levels tail_lt .. J-1 in LDS, one workgroup per column)
  int tail_lt = -1;                 // shallowest level whose tail fits in LDS
  std::vector<TailArgs<C>> tails;   // launch arguments for start levels tail_lt .. J-2
  std::vector<size_t> tail_bytes;
  char* wsbase = nullptr;
  bool owns_ws = false;
  int lbs = 0;                      // lanes per row (log2) of the cycle's sweeps at the current width
  int lbsF = 0;                     // the same at the full width (outer residual, solver bookkeeping)
  int curB = 0;                     // columns the cycle runs on: nrhs, or fewer while compacted
  int ncu = 0;                      // compute units of the device
  // active-column compaction of mg_solve: column b's cycle data at slot cmap[b] of curB
  int* cmap = nullptr;              // device [nrhs]
  int* vmapd = nullptr;             // per-column operators: device [nrhs], operator column of each slot
  double* colstage = nullptr;       // per-column operators: one column's level arrays (mg_load_column)
  double* colhost = nullptr;        // pinned host: all level arrays of one column (mg_load_column)
  size_t colhost_n = 0;             // its size in doubles
  int* cfrom = nullptr;             // device [nrhs]: old slot of each new slot (repack)
  int* hmap = nullptr;              // pinned host [3 nrhs]: flags, new map, repack sources
  std::vector<int> hcur;            // host copy of cmap
  bool compacted = false;
  // device-side host copies kept alive during setup
  std::vector<uvector<char>> staging;

  ~Engine() override {
    if (owns_ws && wsbase) (void)hipFree(wsbase);
    if (kr_own) (void)hipFree(kr_own);
    if (tile_mem) (void)hipFree(tile_mem);
    if (hcount) (void)hipHostFree(hcount);
    if (hmap) (void)hipHostFree(hmap);
    if (colhost) (void)hipHostFree(colhost);
  }

  bool bwd() const { return (pl.flags & MG_FLAG_BACKWARD) != 0; }
  bool wgt() const { return pl.agg != MG_AGG_MEAN; }
  int per() const { return 2 + (pl.KB + 1) + (pl.KR + 1) + (pl.KP + 1); }
  double theta(int l) const { return pl.params[(size_t)l * per()]; }
  double eta(int l) const { return pl.params[(size_t)l * per() + 1]; }
  const double* cB(int l) const { return &pl.params[(size_t)l * per() + 2]; }
  const double* cR(int l) const { return cB(l) + pl.KB + 1; }
  const double* cP(int l) const { return cR(l) + pl.KR + 1; }

  // slots of the reverse sweep, in launch order (kind, level, k)
  void enum_slots(int l) {
    const int J = pl.J;
    if (l == J - 1) return;
    auto add = [&](int kind, int K) {
      for (int k = 0; k <= K; ++k) {
        h_desc.push_back(kind); h_desc.push_back(l); h_desc.push_back(k);
        h_cnt.push_back((int)d[l].rblocks);
        h_off.push_back(h_off.empty() ? 0 : h_off.back() + h_cnt[h_cnt.size() - 2]);
      }
    };
    for (int j = 0; j < pl.nu_post; ++j) add(0, pl.KB);
    add(2, pl.KP);
    enum_slots(l + 1);
    add(1, pl.KR);
    for (int j = 0; j < pl.nu_pre; ++j) add(0, pl.KB);
  }

  // launch shapes of level l's row sweeps at the current cycle width
  void level_launch(int l) {
    DL& x = d[l];
    const int n = pl.lv[l].n;
    x.blocks = nblocks((long)n << lbs);
    const long rpb = 256 >> lbs;
    const long b4 = (n + 4 * rpb - 1) / (4 * rpb);
    x.rows4 = b4 >= 512 ? 1 : 0;   // 2048 was 0.7 % slower on the 513 workload
    x.rblocks = (unsigned)(x.rows4 ? b4 : (n + rpb - 1) / rpb);
  }
  // persistent grid of level l's fused convolution of order K: the resident workgroups of
  // every XCD, or fewer when there are fewer (tile, column group) items
  void tile_grid(int l, int K) {
    DL& x = d[l];
    const long W = (long)x.td.ntiles * x.td.ngroups;
    const long per = std::min<long>((W + 7) / 8, (long)std::max(1, ncu / 8) * x.tocc[K]);
    x.tgrid[K] = (unsigned)(8 * std::max<long>(per, 1));
  }
  // run the cycle on Bc columns (Bc <= nrhs): every row sweep's lanes and blocks, and the
  // fused convolution's column groups and grid
  void set_width(int Bc) {
    curB = Bc;
    lbs = lb_shift(Bc);
    for (int l = 0; l < pl.J; ++l) {
      level_launch(l);
      if (d[l].td.ntiles) {
        d[l].td.ngroups = Bc / kTileCols;
        for (int K = 2; K <= d[l].td.KM; ++K) tile_grid(l, K);
      }
    }
  }

  // assign device pointers (base == nullptr: sizes only)
  size_t carve(char* base) {
    Bump bp;
    bp.base = base;
    const int J = pl.J, B = pl.B;
    d.assign(J, DL{});
    lbs = lbsF = lb_shift(B);
    curB = B;
    compacted = false;
    for (int l = 0; l < J; ++l) {
      const HLevel& H = pl.lv[l];
      DL& x = d[l];
      const int n = H.n;
      level_launch(l);
      const int ld = round_up(n, 4);
      x.L.n = n;
      x.L.ld = ld;
      x.L.w = H.off.w;
      x.L.col = bp.take<int>((size_t)H.off.w * ld);
      const size_t nvv = pl.nv ? (size_t)pl.nv : 1;   // operator columns (per-column operators: nrhs)
      x.L.vs = pl.nv;
      x.L.vmap = nullptr;
      x.L.val = bp.take<C>((size_t)H.off.w * ld * nvv);
      x.L.diag = bp.take<C>(ld * nvv);
      x.L.invdiag = bp.take<C>(ld * nvv);
      x.L.invdeg = bp.take<C>(ld);
      if (H.graph_is_A) {
        x.L.wg = H.off.w;
        x.L.gcol = x.L.col;
      } else {
        x.L.wg = H.graph.w;
        x.L.gcol = bp.take<int>((size_t)H.graph.w * ld);
      }
      x.L.gval = pl.agg != MG_AGG_MEAN ? bp.take<C>((size_t)x.L.wg * ld) : nullptr;
      const size_t nv = (size_t)n * B;
      if (l > 0) { x.f = bp.take<TU>(nv); x.u = bp.take<TU>(nv); }
      x.s = bp.take<TH>(nv); x.ya = bp.take<TH>(nv); x.yb = bp.take<TH>(nv); x.x = bp.take<TH>(nv);
      x.r = bp.take<TU>(nv);
      if (bwd()) {
        for (int j = 0; j < pl.nu_pre + pl.nu_post; ++j) x.S[j] = bp.take<TH>(nv);
        x.Rv = bp.take<TU>(nv); x.X = bp.take<TH>(nv); x.ut = bp.take<TU>(nv); x.g = bp.take<TU>(nv);
        x.za = bp.take<TU>(nv); x.zb = bp.take<TU>(nv); x.acc = bp.take<TU>(nv); x.q = bp.take<TU>(nv);
        x.gfo = bp.take<TU>(nv); x.gin = bp.take<TU>(nv);
      }
    }
    for (int l = 0; l + 1 < J; ++l) {
      DL& x = d[l];
      auto mk = [&](const HEll& e, Xfer<C>& t) {
        t.n = e.n; t.w = e.w;
        t.col = bp.take<int>((size_t)e.w * e.n);
        t.val = bp.take<C>((size_t)e.w * e.n);
      };
      mk(pl.P[l], x.P);
      mk(pl.PT[l], x.PT);
      if (pl.R_is_PT) { x.R = x.PT; x.RT = x.P; }
      else { mk(pl.R[l], x.R); mk(pl.RT[l], x.RT); }
    }
    if constexpr (std::is_same<C, double>::value) {
      L64 = d[0].L;
    } else {
      L64.n = d[0].L.n; L64.ld = d[0].L.ld; L64.w = d[0].L.w; L64.col = d[0].L.col; L64.wg = d[0].L.wg;
      L64.gcol = d[0].L.gcol;
      L64.vs = pl.nv;
      L64.vmap = nullptr;
      const size_t nvv = pl.nv ? (size_t)pl.nv : 1;
      L64.val = bp.take<double>((size_t)pl.lv[0].off.w * d[0].L.ld * nvv);
      L64.diag = bp.take<double>(d[0].L.ld * nvv);
      L64.invdiag = nullptr;
      L64.invdeg = nullptr;
      L64.gval = nullptr;
    }
    const int nJ = pl.lv[J - 1].n;
    Ainv = bp.take<double>((size_t)nJ * nJ * (pl.nv ? pl.nv : 1));
    gj = bp.take<double>((size_t)nJ * 2 * nJ);
    if (pl.nv) {
      // mg_load_column: one column's operator of the largest level, staged in FP64, and the
      // vector-to-operator column map of a compacted cycle
      size_t st = 0;
      for (int l = 0; l < J; ++l) st = std::max(st, (size_t)(pl.lv[l].off.w + 1) * round_up(pl.lv[l].n, 4));
      colstage = bp.take<double>(st);
      vmapd = bp.take<int>(B);
    }
    dinfo = bp.take<int>(1);
    const size_t n0B = (size_t)pl.lv[0].n * B;
    r0 = bp.take<TU>(n0B);
    e0 = bp.take<TU>(n0B);
    dbuf = bp.take<double>(n0B);
    part = bp.take<double>((size_t)kOuterBlocks * B);
    norms = bp.take<double>(B);
    fnorm = bp.take<double>(B);
    init = bp.take<double>(B);
    lalpha = bp.take<double>(B);
    lbeta = bp.take<double>(B);
    dstat = bp.take<int>(3 * B + 1);
    cmap = bp.take<int>(B);
    cfrom = bp.take<int>(B);
    dprm = bp.take<double>(pl.params.size());
    if (bwd()) {
      h_off.clear(); h_cnt.clear(); h_desc.clear();
      enum_slots(0);
      nslots = (int)h_cnt.size();
      const long tot = nslots ? h_off.back() + h_cnt.back() : 0;
      dpart = bp.take<double>(tot);
      dots = bp.take<double>(nslots);
      doff = bp.take<long>(nslots);
      dcnt = bp.take<int>(nslots);
      ddesc = bp.take<int>(3 * (size_t)nslots);
    }
    return bp.off + 256;
  }

  size_t ws_bytes() override { return carve(nullptr); }

  size_t ck_bytes() override {
    size_t b = 0;
    for (int l = 0; l < pl.J; ++l) b += 2 * (((size_t)pl.lv[l].n * pl.B * sizeof(TU) + 255) & ~size_t(255));
    return b;
  }

  struct Ck {
    TU* f[32];
    TU* u[32];
  };
  Ck ck_ptrs(void* base) const {
    Ck c{};
    char* p = static_cast<char*>(base);
    for (int l = 0; l < pl.J; ++l) {
      const size_t b = ((size_t)pl.lv[l].n * pl.B * sizeof(TU) + 255) & ~size_t(255);
      c.f[l] = reinterpret_cast<TU*>(p); p += b;
      c.u[l] = reinterpret_cast<TU*>(p); p += b;
    }
    return c;
  }

  template <class T, class V>
  mg_status up(T* dst, const V& src, hipStream_t st) {
    if (src.empty()) return MG_OK;
    uvector<char> buf(src.size() * sizeof(T));
    T* t = reinterpret_cast<T*>(buf.data());
    const long cnt = (long)src.size();
    par_rows((int)((cnt + 1023) / 1024), [&](int b0, int b1) {
      for (long i = (long)b0 * 1024; i < std::min(cnt, (long)b1 * 1024); ++i) t[i] = (T)src[i];
    });
    HIP_TRY(hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, st));
    staging.push_back(std::move(buf));
    return MG_OK;
  }
  template <class V>
  mg_status upi(const int* dst, const V& src, hipStream_t st) {
    if (src.empty()) return MG_OK;
    HIP_TRY(hipMemcpyAsync(const_cast<int*>(dst), src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice, st));
    return MG_OK;
  }

  // Ainv (operator column b) = A^{-1} of the dense coarsest operator Ad (row-major n_J x n_J):
  // Gauss-Jordan with partial pivoting in FP64 on the device; *dinfo != 0 if singular
  mg_status coarse_inverse(const double* Ad, int b, hipStream_t st) {
    const int nJ = pl.lv[pl.J - 1].n;
    std::vector<double> W((size_t)nJ * 2 * nJ, 0.0);
    for (int i = 0; i < nJ; ++i) {
      for (int j = 0; j < nJ; ++j) W[(size_t)i * 2 * nJ + j] = Ad[(size_t)i * nJ + j];
      W[(size_t)i * 2 * nJ + nJ + i] = 1.0;
    }
    MG_TRY(up(gj, W, st));
    hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, st, nJ, gj, dinfo);
    LAUNCH_OK();
    HIP_TRY(hipMemcpy2DAsync(Ainv + (size_t)b * nJ * nJ, nJ * sizeof(double), gj + nJ, 2 * nJ * sizeof(double),
                             nJ * sizeof(double), nJ, hipMemcpyDeviceToDevice, st));
    return MG_OK;
  }

  mg_status setup(void* ws, hipStream_t st) override {
    const size_t need = ws_bytes();
    if (ws) {
      wsbase = static_cast<char*>(ws);
    } else {
      HIP_TRY(hipMalloc(&wsbase, need));
      owns_ws = true;
    }
    carve(wsbase);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&hcount), sizeof(int) * 4, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&hmap), sizeof(int) * 3 * pl.B, hipHostMallocDefault));
    const int J = pl.J;
    for (int l = 0; l < J; ++l) {
      const HLevel& H = pl.lv[l];
      DL& x = d[l];
      MG_TRY(upi(x.L.col, H.off.col, st));
      std::vector<double> ideg(x.L.ld, 0.0);
      for (int i = 0; i < H.n; ++i) ideg[i] = H.invdeg[i];
      MG_TRY(up(const_cast<C*>(x.L.invdeg), ideg, st));
      if (pl.nv) {
        // per-column operators: [slot][row][column] values, [row][column] diagonals
        MG_TRY(up(const_cast<C*>(x.L.val), H.offv, st));
        std::vector<double> inv(H.diagv.size(), 0.0);
        for (int i = 0; i < H.n; ++i)
          for (int b = 0; b < pl.nv; ++b) inv[(size_t)i * pl.nv + b] = 1.0 / H.diagv[(size_t)i * pl.nv + b];
        MG_TRY(up(const_cast<C*>(x.L.diag), H.diagv, st));
        MG_TRY(up(const_cast<C*>(x.L.invdiag), inv, st));
      } else {
        MG_TRY(up(const_cast<C*>(x.L.val), H.off.val, st));
        std::vector<double> dg(x.L.ld, 1.0), inv(x.L.ld, 0.0);
        for (int i = 0; i < H.n; ++i) {
          dg[i] = H.diag[i];
          inv[i] = 1.0 / H.diag[i];
        }
        MG_TRY(up(const_cast<C*>(x.L.diag), dg, st));
        MG_TRY(up(const_cast<C*>(x.L.invdiag), inv, st));
      }
      if (!H.graph_is_A) MG_TRY(upi(x.L.gcol, H.graph.col, st));
      if (x.L.gval) MG_TRY(up(const_cast<C*>(x.L.gval), H.gval, st));
    }
    for (int l = 0; l + 1 < J; ++l) {
      DL& x = d[l];
      MG_TRY(upi(x.P.col, pl.P[l].col, st));
      MG_TRY(up(const_cast<C*>(x.P.val), pl.P[l].val, st));
      MG_TRY(upi(x.PT.col, pl.PT[l].col, st));
      MG_TRY(up(const_cast<C*>(x.PT.val), pl.PT[l].val, st));
      if (!pl.R_is_PT) {
        MG_TRY(upi(x.R.col, pl.R[l].col, st));
        MG_TRY(up(const_cast<C*>(x.R.val), pl.R[l].val, st));
        MG_TRY(upi(x.RT.col, pl.RT[l].col, st));
        MG_TRY(up(const_cast<C*>(x.RT.val), pl.RT[l].val, st));
      }
    }
    if (!std::is_same<C, double>::value) {
      if (pl.nv) {
        MG_TRY(up(const_cast<double*>(L64.val), pl.lv[0].offv, st));
        MG_TRY(up(const_cast<double*>(L64.diag), pl.lv[0].diagv, st));
      } else {
        MG_TRY(up(const_cast<double*>(L64.val), pl.lv[0].off.val, st));
        std::vector<double> dg(L64.ld, 1.0);
        for (int i = 0; i < L64.n; ++i) dg[i] = pl.lv[0].diag[i];
        MG_TRY(up(const_cast<double*>(L64.diag), dg, st));
      }
    }
    // coarsest inverse (one per operator column): W = [A | I], Gauss-Jordan on the device
    const int nJ = pl.lv[J - 1].n;
    for (int b = 0; b < (pl.nv ? pl.nv : 1); ++b) {
      MG_TRY(coarse_inverse(pl.nv ? &pl.AcoarseV[(size_t)b * nJ * nJ] : pl.Acoarse.data(), b, st));
      if (pl.nv) {
        HIP_TRY(hipMemcpyAsync(hcount, dinfo, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (hcount[0] != 0)
          return fail(MG_ERR_SHAPE, "coarsest matrix of column " + std::to_string(b) + " is singular");
      }
    }
    MG_TRY(up(dprm, pl.params, st));
    if (bwd()) {
      HIP_TRY(hipMemcpyAsync(doff, h_off.data(), h_off.size() * sizeof(long), hipMemcpyHostToDevice, st));
      MG_TRY(upi(dcnt, h_cnt, st));
      MG_TRY(upi(ddesc, h_desc, st));
    }
    int info = 0;
    HIP_TRY(hipMemcpyAsync(hcount, dinfo, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    info = hcount[0];
    staging.clear();
    staging.shrink_to_fit();
    if (info != 0) return fail(MG_ERR_SHAPE, "coarsest matrix is singular (zero pivot in column " + std::to_string(info - 1) + ")");
    MG_TRY(setup_tiles(st));
    MG_TRY(setup_tail());
    sizes.resize(J);
    widths.resize(J);
    for (int l = 0; l < J; ++l) { sizes[l] = pl.lv[l].n; widths[l] = pl.lv[l].off.w; }
    return MG_OK;
  }

  // Choose the shallowest start level without fused-convolution tiles whose
  // coarse tail fits the workgroup's LDS, and prepare the launch arguments
  // for every start level below it.
  mg_status setup_tail() {
    tail_lt = -1;
    tails.clear();
    tail_bytes.clear();
    if (pl.flags & MG_FLAG_NO_TAIL) return MG_OK;
    int dev = 0, maxlds = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int J = pl.J;
    auto r4 = [](long x) { return (x + 3) / 4 * 4; };
    auto bytes_from = [&](int lt) {
      long elems = 4 * r4(pl.lv[lt].n);
      for (int l = lt; l < J; ++l) elems += 2 * r4(pl.lv[l].n);
      return (size_t)elems * sizeof(C);
    };
    // levels with fused-convolution tiles keep their per-level launches
    for (int lt = 0; lt <= J - 2; ++lt)
      if (J - lt <= kTailMaxLevels && bytes_from(lt) <= (size_t)maxlds && d[lt].td.ntiles == 0) {
        tail_lt = lt;
        break;
      }
    if (tail_lt < 0) return MG_OK;
    const void* tail_fn = wgt() ? reinterpret_cast<const void*>(&k_tail<1, true, C, TU>)
                                : reinterpret_cast<const void*>(&k_tail<1, false, C, TU>);
    if (bytes_from(tail_lt) > 65536 &&
        hipFuncSetAttribute(tail_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes_from(tail_lt)) !=
            hipSuccess) {
      (void)hipGetLastError();
      tail_lt = -1;   // large dynamic LDS unavailable: keep the per-level sweeps
      return MG_OK;
    }
    for (int lt = tail_lt; lt <= J - 2; ++lt) {
      TailArgs<C> t{};
      t.nl = J - lt;
      long off = 0;
      for (int q = 0; q < t.nl; ++q) {
        const int l = lt + q;
        t.lv[q].L = d[l].L;
        if (l < J - 1) { t.lv[q].P = d[l].P; t.lv[q].R = d[l].R; }
        t.lv[q].off_u = (int)off; off += r4(pl.lv[l].n);
        t.lv[q].off_f = (int)off; off += r4(pl.lv[l].n);
      }
      const long ns = r4(pl.lv[lt].n);
      t.off_s = (int)off; off += ns;
      t.off_ya = (int)off; off += ns;
      t.off_yb = (int)off; off += ns;
      t.off_t = (int)off; off += ns;
      t.KB = pl.KB; t.KR = pl.KR; t.KP = pl.KP;
      t.nu_pre = pl.nu_pre; t.nu_post = pl.nu_post; t.per = per();
      t.prm = dprm + (size_t)lt * per();
      t.Ainv = Ainv;
      t.nJ = pl.lv[J - 1].n;
      t.lt = lt;
      tails.push_back(t);
      tail_bytes.push_back(bytes_from(lt));
    }
    return MG_OK;
  }

  // Tiles of the fused K-hop convolution (FP32/BF16 cycles, B a multiple of
  // kTileCols): levels with at least kTileMinRows rows (the coarse tail then
  // starts below them), halo depth the largest
  // convolution order >= 2; tile shape shrunk until one workgroup's LDS fits
  // kTileLds.  The lists live in library-owned device memory.
#ifndef MGL_TILE_LDS_KB
#define MGL_TILE_LDS_KB 80
#endif
// bands per band group of the tile order (on the 513 workload: 1, 2, 8 and 16 made the
// finest-level convolution 0-2 % slower and the cycle 0.3-1 % slower than 4)
#ifndef MGL_TILE_GROUP
#define MGL_TILE_GROUP 4
#endif
#ifndef MGL_TILE_MIN_ROWS
#define MGL_TILE_MIN_ROWS 2048
#endif
  static constexpr int kTileMinRows = MGL_TILE_MIN_ROWS;
  static constexpr size_t kTileLds = MGL_TILE_LDS_KB * 1024;
  mg_status setup_tiles(hipStream_t st) {
    if constexpr (std::is_same<C, float>::value) return setup_tiles_f(st);
    else return MG_OK;
  }
  mg_status setup_tiles_f(hipStream_t st) {
    if ((pl.flags & MG_FLAG_NO_TILES) || B() % kTileCols != 0) return MG_OK;
    int KM = 0;
    for (int K : {pl.KB, pl.KR, pl.KP})
      if (K >= 2) KM = std::max(KM, K);
    if (KM < 2) return MG_OK;
    // per-item limits of the kernel's register pipeline
    auto fits = [&](const TilePlan& t) {
      const int m = t.maxcnt[KM - 1];
      return t.maxcnt[KM] <= kTileRows * kTileNp && t.maxcnt[0] <= kTileOwnPerThread * kTileNp &&
             m * t.wg / 4 <= kTileMeta * kTileThreads && m <= kTileMeta * kTileThreads &&
             tile_lds_bytes(t, KM, kTileCols) <= kTileLds;
    };
    std::vector<TilePlan> tp(pl.J);
    std::vector<std::vector<float>> lidg(pl.J), lgw(pl.J);
    std::vector<std::vector<uint16_t>> lcb(pl.J);
    size_t bytes = 0;
    auto a256 = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
    for (int l = 0; l < pl.J; ++l) {
      const HLevel& H = pl.lv[l];
      if (H.n < kTileMinRows) continue;
      const HEll& g = H.graph_is_A ? H.off : H.graph;
      for (int side : {16, 15, 14, 12, 10, 8}) {
        if (build_tiles(H.n, g.ld, g.w, g.col.data(), KM, side, side, tp[l], MGL_TILE_GROUP) && fits(tp[l])) break;
        tp[l] = TilePlan{};
      }
      const TilePlan& t = tp[l];
      if (!t.ntiles) continue;
      if (!check_tiles(H.n, g.ld, g.col.data(), t))
        return fail(MG_ERR_STATE, "tile lists of level " + std::to_string(l) + " are inconsistent");
      // row scales and edge weights of the listed rows, in the device's precision
      lidg[l].resize(t.lcol.size() / t.wg);
      if (wgt()) lgw[l].resize(t.lcol.size());
      for (int k = 0; k < t.ntiles; ++k) {
        const int* L = &t.node[t.toff[k]];
        const int m0 = t.goff[k], rows = (t.goff[k + 1] - m0) / t.wg;
        for (int r = 0; r < rows; ++r) {
          lidg[l][m0 / t.wg + r] = (float)H.invdeg[L[r]];
          if (wgt())
            for (int s = 0; s < t.wg; ++s) lgw[l][m0 + (size_t)r * t.wg + s] = (float)H.gval[(size_t)s * g.ld + L[r]];
        }
      }
      bytes += a256((t.ntiles + 1) * sizeof(int)) * 2 + a256(t.node.size() * sizeof(int)) +
               a256(t.cnt.size() * sizeof(int)) + a256(t.lcol.size() * sizeof(uint16_t)) +
               a256(lidg[l].size() * sizeof(float)) + a256(lgw[l].size() * sizeof(float));
    }
    if (!bytes) return MG_OK;
    HIP_TRY(hipMalloc(&tile_mem, bytes));
    tile_mem_bytes = bytes;
    char* p = tile_mem;
    bool ok = true;
    auto put = [&](const void* src, size_t b) -> void* {
      void* dst = p;
      p += a256(b);
      if (b && hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, st) != hipSuccess) ok = false;
      return dst;
    };
    size_t maxlds = 0;
    for (int l = 0; l < pl.J; ++l) {
      const TilePlan& t = tp[l];
      if (!t.ntiles) continue;
      TileDev& td = d[l].td;
      td.ntiles = t.ntiles; td.KM = t.KM; td.wg = t.wg; td.ngroups = B() / kTileCols;
      td.toff = static_cast<const int*>(put(t.toff.data(), t.toff.size() * sizeof(int)));
      td.goff = static_cast<const int*>(put(t.goff.data(), t.goff.size() * sizeof(int)));
      td.node = static_cast<const int*>(put(t.node.data(), t.node.size() * sizeof(int)));
      td.cnt = static_cast<const int*>(put(t.cnt.data(), t.cnt.size() * sizeof(int)));
      // local columns as byte offsets from the buffer's row of zeros (one LDS row: kTileCols floats);
      // at most kTileRows * kTileNp listed rows (fits above), so they fit 16 bits
      static_assert((kTileRows * kTileNp + 1) * kTileCols * sizeof(float) <= 65535, "16-bit LDS offsets");
      lcb[l].resize(t.lcol.size());
      for (size_t k = 0; k < t.lcol.size(); ++k) lcb[l][k] = (uint16_t)(t.lcol[k] * (kTileCols * sizeof(float)));
      td.lcol = static_cast<const uint16_t*>(put(lcb[l].data(), lcb[l].size() * sizeof(uint16_t)));
      td.lidg = static_cast<const float*>(put(lidg[l].data(), lidg[l].size() * sizeof(float)));
      td.lgw = wgt() ? static_cast<const float*>(put(lgw[l].data(), lgw[l].size() * sizeof(float))) : nullptr;
      for (int K = 2; K <= t.KM; ++K) {
        const TileLayout y = tile_layout(t, K, kTileCols);
        d[l].tlo[K] = TileLds{y.xs, y.y0, y.y1, y.col, y.idg};
        d[l].tlds[K] = tile_lds_bytes(t, K, kTileCols);
        maxlds = std::max(maxlds, d[l].tlds[K]);
      }
    }
    if (!ok) return fail(MG_ERR_HIP, "tile list upload failed");
    const void* fns[] = {
        reinterpret_cast<const void*>(&k_conv_tile<false, false, TH, TU>),
        reinterpret_cast<const void*>(&k_conv_tile<false, true, TH, TU>),
        reinterpret_cast<const void*>(&k_conv_tile<false, false, TU, TH>),
        reinterpret_cast<const void*>(&k_conv_tile<false, true, TU, TH>),
        reinterpret_cast<const void*>(&k_conv_tile<true, false, TH, TU>),
        reinterpret_cast<const void*>(&k_conv_tile<true, true, TH, TU>),
        reinterpret_cast<const void*>(&k_conv_tile<true, false, TU, TH>),
        reinterpret_cast<const void*>(&k_conv_tile<true, true, TU, TH>)};
    if (maxlds > 65536)
      for (const void* fn : fns)
        HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)maxlds));
    // persistent grid: resident workgroups per XCD (the instances share one
    // register and LDS footprint up to the weights; take the smallest)
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    for (int l = 0; l < pl.J; ++l) {
      if (!d[l].td.ntiles) continue;
      for (int K = 2; K <= d[l].td.KM; ++K) {
        int occ = 1 << 30;
        for (const void* fn : fns) {
          int nb = 0;
          HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kTileThreads, d[l].tlds[K]));
          occ = std::min(occ, nb);
        }
        if (occ < 1) return fail(MG_ERR_STATE, "fused convolution does not fit one compute unit");
        d[l].tocc[K] = occ;
        tile_grid(l, K);
      }
    }
    HIP_TRY(hipStreamSynchronize(st));   // the host lists are freed on return
    return MG_OK;
  }

  bool tiled(int l, int K, const void* x, const void* out) const {
    const TileDev& td = d[l].td;
    return td.ntiles > 0 && K >= 2 && K <= td.KM && x != out && ((uintptr_t)x % 16) == 0 &&
           ((uintptr_t)out % 16) == 0;
  }

  // fused convolution: mode 0 out = Phi(x), mode 1 out = (oz ? 0 : out) + scale Phi(x);
  // with xsc, x_i xsc_i in place of x_i
  template <class TX, class TO>
  mg_status conv_tile(int l, const double* c, int K, const TX* x, TO* out, int mode, double scale, int oz,
                      hipStream_t st, const C* xsc = nullptr) {
    if constexpr (std::is_same<C, float>::value) {
      const DL& D = d[l];
      TileCoef cf{};
      for (int k = 0; k <= K; ++k) cf.c[k] = (float)c[k];
      const double bytes = nB(l) * (sizeof(TX) + sizeof(TO) * ((mode && !oz) ? 2 : 1)) +
                           (double)D.L.wg * D.L.n * (4 + (wgt() ? sizeof(C) : 0)) + (double)D.L.n * sizeof(C) +
                           (xsc ? (double)D.L.n * sizeof(C) : 0.0);
      if (l == 0)
        TIMED(MG_KF_CONV, bytes,
              WG_SPLIT(hipLaunchKernelGGL((k_conv_tile<true, WGv, TX, TO>), dim3(D.tgrid[K]), dim3(kTileThreads),
                                          D.tlds[K], st, D.td, B(), K, cf, x, out, mode, (float)scale, oz,
                                          D.tlo[K], xsc)));
      else
        TIMED(MG_KF_CONV, bytes,
              WG_SPLIT(hipLaunchKernelGGL((k_conv_tile<false, WGv, TX, TO>), dim3(D.tgrid[K]), dim3(kTileThreads),
                                          D.tlds[K], st, D.td, B(), K, cf, x, out, mode, (float)scale, oz,
                                          D.tlo[K], xsc)));
      return MG_OK;
    } else {
      return fail(MG_ERR_STATE, "fused convolution needs FP32 cycles");
    }
  }

  // e = LMG(A_l, f, 0) (fmg: e = FMG(f)) for levels l .. J-1 in one launch (l >= tail_lt)
  mg_status run_tail(int l, const TU* f, TU* e, hipStream_t st, int fmg = 0) {
    const int q = l - tail_lt;
    WG_SPLIT(hipLaunchKernelGGL((k_tail<1, WGv, C, TU>), dim3(B()), dim3(1024), tail_bytes[q], st, tails[q], B(),
                                f, e, fmg));
    LAUNCH_OK();
    return MG_OK;
  }

  // replace column b's operators on every level (per-column operator contexts)
  mg_status load_column(int b, const double* const* vals, hipStream_t st) override {
    if (!pl.nv) return fail(MG_ERR_STATE, "context was set up without per-column operators");
    if (b < 0 || b >= pl.nv) return fail(MG_ERR_INVALID_ARG, "column out of range");
    if (!vals) return fail(MG_ERR_INVALID_ARG, "null values");
    for (int l = 0; l < pl.J; ++l)
      if (!vals[l]) return fail(MG_ERR_INVALID_ARG, "null values of level " + std::to_string(l));
    const int J = pl.J;
    // every level's arrays into one pinned host buffer (kept for the next
    // call: no page faults, and the copies run at the host link's DMA rate),
    // validated first, so a refused column leaves the context unchanged
    std::vector<size_t> at(J + 1, 0);
    for (int l = 0; l < J; ++l) at[l + 1] = at[l] + (size_t)(pl.lv[l].off.w + 1) * pl.lv[l].off.ld;
    if (colhost_n < at[J]) {
      if (colhost) HIP_TRY(hipHostFree(colhost));
      colhost = nullptr;
      colhost_n = 0;
      HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&colhost), at[J] * sizeof(double), hipHostMallocDefault));
      colhost_n = at[J];
    }
    for (int l = 0; l < J; ++l) {
      const HLevel& H = pl.lv[l];
      const int w = H.off.w, ld = H.off.ld;
      mg_csr pat{H.n, H.n, (int64_t)pl.pcol[l].size(), pl.prow[l].data(), pl.pcol[l].data(), nullptr};
      MG_TRY(column_arrays(&pat, vals[l], H, colhost + at[l], colhost + at[l] + (size_t)w * ld, l, b));
    }
    for (int l = 0; l < J; ++l) {
      const HLevel& H = pl.lv[l];
      const int w = H.off.w, ld = H.off.ld;
      HIP_TRY(hipMemcpyAsync(colstage, colhost + at[l], (at[l + 1] - at[l]) * sizeof(double), hipMemcpyHostToDevice,
                             st));
      const bool f64 = l == 0 && !std::is_same<C, double>::value;
      const long cnt = std::max<long>((long)w * ld, ld);
      hipLaunchKernelGGL((k_put_column<C>), dim3(nblocks(cnt)), dim3(256), 0, st, w, ld, H.n, pl.nv, b,
                         (const double*)colstage, (const double*)(colstage + (size_t)w * ld), const_cast<C*>(d[l].L.val),
                         const_cast<C*>(d[l].L.diag), const_cast<C*>(d[l].L.invdiag),
                         f64 ? const_cast<double*>(L64.val) : nullptr, f64 ? const_cast<double*>(L64.diag) : nullptr);
      LAUNCH_OK();
    }
    // the next call rewrites colhost: its copies end first (the stream orders the
    // reuse of colstage between levels)
    HIP_TRY(hipStreamSynchronize(st));
    const int nJ = pl.lv[J - 1].n;
    std::vector<double> Ad((size_t)nJ * nJ, 0.0);
    const std::vector<int32_t>& rp = pl.prow[J - 1];
    const std::vector<int32_t>& cl = pl.pcol[J - 1];
    for (int i = 0; i < nJ; ++i)
      for (int q = rp[i]; q < rp[i + 1]; ++q) Ad[(size_t)i * nJ + cl[q]] = vals[J - 1][q];
    MG_TRY(coarse_inverse(Ad.data(), b, st));
    HIP_TRY(hipMemcpyAsync(hcount, dinfo, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    staging.clear();
    if (hcount[0] != 0) return fail(MG_ERR_SHAPE, "coarsest matrix of the new column is singular");
    return MG_OK;
  }

  mg_status set_params(const double* v, hipStream_t st) override {
    for (size_t i = 0; i < pl.params.size(); ++i)
      if (!std::isfinite(v[i])) return fail(MG_ERR_INVALID_ARG, "non-finite parameter");
    pl.params.assign(v, v + pl.params.size());
    to_power_series(pl.params, pl.J, pl.KB, pl.KR, pl.KP, pl.basis);
    HIP_TRY(hipMemcpyAsync(dprm, pl.params.data(), pl.params.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MG_OK;
  }

  // ---------------------------------------------------------------- forward building blocks
  int B() const { return curB; }     // columns of the cycle's vectors
  int BF() const { return pl.B; }    // columns of the solver-level (FP64) vectors

  template <class TY, class TX, class TO>
  mg_status hop(int l, const TY* yin, double a, const TX* x, double c, TO* out, int mode, double scale, int oz,
                hipStream_t st) {
    const DL& D = d[l];
    const double nB = (double)D.L.n * B();
    const double bytes = nB * (sizeof(TY) + sizeof(TX) + sizeof(TO) * ((mode && !oz) ? 2 : 1)) +
                         (double)D.L.wg * D.L.n * (4 + (wgt() ? sizeof(C) : 0)) + (double)D.L.n * sizeof(C);
    TIMED(MG_KF_HOP, bytes,
          WG_SPLIT(ROWS_LAUNCH_F(D, l == 0, k_hop, (WGv, C, TY, TX, TO), D.L, B(), lbs, yin, (C)a, x,
                                 (C)c, out, mode, (C)scale, oz)));
    return MG_OK;
  }

  // algorithmic bytes of streaming A_l once (ELL indices, values, diagonal)
  double bytes_A(int l) const { return (double)d[l].L.w * d[l].L.n * (4 + sizeof(C)) + (double)d[l].L.n * sizeof(C); }
  double bytes_X(const Xfer<C>& x) const { return (double)x.w * x.n * (4 + sizeof(C)); }
  double nB(int l) const { return (double)d[l].L.n * B(); }

  // u = (oz ? 0 : u) + scale * sum_k c_k M^k x
  mg_status conv_add(int l, const double* c, int K, const TH* x, double scale, TU* u, int oz, hipStream_t st) {
    const DL& D = d[l];
    if (K == 0) {
      hipLaunchKernelGGL((k_axpy<C, TH, TU>), dim3(D.blocks), dim3(256), 0, st, D.L.n, B(), lbs, x, (C)(scale * c[0]),
                         u, oz);
      LAUNCH_OK();
      return MG_OK;
    }
    if (tiled(l, K, x, u)) return conv_tile<TH, TU>(l, c, K, x, u, 1, scale, oz, st);
    const TH* yin = x;
    double a = c[K];
    TH* buf[2] = {D.ya, D.yb};
    int cur = 0;
    for (int k = K - 1; k >= 1; --k) {
      MG_TRY(hop<TH, TH, TH>(l, yin, a, x, c[k], buf[cur], 0, 0.0, 0, st));
      yin = buf[cur];
      cur ^= 1;
      a = 1.0;
    }
    return hop<TH, TH, TU>(l, yin, a, x, c[0], u, 1, scale, oz, st);
  }

  // one learnable smoothing step; s receives D^{-1}(f - A u), except that with
  // keep_s = false a zero iterate's step runs as one fused convolution of D^{-1} f
  // (same arithmetic; s is not written)
  mg_status smooth(int l, const TU* f, TU* u, int uz, TH* s, hipStream_t st, bool keep_s = true) {
    const DL& D = d[l];
    if constexpr (std::is_same<TH, TU>::value && std::is_same<C, float>::value) {
      if (uz && !keep_s && pl.KB >= 2 && !pl.nv && tiled(l, pl.KB, f, u))
        return conv_tile<TU, TU>(l, cB(l), pl.KB, f, u, 1, eta(l) * theta(l), 1, st, D.L.invdiag);
    }
    TIMED(MG_KF_RESID, nB(l) * (sizeof(TU) * (uz ? 1 : 2) + sizeof(TH)) + (uz ? 0.0 : bytes_A(l)) +
                           (double)D.L.n * sizeof(C),
          PCV_SPLIT(ROWS_LAUNCH_F(D, l == 0, k_resid, (PCVv, C, TU, TH), D.L, B(), lbs, f, u, uz, 1, s)));
    return conv_add(l, cB(l), pl.KB, s, eta(l) * theta(l), u, uz, st);
  }

  // rc = R_l Phi_R(f - A u)
  mg_status restrict_(int l, const TU* f, const TU* u, int uz, TU* rc, hipStream_t st) {
    const DL& D = d[l];
    const int K = pl.KR;
    const double* c = cR(l);
    const unsigned cb = d[l + 1].blocks;
    if (K == 0) {
      TIMED(MG_KF_RESTRICT, nB(l) * sizeof(TU) * (uz ? 1 : 2) + (uz ? 0.0 : bytes_A(l)) + bytes_X(D.R) +
                                nB(l + 1) * sizeof(TU),
            RESTRICT_LAUNCH(cb, (false, C, TU, TU, TU), D.R, D.L, B(), lbs, 2,
                               (const TU*)nullptr, (C)0, (const TU*)nullptr, (C)0, f, u, uz, (C)c[0], rc));
      return MG_OK;
    }
    TIMED(MG_KF_RESID, nB(l) * sizeof(TU) * (uz ? 2 : 3) + (uz ? 0.0 : bytes_A(l)),
          PCV_SPLIT(ROWS_LAUNCH_F(D, l == 0, k_resid, (PCVv, C, TU, TU), D.L, B(), lbs, f, u, uz, 0,
                             D.r)));
    const double rbytes = nB(l) * 2 * sizeof(TU) + (double)D.L.wg * D.L.n * 4 + (double)D.L.n * sizeof(C) +
                          bytes_X(D.R) + nB(l + 1) * sizeof(TU);
    if (K == 1) {
      TIMED(MG_KF_RESTRICT, rbytes,
            WG_SPLIT(RESTRICT_LAUNCH(cb, (WGv, C, TU, TU, TU), D.R, D.L, B(), lbs, 1,
                               (const TU*)D.r, (C)c[1], (const TU*)D.r, (C)c[0], (const TU*)nullptr,
                               (const TU*)nullptr, 0, (C)1, rc)));
      return MG_OK;
    }
    if (tiled(l, K, D.r, D.ya)) {
      // y = Phi_R(r) in one fused launch, then the plain restriction of y
      MG_TRY(conv_tile<TU, TH>(l, c, K, D.r, D.ya, 0, 1.0, 0, st));
      TIMED(MG_KF_RESTRICT, nB(l) * sizeof(TH) + bytes_X(D.R) + nB(l + 1) * sizeof(TU),
            RESTRICT_LAUNCH(cb, (false, C, TU, TH, TU), D.R, D.L, B(), lbs, 0, (const TH*)D.ya, (C)0,
                            (const TU*)nullptr, (C)0, (const TU*)nullptr, (const TU*)nullptr, 0, (C)1, rc));
      return MG_OK;
    }
    MG_TRY(hop<TU, TU, TH>(l, D.r, c[K], D.r, c[K - 1], D.ya, 0, 0.0, 0, st));
    const TH* y = D.ya;
    TH* bufs[2] = {D.ya, D.yb};
    int cur = 1;
    for (int k = K - 2; k >= 1; --k) {
      MG_TRY(hop<TH, TU, TH>(l, y, 1.0, D.r, c[k], bufs[cur], 0, 0.0, 0, st));
      y = bufs[cur];
      cur ^= 1;
    }
    TIMED(MG_KF_RESTRICT, rbytes - nB(l) * (sizeof(TU) - sizeof(TH)),
          WG_SPLIT(RESTRICT_LAUNCH(cb, (WGv, C, TU, TH, TU), D.R, D.L, B(), lbs, 1, y,
                             (C)1, (const TU*)D.r, (C)c[0], (const TU*)nullptr, (const TU*)nullptr, 0, (C)1, rc)));
    return MG_OK;
  }

  // u = (uz ? 0 : u) + Phi_P(P ec);  xbuf receives P ec when K >= 1
  mg_status prolong(int l, const TU* ec, TU* u, int uz, TH* xbuf, hipStream_t st) {
    const DL& D = d[l];
    if (pl.KP == 0) {
      TIMED(MG_KF_PROLONG, nB(l + 1) * sizeof(TU) + bytes_X(D.P) + nB(l) * sizeof(TU) * (uz ? 1 : 2),
            ROWS_LAUNCH(D, k_prolong, (C, TU, TU), D.P, B(), lbs, ec, u, 1,
                               (C)cP(l)[0], uz));
      return MG_OK;
    }
    TIMED(MG_KF_PROLONG, nB(l + 1) * sizeof(TU) + bytes_X(D.P) + nB(l) * sizeof(TH),
          ROWS_LAUNCH(D, k_prolong, (C, TU, TH), D.P, B(), lbs, ec, xbuf, 0,
                             (C)1, 0));
    return conv_add(l, cP(l), pl.KP, xbuf, 1.0, u, uz, st);
  }

  mg_status coarse(const TU* f, TU* u, int trans, hipStream_t st) {
    const int n = pl.lv[pl.J - 1].n;
    hipLaunchKernelGGL((k_coarse<TU>), dim3(nblocks((long)n * B())), dim3(256), 0, st, n, B(), Ainv, f, u, trans,
                       pl.nv ? 1 : 0, (const int*)d[pl.J - 1].L.vmap);
    LAUNCH_OK();
    return MG_OK;
  }

  // u = LMG(A_l, f, u) (Alg. 2); uz: u is identically zero on entry
  mg_status fwd(int l, const TU* f, TU* u, int uz, const Ck* ck, hipStream_t st) {
    if (tail_lt >= 0 && l >= tail_lt && l < pl.J - 1 && uz && !ck) return run_tail(l, f, u, st);
    if (l == pl.J - 1) return coarse(f, u, 0, st);
    DL& D = d[l];
    for (int j = 0; j < pl.nu_pre; ++j) {
      MG_TRY(smooth(l, f, u, uz, D.s, st, false));
      uz = 0;
    }
    TU* fn = ck ? ck->f[l + 1] : d[l + 1].f;
    TU* un = ck ? ck->u[l + 1] : d[l + 1].u;
    MG_TRY(restrict_(l, f, u, uz, fn, st));
    MG_TRY(fwd(l + 1, fn, un, 1, ck, st));
    MG_TRY(prolong(l, un, u, uz, D.x, st));
    uz = 0;
    for (int j = 0; j < pl.nu_post; ++j) MG_TRY(smooth(l, f, u, 0, D.s, st));
    return MG_OK;
  }

  template <class TI, class TO>
  mg_status copy(const TI* in, TO* out, long cnt, hipStream_t st) {
    hipLaunchKernelGGL((k_copy<TI, TO>), dim3(nblocks(cnt)), dim3(256), 0, st, cnt, in, out);
    LAUNCH_OK();
    return MG_OK;
  }

  mg_status vcycle(const void* fv, void* uv, void* ckv, hipStream_t st) override {
    const TU* f = static_cast<const TU*>(fv);
    TU* u = static_cast<TU*>(uv);
    const long n0B = (long)pl.lv[0].n * B();
    if (ckv) {
      Ck ck = ck_ptrs(ckv);
      MG_TRY(copy(f, ck.f[0], n0B, st));
      MG_TRY(copy((const TU*)u, ck.u[0], n0B, st));
      return fwd(0, f, u, 0, &ck, st);
    }
    return fwd(0, f, u, 0, nullptr, st);
  }

  // outer residual: contiguous row chunks (a multiple of 4 rows), at most kOuterBlocks blocks
  int outer_chunk() const {
    const long n = pl.lv[0].n;
    const long rows_per_pass = 4L * (256 >> lbsF);
    long chunk = std::max<long>(rows_per_pass, (n + kOuterBlocks - 1) / kOuterBlocks);
    chunk = (chunk + 3) / 4 * 4;
    return (int)chunk;
  }
  unsigned outer_blocks() const {
    const long c = outer_chunk();
    return (unsigned)((pl.lv[0].n + c - 1) / c);
  }

  // r = f - A u (FP64, all nrhs columns) with per-column norms; rc receives fl_p(r).  With e
  // (the solver's fused update): the iterate is u + e in the active columns, written to uo
  // (!= u), and stopped columns are not touched.  While the cycle runs compacted, rc and e
  // hold column b at slot cmap[b] of the current width.
  template <class TR>
  mg_status outer_resid(const double* f, const double* u, double* r64, TR* rc, double* nrm, hipStream_t st,
                        const TU* e = nullptr, const int* act = nullptr, double* uo = nullptr) {
    const int l = 0;   // timing level of the finest-level outer residual
    const unsigned g = outer_blocks();
    const int Bc = (e && compacted) ? B() : BF();
    const int* map = (e && compacted) ? cmap : nullptr;
    const double nb0 = (double)L64.n * BF();
    const double ob = nb0 * 16 + (double)L64.w * L64.n * 12 + (double)L64.n * 8 + (r64 ? nb0 * 8 : 0.0) +
                      (rc ? nb0 * sizeof(TR) : 0.0) + (e ? nb0 * (sizeof(TU) + 8) : 0.0);
    if (e) {
      TIMED(MG_KF_OUTER, ob, PCV_SPLIT(
            if (lbsF == 6) hipLaunchKernelGGL((k_outer_resid<true, true, PCVv, TR, TU>), dim3(g), dim3(256), 0, st, L64,
                                              BF(), lbsF, outer_chunk(), f, u, r64, rc, part, e, act, uo, Bc, map);
            else hipLaunchKernelGGL((k_outer_resid<false, true, PCVv, TR, TU>), dim3(g), dim3(256), 0, st, L64, BF(),
                                    lbsF, outer_chunk(), f, u, r64, rc, part, e, act, uo, Bc, map)));
    } else {
      TIMED(MG_KF_OUTER, ob, PCV_SPLIT(
            if (lbsF == 6) hipLaunchKernelGGL((k_outer_resid<true, false, PCVv, TR, TU>), dim3(g), dim3(256), 0, st, L64,
                                              BF(), lbsF, outer_chunk(), f, u, r64, rc, part, (const TU*)nullptr,
                                              (const int*)nullptr, (double*)nullptr, Bc, map);
            else hipLaunchKernelGGL((k_outer_resid<false, false, PCVv, TR, TU>), dim3(g), dim3(256), 0, st, L64, BF(),
                                    lbsF, outer_chunk(), f, u, r64, rc, part, (const TU*)nullptr, (const int*)nullptr,
                                    (double*)nullptr, Bc, map)));
    }
    if (nrm) {
      hipLaunchKernelGGL(k_norm_final, dim3(BF()), dim3(256), 0, st, part, (int)g, BF(), nrm, e ? act : nullptr);
      LAUNCH_OK();
    }
    return MG_OK;
  }

  // Compact the cycle to the columns still iterating (act flags on the device), rounded up to
  // a multiple of kTileCols columns: a new column map, the pending cycle input r0 gathered
  // into the new layout, and the narrower launch shapes.  Every kernel treats the columns
  // independently, so a column's arithmetic does not change.
  mg_status compact(int active, hipStream_t st) {
    const int Bn = round_up(std::max(active, 1), kTileCols);
    if (Bn >= B()) return MG_OK;
    const int F = BF();
    int* hact = hmap;
    int* hnew = hmap + F;
    int* hfrom = hmap + 2 * F;
    HIP_TRY(hipMemcpyAsync(hact, st_ptr(), F * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hcur.empty()) {
      hcur.resize(F);
      for (int b = 0; b < F; ++b) hcur[b] = b;
    }
    int slot = 0;
    for (int c = 0; c < Bn; ++c) hfrom[c] = -1;
    for (int b = 0; b < F; ++b) {
      if (hact[b] && slot < Bn) {
        hnew[b] = slot;
        hfrom[slot] = hcur[b];
        ++slot;
      } else {
        hnew[b] = -1;
      }
    }
    HIP_TRY(hipMemcpyAsync(cfrom, hfrom, Bn * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(cmap, hnew, F * sizeof(int), hipMemcpyHostToDevice, st));
    const long cnt = (long)pl.lv[0].n * Bn;
    hipLaunchKernelGGL((k_repack<TU>), dim3(nblocks(cnt)), dim3(256), 0, st, pl.lv[0].n, B(), Bn, (const int*)cfrom,
                       (const TU*)r0, e0);
    LAUNCH_OK();
    std::swap(r0, e0);
    for (int b = 0; b < F; ++b) hcur[b] = hnew[b];
    if (pl.nv) {
      // per-column operators: slot s uses the operator of the column it holds (padding: column 0)
      int* hv = hfrom;   // the repack sources were uploaded above; reuse after a sync
      HIP_TRY(hipStreamSynchronize(st));
      for (int c = 0; c < Bn; ++c) hv[c] = 0;
      for (int b = 0; b < F; ++b)
        if (hnew[b] >= 0) hv[hnew[b]] = b;
      HIP_TRY(hipMemcpyAsync(vmapd, hv, Bn * sizeof(int), hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));
      set_vmap(vmapd);
    }
    compacted = true;
    set_width(Bn);
    return MG_OK;
  }
  void uncompact() {
    if (!compacted) return;
    compacted = false;
    hcur.clear();
    if (pl.nv) set_vmap(nullptr);
    set_width(BF());
  }
  // the vector-to-operator column map of every level's sweeps (and the coarse tail's copies)
  void set_vmap(const int* vm) {
    for (auto& x : d) x.L.vmap = vm;
    for (auto& t : tails)
      for (int q = 0; q < t.nl; ++q) t.lv[q].L.vmap = vm;
  }

  mg_status residual(const double* f, const double* u, double* r, double* nrm, hipStream_t st) override {
    return outer_resid<TU>(f, u, r, nullptr, nrm, st);
  }

  // Residual loss of Alg. 3 and its gradients (kernels k_colsq, k_loss_coef, k_loss_grad):
  // r = f - A u in FP64 (dbuf), the column norms of r and f, the loss and the
  // per-column coefficients, then gu = -alpha A r and gf = alpha r - beta f in one sweep.
  mg_status residual_loss(int kind, const double* f, const double* u, const double* gseed, double* loss,
                          double* gu, double* gf, hipStream_t st) override {
    if (kind != MG_LOSS_MEAN_REL_SQ && kind != MG_LOSS_RESID_NORM) return fail(MG_ERR_INVALID_ARG, "unknown loss kind");
    if (gu && !(bwd() && pl.lv[0].sym_A))
      return fail(MG_ERR_UNSUPPORTED, "dL/du needs a symmetric A_0 and a context set up with MG_FLAG_BACKWARD");
    MG_TRY(outer_resid<TU>(f, u, dbuf, (TU*)nullptr, norms, st));
    const unsigned g = outer_blocks();
    const int n0 = pl.lv[0].n;
    if (lbs == 6) hipLaunchKernelGGL((k_colsq<true>), dim3(g), dim3(256), 0, st, n0, B(), lbs, outer_chunk(), f, part);
    else hipLaunchKernelGGL((k_colsq<false>), dim3(g), dim3(256), 0, st, n0, B(), lbs, outer_chunk(), f, part);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_norm_final, dim3(B()), dim3(256), 0, st, part, (int)g, B(), fnorm, (const int*)nullptr);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_loss_coef, dim3(1), dim3(256), 0, st, (const double*)norms, (const double*)fnorm, B(), kind,
                       gseed, lalpha, lbeta, loss);
    LAUNCH_OK();
    if (gu || gf) {
      const DL& D = d[0];
      const double* r = dbuf;
      if (lbs == 6) {
        if (D.rows4) hipLaunchKernelGGL((k_loss_grad<4, true>), dim3(D.rblocks), dim3(256), 0, st, L64, B(), lbs, r, f,
                                        (const double*)lalpha, (const double*)lbeta, gu, gf);
        else hipLaunchKernelGGL((k_loss_grad<1, true>), dim3(D.rblocks), dim3(256), 0, st, L64, B(), lbs, r, f,
                                (const double*)lalpha, (const double*)lbeta, gu, gf);
      } else {
        if (D.rows4) hipLaunchKernelGGL((k_loss_grad<4, false>), dim3(D.rblocks), dim3(256), 0, st, L64, B(), lbs, r, f,
                                        (const double*)lalpha, (const double*)lbeta, gu, gf);
        else hipLaunchKernelGGL((k_loss_grad<1, false>), dim3(D.rblocks), dim3(256), 0, st, L64, B(), lbs, r, f,
                                (const double*)lalpha, (const double*)lbeta, gu, gf);
      }
      LAUNCH_OK();
    }
    return MG_OK;
  }

  mg_status refine(const double* f, const double* uin, double* uout, void* ckv, hipStream_t st) override {
    const long n0B = (long)pl.lv[0].n * B();
    Ck ck{};
    if (ckv) ck = ck_ptrs(ckv);
    TU* rc = ckv ? ck.f[0] : r0;
    MG_TRY(outer_resid<TU>(f, uin, nullptr, rc, nullptr, st));
    MG_TRY(fwd(0, rc, e0, 1, ckv ? &ck : nullptr, st));
    if (uout != uin) MG_TRY(copy(uin, uout, n0B, st));
    hipLaunchKernelGGL((k_update<TU>), dim3(d[0].blocks), dim3(256), 0, st, pl.lv[0].n, B(), lbs, (const TU*)e0, uout,
                       (const int*)nullptr, 1.0);
    LAUNCH_OK();
    return MG_OK;
  }

  mg_status solve(const double* f, double* u, mg_rhs_info* info, hipStream_t st) override {
    const int n0 = pl.lv[0].n;
    // ||f|| per column: residual of u = 0 is f itself
    hipLaunchKernelGGL((k_fill0<double>), dim3(nblocks((long)n0 * BF())), dim3(256), 0, st, (long)n0 * BF(), dbuf);
    LAUNCH_OK();
    MG_TRY(outer_resid<TU>(f, dbuf, nullptr, (TU*)nullptr, fnorm, st));
    // iterate m of a column that is still updating lives in ua = (m even ? u : dbuf); each
    // update u + e is written to the other buffer by the next residual sweep (fused)
    MG_TRY(outer_resid<TU>(f, u, nullptr, r0, norms, st));
    double* ua = u;
    double* ub = dbuf;
    struct Restore {   // the cycle is back at full width however the loop ends
      Engine* e;
      ~Restore() { e->uncompact(); }
    } restore{this};
    int m = 0;
    for (; m < pl.max_outer; ++m) {
      hipLaunchKernelGGL(k_solve_check, dim3(1), dim3(256), 0, st, norms, fnorm, init, st_ptr(), BF(), pl.rtol, pl.divf,
                         m == 0 ? 1 : 0);
      LAUNCH_OK();
      if ((m + 1) % pl.check_every == 0 || m == 0) {
        HIP_TRY(hipMemcpyAsync(hcount, st_ptr() + 3 * BF(), sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (hcount[0] == 0) break;
        if (!(pl.flags & MG_FLAG_NO_COMPACT)) MG_TRY(compact(hcount[0], st));
      }
      MG_TRY(fwd(0, r0, e0, 1, nullptr, st));
      MG_TRY(outer_resid<TU>(f, ua, nullptr, r0, norms, st, e0, st_ptr(), ub));
      std::swap(ua, ub);
    }
    uncompact();
    // columns that ended after an odd number of updates hold their iterate in dbuf (the update
    // counts are the solver's per-column counts before the cap's final check below)
    hipLaunchKernelGGL(k_copy_odd, dim3(d[0].blocks), dim3(256), 0, st, n0, BF(), lbsF, (const int*)(st_ptr() + BF()),
                       (const double*)dbuf, u);
    LAUNCH_OK();
    if (m == pl.max_outer) {
      // the last iterate's residual is in norms: account for it
      hipLaunchKernelGGL(k_solve_check, dim3(1), dim3(256), 0, st, norms, fnorm, init, st_ptr(), BF(), pl.rtol, pl.divf, 0);
      LAUNCH_OK();
    }
    std::vector<int> hst(3 * BF() + 1);
    std::vector<double> hn(BF()), hf(BF());
    HIP_TRY(hipMemcpyAsync(hst.data(), st_ptr(), hst.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hn.data(), norms, BF() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hf.data(), fnorm, BF() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    mg_status ret = MG_OK;
    for (int b = 0; b < BF(); ++b) {
      // iters counted for columns still active after a check: they were updated
      // only if a cycle followed; a column active at the end ran every cycle
      int it = hst[BF() + b];
      if (hst[b]) it = std::min(it, m);
      const int s = hst[2 * BF() + b];
      if (info) {
        info[b].iters = it;
        info[b].status = s;
        info[b].relres = hf[b] > 0 ? hn[b] / hf[b] : hn[b];
      }
      if (s == MG_ERR_DIVERGED) ret = MG_ERR_DIVERGED;
      else if (s != MG_OK && ret == MG_OK) ret = MG_ERR_NOT_CONVERGED;
    }
    if (ret != MG_OK) g_err = ret == MG_ERR_DIVERGED ? "a column diverged" : "a column did not converge";
    return ret;
  }
  int* st_ptr() { return dstat; }

  // ---------------------------------------------------------------- full multigrid, FGMRES
  // u = FMG(f) (Sec. 4.2): right-hand sides carried down with the cycle's
  // restriction f_{l+1} = R_l Phi_R,l(f_l), exact solve on the coarsest level,
  // then on each finer level u_l = Phi_P,l(P_l u_{l+1}) followed by one
  // learnable cycle.  Uses the per-level cycle buffers of levels >= 1.
  // Levels from the LDS tail's start down run as one FMG launch of the tail kernel.
  mg_status fmg(const TU* f0, TU* u0, hipStream_t st) {
    const int J = pl.J;
    const int lt = tail_lt >= 0 ? tail_lt : J - 1;   // first level handled in one piece
    const TU* fl = f0;
    for (int l = 0; l < lt; ++l) {
      MG_TRY(restrict_(l, fl, fl, 1, d[l + 1].f, st));
      fl = d[l + 1].f;
    }
    TU* ult = lt == 0 ? u0 : d[lt].u;
    if (lt < J - 1) MG_TRY(run_tail(lt, fl, ult, st, 1));
    else MG_TRY(coarse(fl, ult, 0, st));
    for (int l = lt - 1; l >= 0; --l) {
      const TU* f = l == 0 ? f0 : d[l].f;
      TU* u = l == 0 ? u0 : d[l].u;
      MG_TRY(prolong(l, d[l + 1].u, u, 1, d[l].x, st));
      MG_TRY(fwd(l, f, u, 0, nullptr, st));
    }
    return MG_OK;
  }
  mg_status fmg_entry(const void* f, void* u, hipStream_t st) override {
    return fmg(static_cast<const TU*>(f), static_cast<TU*>(u), st);
  }

  // Krylov workspace (carved from one buffer)
  struct Kr {
    int m = 0, chunk = 0, nblk = 0, lbk = 0;
    long zs = 0;                   // element stride between preconditioned vectors
    double* V = nullptr;           // m + 1 unnormalised basis vectors vt_i, FP64, [n][m + 1][B]
    TU* Z = nullptr;               // m preconditioned vectors zt_j = C(fl(vt_j)), cycle type, [m][n][B]
    double *w = nullptr, *part = nullptr, *h1 = nullptr, *h2 = nullptr, *n2 = nullptr, *n4 = nullptr,
           *y = nullptr, *beta = nullptr;
    KrState S{};
  };
  static constexpr int kKrBlocks = 1024;
  size_t kr_carve(int m, char* base, Kr& k) {
    Bump bp;
    bp.base = base;
    const int n = pl.lv[0].n, Bn = B();
    const long nB = (long)n * Bn;
    k.lbk = 0;
    while ((1 << k.lbk) < Bn) ++k.lbk;
    const long rpb = 256 >> k.lbk;
    k.m = m;
    k.chunk = (int)std::max<long>(rpb, (n + kKrBlocks - 1) / kKrBlocks);
    k.nblk = (int)((n + k.chunk - 1) / k.chunk);
    k.zs = (nB + 127) / 128 * 128;
    k.V = bp.take<double>((size_t)(m + 1) * nB);
    k.Z = bp.take<TU>((size_t)m * k.zs);
    k.w = bp.take<double>(nB);
    k.part = bp.take<double>((size_t)k.nblk * (m + 2) * Bn);
    k.h1 = bp.take<double>((size_t)(m + 2) * Bn);
    k.h2 = bp.take<double>((size_t)(m + 2) * Bn);
    k.n2 = bp.take<double>(Bn);
    k.n4 = bp.take<double>(Bn);
    k.y = bp.take<double>((size_t)m * Bn);
    k.beta = bp.take<double>(Bn);
    k.S.m = m;
    k.S.H = bp.take<double>((size_t)(m + 1) * m * Bn);
    k.S.cs = bp.take<double>((size_t)m * Bn);
    k.S.sn = bp.take<double>((size_t)m * Bn);
    k.S.g = bp.take<double>((size_t)(m + 1) * Bn);
    k.S.sig = bp.take<double>((size_t)(m + 1) * Bn);
    k.S.fnorm = bp.take<double>(Bn);
    k.S.act = bp.take<int>(Bn);
    k.S.jd = bp.take<int>(Bn);
    k.S.flag = bp.take<int>(1);
    k.S.st = bp.take<int>(3 * (size_t)Bn + 1);
    return bp.off + 256;
  }
  size_t fgmres_bytes(int restart) override {
    Kr k;
    return kr_carve(restart, nullptr, k);
  }

  // Gram-Schmidt sweeps over nv basis vectors with NG >= nv register accumulators;
  // the update sweep forms the next pass's dot products while nv <= kKrFuse
  static constexpr int kKrFuse = 32;
  // call fn with std::integral_constant<int, NG>, NG the register block for nv
  // basis vectors: nv rounded up to a multiple of 4 (of 8 above 32)
  template <class F>
  static void kr_ng(int nv, F&& fn) {
    using std::integral_constant;
    switch ((nv + 3) / 4) {
      case 1: fn(integral_constant<int, 4>{}); break;
      case 2: fn(integral_constant<int, 8>{}); break;
      case 3: fn(integral_constant<int, 12>{}); break;
      case 4: fn(integral_constant<int, 16>{}); break;
      case 5: fn(integral_constant<int, 20>{}); break;
      case 6: fn(integral_constant<int, 24>{}); break;
      case 7: fn(integral_constant<int, 28>{}); break;
      case 8: fn(integral_constant<int, 32>{}); break;
      case 9: case 10: fn(integral_constant<int, 40>{}); break;
      case 11: case 12: fn(integral_constant<int, 48>{}); break;
      case 13: case 14: fn(integral_constant<int, 56>{}); break;
      default: fn(integral_constant<int, 64>{}); break;
    }
  }
  template <int NG>
  void kr_dot_ng(const Kr& k, int nv, const double* w, long wrs, const int* skip, hipStream_t st) {
    hipLaunchKernelGGL((k_kr_dot<NG>), dim3(k.nblk), dim3(256), 0, st, pl.lv[0].n, B(), k.lbk, k.chunk, nv,
                       (const double*)k.V, k.m + 1, (const double*)k.S.sig, w, wrs, k.part, skip);
  }
  template <int NG, bool DOTS>
  void kr_upd_ng(const Kr& k, int nv, const double* h, const double* wi, long wis, double* wo, long wos,
                 const int* skip, hipStream_t st) {
    hipLaunchKernelGGL((k_kr_upd<NG, TU, DOTS>), dim3(k.nblk), dim3(256), 0, st, pl.lv[0].n, B(), k.lbk, k.chunk,
                       nv, (const double*)k.V, k.m + 1, (const double*)k.S.sig, h, wi, wis, wo, wos, r0, k.part,
                       skip);
  }
  // out[0..nv) = <w, v_t>, out[nv] = ||w||^2 (per column; zero when skipped)
  mg_status kr_dot(const Kr& k, int nv, const double* w, long wrs, double* out, const int* skip, hipStream_t st) {
    const int l = skip ? -2 : 0;
    TIMED(MG_KF_KRYLOV, nB(0) * 8.0 * (nv + 1), kr_ng(nv, [&](auto ng) {
            kr_dot_ng<decltype(ng)::value>(k, nv, w, wrs, skip, st);
          }));
    hipLaunchKernelGGL(k_kr_reduce, dim3(nv + 1), dim3(1024), 0, st, (const double*)k.part, k.nblk, nv + 1, B(),
                       k.lbk, out, skip);
    LAUNCH_OK();
    return MG_OK;
  }
  // wo = wi - sum_t h_t v_t, r0 = fl(wo); dots: out[0..nv) = <wo, v_t>, out[nv] = ||wo||^2,
  // else out[0] = ||wo||^2 (zero when skipped)
  // (the conditional second pass is not timed: whether it ran is known only on the device)
  mg_status kr_upd(const Kr& k, int nv, const double* h, const double* wi, long wis, double* wo, long wos,
                   bool dots, double* out, const int* skip, hipStream_t st) {
    const int l = skip ? -2 : 0;
    TIMED(MG_KF_KRYLOV, nB(0) * (8.0 * (nv + 2) + sizeof(TU)), kr_ng(nv, [&](auto ng) {
            constexpr int NG = decltype(ng)::value;
            if constexpr (NG <= kKrFuse) {
              if (dots) kr_upd_ng<NG, true>(k, nv, h, wi, wis, wo, wos, skip, st);
              else kr_upd_ng<NG, false>(k, nv, h, wi, wis, wo, wos, skip, st);
            } else {
              kr_upd_ng<NG, false>(k, nv, h, wi, wis, wo, wos, skip, st);
            }
          }));
    const int rows = dots ? nv + 1 : 1;
    hipLaunchKernelGGL(k_kr_reduce, dim3(rows), dim3(1024), 0, st, (const double*)k.part, k.nblk, rows, B(), k.lbk,
                       out, skip);
    LAUNCH_OK();
    return MG_OK;
  }
  mg_status kr_count(const Kr& k, int* cnt, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(hcount, k.S.st + 3 * B(), sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *cnt = hcount[0];
    return MG_OK;
  }

  // Flexible GMRES(m) with right preconditioning (Saad 1993), per column, from
  // the given x.  The preconditioner z = C(v) runs in the cycle precision on
  // fl(v); A z, the basis and the iterate are FP64, so the Arnoldi relation
  // A Z_m = V_{m+1} H_m holds to FP64 rounding whatever C does.
  mg_status fgmres(const double* f, double* x, const mg_krylov_options* o, void* work, size_t wbytes,
                   mg_rhs_info* info, hipStream_t st) override {
    if (pl.nv) return fail(MG_ERR_UNSUPPORTED, "FGMRES with per-column operators is not built");
    const int m = o->restart, Bn = B(), n0 = pl.lv[0].n;
    const long n0B = (long)n0 * Bn;
    Kr k;
    const size_t need = kr_carve(m, nullptr, k);
    char* base = nullptr;
    if (work) {
      if (wbytes < need) return fail(MG_ERR_OOM, "Krylov workspace too small: need " + std::to_string(need) + " bytes");
      base = static_cast<char*>(work);
    } else {
      if (kr_own_bytes < need) {
        if (kr_own) {
          HIP_TRY(hipStreamSynchronize(st));
          HIP_TRY(hipFree(kr_own));
          kr_own = nullptr;
          kr_own_bytes = 0;
        }
        if (hipMalloc(&kr_own, need) != hipSuccess) {
          (void)hipGetLastError();
          kr_own = nullptr;
          return fail(MG_ERR_OOM, "cannot allocate " + std::to_string(need) + " bytes of Krylov workspace");
        }
        kr_own_bytes = need;
      }
      base = kr_own;
    }
    kr_carve(m, base, k);
    const unsigned eb = d[0].blocks;
    // ||f|| (the residual of x = 0) fixes the stopping threshold and clears the totals
    hipLaunchKernelGGL((k_fill0<double>), dim3(nblocks(n0B)), dim3(256), 0, st, n0B, dbuf);
    LAUNCH_OK();
    MG_TRY(outer_resid<TU>(f, dbuf, nullptr, (TU*)nullptr, k.beta, st));
    hipLaunchKernelGGL(k_kr_start, dim3(1), dim3(256), 0, st, k.S, Bn, (const double*)k.beta, o->rtol, 1);
    LAUNCH_OK();
    int total = 0, cnt = 0;
    for (;;) {
      // vt_0 = f - A x (FP64) and its cycle-type copy, the first preconditioner input
      MG_TRY(outer_resid<TU>(f, x, k.w, r0, k.beta, st));
      hipLaunchKernelGGL(k_kr_put0, dim3(eb), dim3(256), 0, st, n0, Bn, lbs, (const double*)k.w, k.V, m + 1);
      LAUNCH_OK();
      hipLaunchKernelGGL(k_kr_start, dim3(1), dim3(256), 0, st, k.S, Bn, (const double*)k.beta, o->rtol, 0);
      LAUNCH_OK();
      MG_TRY(kr_count(k, &cnt, st));
      if (cnt == 0 || total >= o->max_iter) break;
      int j = 0;
      while (j < m && total < o->max_iter) {
        TU* zj = k.Z + (size_t)j * k.zs;
        switch (o->precond) {
          case MG_PC_NONE: MG_TRY(copy((const TU*)r0, zj, n0B, st)); break;
          case MG_PC_VCYCLE: MG_TRY(fwd(0, r0, zj, 1, nullptr, st)); break;
          default: MG_TRY(fmg(r0, zj, st)); break;
        }
        // w = A z_j with z_j = sig_j zt_j
        ROWS_LAUNCH(d[0], k_kr_amul, (TU), L64, Bn, lbs, (const TU*)zj, (const double*)(k.S.sig + (size_t)j * Bn),
                    k.w);
        LAUNCH_OK();
        const int nv = j + 1;
        double* vn = k.V + (size_t)(j + 1) * Bn;     // basis slot j + 1 (row stride (m + 1) B)
        const long vrs = (long)(m + 1) * Bn;
        // classical Gram-Schmidt; the second pass is applied only where needed
        MG_TRY(kr_dot(k, nv, k.w, Bn, k.h1, nullptr, st));
        const bool fuse = nv <= kKrFuse;
        const double* n2 = fuse ? k.h2 + (size_t)nv * Bn : k.n2;
        MG_TRY(kr_upd(k, nv, k.h1, k.w, Bn, vn, vrs, fuse, fuse ? k.h2 : k.n2, nullptr, st));
        hipLaunchKernelGGL(k_kr_reorth, dim3(1), dim3(256), 0, st, k.S, Bn, (const double*)(k.h1 + (size_t)nv * Bn),
                           n2, o->reorth * o->reorth);
        LAUNCH_OK();
        if (!fuse) MG_TRY(kr_dot(k, nv, vn, vrs, k.h2, k.S.flag, st));
        MG_TRY(kr_upd(k, nv, k.h2, vn, vrs, vn, vrs, false, k.n4, k.S.flag, st));
        hipLaunchKernelGGL(k_kr_givens, dim3(1), dim3(256), 0, st, k.S, Bn, j, (const double*)k.h1,
                           (const double*)k.h2, n2, (const double*)k.n4, o->rtol);
        LAUNCH_OK();
        ++j;
        ++total;
        MG_TRY(kr_count(k, &cnt, st));
        if (cnt == 0) break;
      }
      hipLaunchKernelGGL(k_kr_lsq, dim3(1), dim3(256), 0, st, k.S, Bn, j, k.y);
      LAUNCH_OK();
      hipLaunchKernelGGL((k_kr_xupd<TU>), dim3(eb), dim3(256), 0, st, n0, Bn, lbs, j, (const TU*)k.Z, k.zs,
                         (const double*)k.y, x);
      LAUNCH_OK();
    }
    // fixed-size host buffers (B <= kMaxB): the solve allocates nothing when the caller brings the workspace
    int hst[3 * kMaxB + 1];
    double hb[kMaxB], hf[kMaxB];
    HIP_TRY(hipMemcpyAsync(hst, k.S.st, (3 * (size_t)Bn + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hb, k.beta, Bn * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hf, k.S.fnorm, Bn * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    mg_status ret = MG_OK;
    for (int b = 0; b < Bn; ++b) {
      const int s = hst[2 * Bn + b];
      if (info) {
        info[b].iters = hst[Bn + b];
        info[b].status = s;
        info[b].relres = hf[b] > 0 ? hb[b] / hf[b] : hb[b];
      }
      if (s == MG_ERR_DIVERGED) ret = MG_ERR_DIVERGED;
      else if (s != MG_OK && ret == MG_OK) ret = MG_ERR_NOT_CONVERGED;
    }
    if (ret != MG_OK) g_err = ret == MG_ERR_DIVERGED ? "a column's residual is not finite" : "a column did not converge";
    return ret;
  }

  // ---------------------------------------------------------------- reverse sweep
  int slot = 0;

  // z_0 = src, z_k = M^T z_{k-1};  acc = sum_k c_k z_k;  dot slots <z_k, sdot>
  mg_status chainT(int l, const double* c, int K, const TU* src, const void* sdot, bool sdot_is_TH, hipStream_t st) {
    const DL& D = d[l];
    TU* zbuf[2] = {D.za, D.zb};
    const TU* zprev = src;
    int cur = 0;
    for (int k = 0; k <= K; ++k) {
      if (slot >= nslots) return fail(MG_ERR_STATE, "reverse sweep slot overflow");
      double* pp = dpart + h_off[slot];
      TU* zout = (k >= 1 && k < K) ? zbuf[cur] : nullptr;
      const TU* zin = k == 0 ? nullptr : zprev;
      const TU* zsrc = k == 0 ? src : nullptr;
      if (sdot_is_TH)
        WG_SPLIT(ROWS_LAUNCH(D, k_hopT, (WGv, C, TU, TH), D.L, B(), lbs, zin, zsrc, zout,
                             (C)c[k], D.acc, k == 0 ? 1 : 0, static_cast<const TH*>(sdot), pp));
      else
        WG_SPLIT(ROWS_LAUNCH(D, k_hopT, (WGv, C, TU, TU), D.L, B(), lbs, zin, zsrc, zout,
                             (C)c[k], D.acc, k == 0 ? 1 : 0, static_cast<const TU*>(sdot), pp));
      LAUNCH_OK();
      ++slot;
      if (zout) {
        zprev = zout;
        cur ^= 1;
      }
    }
    return MG_OK;
  }

  // reverse of one smoothing step whose Jacobi residual was s: g <- g - A q, gf += q
  mg_status smoothT(int l, const TH* s, TU* g, TU* gf, int& gfz, hipStream_t st) {
    const DL& D = d[l];
    MG_TRY(chainT(l, cB(l), pl.KB, g, s, true, st));
    hipLaunchKernelGGL((k_scale_acc<C, TU>), dim3(D.blocks), dim3(256), 0, st, D.L, B(), lbs, (const TU*)D.acc,
                       (C)(eta(l) * theta(l)), 1, D.q, gf, gfz);
    LAUNCH_OK();
    gfz = 0;
    ROWS_LAUNCH(D, k_sub_Aq, (C, TU), D.L, B(), lbs, (const TU*)g,
                       (const TU*)D.q, g);
    LAUNCH_OK();
    return MG_OK;
  }

  // reverse of level l: gout = dL/du_out; writes gfl = dL/df_l, gul = dL/du_in (optional)
  mg_status bwd_level(int l, const TU* f, const TU* uin, const TU* gout, TU* gfl, TU* gul, const Ck& ck,
                      hipStream_t st) {
    const long nB = (long)pl.lv[l].n * B();
    if (l == pl.J - 1) {
      MG_TRY(coarse(gout, gfl, 1, st));
      if (gul) {
        hipLaunchKernelGGL((k_fill0<TU>), dim3(nblocks(nB)), dim3(256), 0, st, nB, gul);
        LAUNCH_OK();
      }
      return MG_OK;
    }
    DL& D = d[l];
    // forward recomputation of this level from its checkpoint
    int uz = uin ? 0 : 1;
    if (uin) MG_TRY(copy(uin, D.ut, nB, st));
    for (int j = 0; j < pl.nu_pre; ++j) {
      MG_TRY(smooth(l, f, D.ut, uz, D.S[j], st));
      uz = 0;
    }
    ROWS_LAUNCH_F(D, l == 0, k_resid, (false, C, TU, TU), D.L, B(), lbs, f, (const TU*)D.ut, uz,
                       0, D.Rv);
    LAUNCH_OK();
    const TU* ec = ck.u[l + 1];
    ROWS_LAUNCH(D, k_prolong, (C, TU, TH), D.P, B(), lbs, ec, D.X, 0, (C)1, 0);
    LAUNCH_OK();
    MG_TRY(prolong(l, ec, D.ut, uz, D.x, st));
    for (int j = 0; j < pl.nu_post; ++j) MG_TRY(smooth(l, f, D.ut, 0, D.S[pl.nu_pre + j], st));
    // reverse
    MG_TRY(copy(gout, D.g, nB, st));
    int gfz = 1;
    for (int j = pl.nu_post - 1; j >= 0; --j) MG_TRY(smoothT(l, D.S[pl.nu_pre + j], D.g, gfl, gfz, st));
    // correction u += Phi_P(P ec):  dL/d ec = P^T Phi_P^T g
    MG_TRY(chainT(l, cP(l), pl.KP, D.g, D.X, true, st));
    DL& Dn = d[l + 1];
    ROWS_LAUNCH(Dn, k_prolong, (C, TU, TU), D.PT, B(), lbs, (const TU*)D.acc,
                       Dn.gin, 0, (C)1, 0);
    LAUNCH_OK();
    MG_TRY(bwd_level(l + 1, ck.f[l + 1], nullptr, Dn.gin, Dn.gfo, nullptr, ck, st));
    // restriction rc = R Phi_R(r):  r_bar = Phi_R^T R^T rc_bar
    ROWS_LAUNCH(D, k_prolong, (C, TU, TU), D.RT, B(), lbs, (const TU*)Dn.gfo, D.q,
                       0, (C)1, 0);
    LAUNCH_OK();
    MG_TRY(chainT(l, cR(l), pl.KR, D.q, D.Rv, false, st));
    hipLaunchKernelGGL((k_scale_acc<C, TU>), dim3(D.blocks), dim3(256), 0, st, D.L, B(), lbs, (const TU*)D.acc, (C)1,
                       0, D.q, gfl, gfz);
    LAUNCH_OK();
    gfz = 0;
    ROWS_LAUNCH(D, k_sub_Aq, (C, TU), D.L, B(), lbs, (const TU*)D.g,
                       (const TU*)D.q, D.g);
    LAUNCH_OK();
    for (int j = pl.nu_pre - 1; j >= 0; --j) MG_TRY(smoothT(l, D.S[j], D.g, gfl, gfz, st));
    if (gul) MG_TRY(copy((const TU*)D.g, gul, nB, st));
    return MG_OK;
  }

  mg_status finish_grads(double* gp, hipStream_t st) {
    if (slot != nslots) return fail(MG_ERR_STATE, "reverse sweep slot count mismatch");
    if (!gp) return MG_OK;
    hipLaunchKernelGGL(k_dots_final, dim3(nslots), dim3(256), 0, st, dpart, doff, dcnt, nslots, dots);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_grad_combine, dim3(1), dim3(1), 0, st, dots, ddesc, nslots, dprm, per(), pl.KB, pl.KR, gp,
                       (int)pl.params.size());
    LAUNCH_OK();
    if (pl.basis == MG_BASIS_CHEBYSHEV) {
      hipLaunchKernelGGL(k_cheb_grad, dim3(1), dim3(64), 0, st, gp, pl.J - 1, per(), pl.KB, pl.KR, pl.KP,
                         cheb_table());
      LAUNCH_OK();
    }
    return MG_OK;
  }

  mg_status bwd_ok() {
    if (!bwd()) return fail(MG_ERR_STATE, "context was set up without MG_FLAG_BACKWARD");
    if (!pl.sym_all) return fail(MG_ERR_UNSUPPORTED, "reverse sweep needs symmetric A_l and graphs");
    return MG_OK;
  }

  mg_status vcycle_bwd(const void* ckv, const void* goutv, void* ginv, void* gfv, double* gp, hipStream_t st) override {
    MG_TRY(bwd_ok());
    if (!ckv || !goutv) return fail(MG_ERR_INVALID_ARG, "checkpoint and gu_out are required");
    Ck ck = ck_ptrs(const_cast<void*>(ckv));
    slot = 0;
    TU* gf = gfv ? static_cast<TU*>(gfv) : d[0].gfo;
    MG_TRY(bwd_level(0, ck.f[0], ck.u[0], static_cast<const TU*>(goutv), gf, static_cast<TU*>(ginv), ck, st));
    return finish_grads(gp, st);
  }

  mg_status refine_bwd(const void* ckv, const double* gout, double* gin, double* gf, double* gp, hipStream_t st) override {
    MG_TRY(bwd_ok());
    if (!ckv || !gout) return fail(MG_ERR_INVALID_ARG, "checkpoint and gu_out are required");
    Ck ck = ck_ptrs(const_cast<void*>(ckv));
    const long n0B = (long)pl.lv[0].n * B();
    slot = 0;
    MG_TRY(copy(gout, d[0].gin, n0B, st));
    MG_TRY(bwd_level(0, ck.f[0], nullptr, d[0].gin, d[0].gfo, nullptr, ck, st));
    MG_TRY(copy((const TU*)d[0].gfo, dbuf, n0B, st));
    if (gf) MG_TRY(copy((const double*)dbuf, gf, n0B, st));
    if (gin) {
      ROWS_LAUNCH(d[0], k_sub_Aq, (double, double), L64, B(), lbs, gout,
                         (const double*)dbuf, gin);
      LAUNCH_OK();
    }
    return finish_grads(gp, st);
  }
};

}  // namespace

struct mg_ctx {
  std::unique_ptr<EngineBase> e;
};

namespace {

// Krylov workspace of the allocation-free entry point mg_fgmres_static: a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes `scratch` itself to a kernel or a copy (in host code
// the name is only a stand-in for the symbol): it uses the device address
// that hipGetSymbolAddress returns for the current device, taken once per
// device at the library's set-up (mg_setup) or on the entry point's first call
// on a device.
constexpr size_t kStaticScratchBytes = (size_t)MG_FGMRES_STATIC_MAX_BYTES;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of the current device's copy of `scratch`
mg_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MG_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MG_ERR_HIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MG_OK;
}

}  // namespace

static EngineBase* make_engine(int prec) {
  switch (prec) {
    case MG_FP64: return new Engine<double, double, double>();
    case MG_FP32: return new Engine<float, float, float>();
    default: return new Engine<float, float, bf16_t>();
  }
}

extern "C" {

int64_t mg_num_params(int32_t nlevels, int32_t KB, int32_t KR, int32_t KP) {
  if (nlevels < 2 || KB < 0 || KR < 0 || KP < 0) return -1;
  return num_params(nlevels, KB, KR, KP);
}

mg_status mg_workspace_bytes(const mg_hierarchy* h, const mg_params* p, const mg_options* o, size_t* ws, size_t* ck) {
  g_err.clear();
  std::unique_ptr<EngineBase> e(make_engine(o ? o->precision : 0));
  MG_TRY(build_plan(h, p, o, e->pl, false));
  if (ws) *ws = e->ws_bytes();
  if (ck) *ck = e->ck_bytes();
  return MG_OK;
}

mg_status mg_setup(const mg_hierarchy* h, const mg_params* p, const mg_options* o, void* ws, size_t ws_bytes,
                   void* stream, mg_ctx** out) {
  g_err.clear();
  if (!out) return fail(MG_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  const ActiveCall guard;
  std::unique_ptr<EngineBase> e(make_engine(o ? o->precision : 0));
  MG_TRY(build_plan(h, p, o, e->pl, true));
  const size_t need = e->ws_bytes();
  if (ws && ws_bytes < need)
    return fail(MG_ERR_OOM, "workspace too small: need " + std::to_string(need) + " bytes");
  MG_TRY(e->setup(ws, static_cast<hipStream_t>(stream)));
  // once per device: the static scratch's address on this device (mg_fgmres_static retries on
  // its first call if this fails; no other entry point needs it)
  void* sp = nullptr;
  if (scratch_address(&sp) != MG_OK) {
    (void)hipGetLastError();
    g_err.clear();
  }
  mg_ctx* c = new mg_ctx;
  c->e = std::move(e);
  *out = c;
  return MG_OK;
}

mg_status mg_set_params(mg_ctx* c, const double* v, void* stream) {
  g_err.clear();
  if (!c || !v) return fail(MG_ERR_INVALID_ARG, "null argument");
  return c->e->set_params(v, static_cast<hipStream_t>(stream));
}

mg_status mg_load_column(mg_ctx* c, int32_t b, const double* const* values, void* stream) {
  g_err.clear();
  if (!c) return fail(MG_ERR_INVALID_ARG, "null context");
  return c->e->load_column(b, values, static_cast<hipStream_t>(stream));
}

mg_status mg_set_solver_options(mg_ctx* c, int32_t max_outer, int32_t check_every, double rtol,
                                double diverge_factor) {
  g_err.clear();
  if (!c) return fail(MG_ERR_INVALID_ARG, "null context");
  if (max_outer < 1 || check_every < 1 || !(rtol >= 0.0))
    return fail(MG_ERR_INVALID_ARG, "max_outer and check_every must be >= 1, rtol >= 0");
  c->e->pl.max_outer = max_outer;
  c->e->pl.check_every = check_every;
  c->e->pl.rtol = rtol;
  c->e->pl.divf = diverge_factor;
  return MG_OK;
}

mg_status mg_vcycle(mg_ctx* c, const void* f, void* u, void* ckpt, void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  return c->e->vcycle(f, u, ckpt, static_cast<hipStream_t>(stream));
}

mg_status mg_vcycle_backward(mg_ctx* c, const void* ckpt, const void* gu_out, void* gu_in, void* gf, double* gp,
                             void* stream) {
  g_err.clear();
  if (!c) return fail(MG_ERR_INVALID_ARG, "null context");
  return c->e->vcycle_bwd(ckpt, gu_out, gu_in, gf, gp, static_cast<hipStream_t>(stream));
}

mg_status mg_residual(mg_ctx* c, const double* f, const double* u, double* r, double* norms, void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  return c->e->residual(f, u, r, norms, static_cast<hipStream_t>(stream));
}

mg_status mg_residual_loss(mg_ctx* c, int32_t kind, const double* f, const double* u, const double* gseed,
                           double* loss, double* gu, double* gf, void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  if ((gu && (gu == u || gu == f)) || (gf && (gf == u || gf == f)) || (gu && gu == gf))
    return fail(MG_ERR_INVALID_ARG, "gradient outputs must not overlap f, u or each other");
  return c->e->residual_loss(kind, f, u, gseed, loss, gu, gf, static_cast<hipStream_t>(stream));
}

mg_status mg_refine_step(mg_ctx* c, const double* f, const double* uin, double* uout, void* ckpt, void* stream) {
  g_err.clear();
  if (!c || !f || !uin || !uout) return fail(MG_ERR_INVALID_ARG, "null argument");
  return c->e->refine(f, uin, uout, ckpt, static_cast<hipStream_t>(stream));
}

mg_status mg_refine_step_backward(mg_ctx* c, const void* ckpt, const double* gout, double* gin, double* gf, double* gp,
                                  void* stream) {
  g_err.clear();
  if (!c) return fail(MG_ERR_INVALID_ARG, "null context");
  return c->e->refine_bwd(ckpt, gout, gin, gf, gp, static_cast<hipStream_t>(stream));
}

mg_status mg_solve(mg_ctx* c, const double* f, double* u, mg_rhs_info* info, void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  return c->e->solve(f, u, info, static_cast<hipStream_t>(stream));
}

mg_status mg_fmg(mg_ctx* c, const void* f, void* u, void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  return c->e->fmg_entry(f, u, static_cast<hipStream_t>(stream));
}

static mg_status check_krylov(const mg_krylov_options* o) {
  if (!o) return fail(MG_ERR_INVALID_ARG, "null Krylov options");
  if (o->restart < 1 || o->restart > 63) return fail(MG_ERR_INVALID_ARG, "restart must be in 1..63");
  if (o->max_iter < 1) return fail(MG_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(o->rtol >= 0.0)) return fail(MG_ERR_INVALID_ARG, "rtol must be >= 0");
  if (o->precond < MG_PC_NONE || o->precond > MG_PC_FMG) return fail(MG_ERR_INVALID_ARG, "unknown preconditioner");
  if (!(o->reorth >= 0.0)) return fail(MG_ERR_INVALID_ARG, "reorth must be >= 0");
  return MG_OK;
}

mg_status mg_fgmres_workspace_bytes(const mg_ctx* c, const mg_krylov_options* o, size_t* bytes) {
  g_err.clear();
  if (!c || !bytes) return fail(MG_ERR_INVALID_ARG, "null argument");
  MG_TRY(check_krylov(o));
  *bytes = c->e->fgmres_bytes(o->restart);
  return MG_OK;
}

mg_status mg_fgmres(mg_ctx* c, const double* f, double* u, const mg_krylov_options* o, void* work, size_t work_bytes,
                    mg_rhs_info* info, void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  MG_TRY(check_krylov(o));
  return c->e->fgmres(f, u, o, work, work_bytes, info, static_cast<hipStream_t>(stream));
}

mg_status mg_fgmres_static(mg_ctx* c, const double* f, double* u, const mg_krylov_options* o, mg_rhs_info* info,
                           void* stream) {
  g_err.clear();
  if (!c || !f || !u) return fail(MG_ERR_INVALID_ARG, "null argument");
  MG_TRY(check_krylov(o));
  const size_t need = c->e->fgmres_bytes(o->restart);
  if (need > kStaticScratchBytes)
    return fail(MG_ERR_OOM, "Krylov workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                                std::to_string(kStaticScratchBytes) + " bytes");
  void* sp = nullptr;
  MG_TRY(scratch_address(&sp));
  return c->e->fgmres(f, u, o, sp, kStaticScratchBytes, info, static_cast<hipStream_t>(stream));
}

mg_status mg_level_info(const mg_ctx* c, int64_t* n, int32_t* wA) {
  g_err.clear();
  if (!c || !n) return fail(MG_ERR_INVALID_ARG, "null argument");
  for (size_t l = 0; l < c->e->sizes.size(); ++l) {
    n[l] = c->e->sizes[l];
    if (wA) wA[l] = c->e->widths[l];
  }
  return MG_OK;
}

mg_status mg_timing_start(mg_ctx* c, int32_t fam, int32_t level) {
  g_err.clear();
  if (!c || fam < MG_KF_NONE || fam > MG_KF_CONV) return fail(MG_ERR_INVALID_ARG, "bad context or kernel family");
  return c->e->timing_start(fam, level);
}

mg_status mg_timing_read(mg_ctx* c, int64_t* n, double* ms, double* bytes) {
  g_err.clear();
  if (!c) return fail(MG_ERR_INVALID_ARG, "null context");
  return c->e->timing_read(n, ms, bytes);
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  delete c;
}

const char* mg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
