// Host-side check of the fused convolution's tiling (csrc/tiles.hpp).
//
// Usage: tiles_check GRAPH KM SIDE
// GRAPH is a binary file: int32 n, int32 w, then the slot-major column array
// col[k * n + i] (k < w, padding col == i).  The program builds the tiles,
// runs the library's invariant check, and emulates the fused convolution
// (every hop of Phi(x) = sum_k c_k M^k x computed per tile from the tile's
// lists, M the neighbour mean) against the same hops applied to the whole
// graph, in double precision, for K = 2 .. KM.  Prints one line:
//   ok <tiles> <listed/n> <max |difference|> <own-node coverage>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "tiles.hpp"

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  FILE* fp = std::fopen(argv[1], "rb");
  if (!fp) return 2;
  int n = 0, w = 0;
  if (std::fread(&n, 4, 1, fp) != 1 || std::fread(&w, 4, 1, fp) != 1) return 2;
  std::vector<int> col((size_t)n * w);
  if (std::fread(col.data(), 4, col.size(), fp) != col.size()) return 2;
  std::fclose(fp);
  const int KM = std::atoi(argv[2]), side = std::atoi(argv[3]);
  mgl::TilePlan tp;
  if (!mgl::build_tiles(n, n, w, col.data(), KM, side, side, tp)) { std::printf("build-failed\n"); return 1; }
  if (!mgl::check_tiles(n, n, col.data(), tp)) { std::printf("check-failed\n"); return 1; }
  std::vector<double> x(n), idg(n);
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (double& v : x) v = U(rng);
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int k = 0; k < w; ++k) c += col[(size_t)k * n + i] != i;
    idg[i] = c ? 1.0 / c : 0.0;
  }
  double maxerr = 0.0;
  std::vector<int> covered(n, 0);
  for (int K = 2; K <= KM; ++K) {
    std::vector<double> c(K + 1);
    for (double& v : c) v = U(rng);
    // whole graph: Horner in M
    std::vector<double> y(x), y2(n);
    double a = c[K];
    for (int k = K - 1; k >= 0; --k) {
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = 0; q < w; ++q) {
          const int j = col[(size_t)q * n + i];
          if (j != i) s += y[j];
        }
        y2[i] = a * (idg[i] * s) + c[k] * x[i];
      }
      y.swap(y2);
      a = 1.0;
    }
    // per tile, from the tile's lists only
    for (int t = 0; t < tp.ntiles; ++t) {
      const int* nd = &tp.node[tp.toff[t]];
      const int* cn = &tp.cnt[(size_t)t * (KM + 1)];
      const uint16_t* lc = &tp.lcol[tp.goff[t]];
      std::vector<double> S(cn[K]), Y(cn[K]), Yn(cn[K]);
      for (int r = 0; r < cn[K]; ++r) S[r] = x[nd[r]];
      const std::vector<double>* yin = &S;
      for (int h = 1; h <= K; ++h) {
        const double aa = h == 1 ? c[K] : 1.0;
        const int rows = cn[K - h];
        for (int r = 0; r < rows; ++r) {
          double s = 0.0;
          for (int q = 0; q < tp.wg; ++q) {
            const int e = lc[(size_t)r * tp.wg + q];   // local column + 1, 0: padding
            if (e == 0) continue;
            const int j = e - 1;
            if (j >= cn[K - h + 1] || j == r) { std::printf("local-column-out-of-range\n"); return 1; }
            s += (*yin)[j];
          }
          Yn[r] = aa * (idg[nd[r]] * s) + c[K - h] * S[r];
        }
        Y.swap(Yn);
        yin = &Y;
      }
      for (int r = 0; r < cn[0]; ++r) {
        maxerr = std::max(maxerr, std::fabs(Y[r] - y[nd[r]]));
        if (K == 2) ++covered[nd[r]];
      }
    }
  }
  int once = 0;
  for (int v : covered) once += v == 1;
  std::printf("ok %d %.4f %.3e %d\n", tp.ntiles, (double)tp.toff[tp.ntiles] / n, maxerr, once == n ? 1 : 0);
  return 0;
}
