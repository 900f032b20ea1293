// Unit-cell context shared by the cell move (cell.hip) and its adjoint
// (cell_ad.hip); internal.
#pragma once

#include "../../include/ctm.h"

#include <rocblas/rocblas.h>

#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "tape.h"

namespace sictm {

constexpr int kCellMaxSide = 16;
constexpr int kCutsPerLaunch = 4;   // X and Y blocks of 4 cuts = 8 problems

inline int imod(int a, int m) { return ((a % m) + m) % m; }

// Environment of one site: tensor pointers and dimensions (rows, cols of the
// corners; in, out of the edges, whose middle leg has the network's Dl).
struct SiteEnv {
  double* C[4];
  double* T[4];
  int Cd[4][2];
  int Td[4][2];
};

}  // namespace sictm

struct ctm_cell {
  ctm_cell_config cfg;
  int Lx = 0, Ly = 0, ns = 0, Dl = 0, chi = 0, k = 0, Nf = 0, Lmax = 0;
  hipStream_t st = nullptr;
  rocblas_handle rb = nullptr;
  char* mem = nullptr;
  std::vector<std::pair<uintptr_t, uintptr_t>> bufs;
  std::string err;
  // sites
  std::vector<double*> A, a, ap, apr;   // ap, apr: [site * 4 + corner]
  std::vector<sictm::SiteEnv> env;
  std::vector<double*> spare;           // [Lmax * 3] targets of the new tensors of a column
  // blocks [dir * ns + cut]: start blocks (X0, Y0) and current ones (X, Y)
  std::vector<double*> X0, Y0, X, Y;
  bool blocks_set = false;              // X0, Y0 hold start blocks
  bool cur_set = false;                 // X, Y hold blocks set with a state
  int last_mode = -1;
  // per-cut work of a column step
  std::vector<double*> Q, Wst, CT;      // [Lmax * 4]
  std::vector<double*> B;               // [Lmax * 6] N x k blocks
  std::vector<double*> rho, u, v, vs, s, sg, vsc, usc, Pl, Prt, Z1, Z2;   // [Lmax]
  std::vector<double*> F;               // full SVD: R, L, M, Ut, Uv, U sorted, Vt sorted, Us, Vs
  double *fs = nullptr, *fE = nullptr, *fsg = nullptr;
  int *finfo = nullptr, *fperm = nullptr;
  // spectra
  std::vector<double*> cpad, csv;       // [ns * 4]
  double* spec[2] = {nullptr, nullptr};
  int spec_cur = 0;
  double* bvec = nullptr;               // [ns][4][Dl] boundary vectors of the initial environment
  double* scal = nullptr;               // [0..63] norms, [64..64+ns) per-site delta
  int* bad = nullptr;
  double* norm_part = nullptr;
  void* qr_ws = nullptr;
  void* svd_ws = nullptr;
  double* sk_part = nullptr;
  long iterations = 0;
  // adjoint: the tape of the last adjoint call (kept for its memory)
  std::unique_ptr<sictm::Tape> tape;
};

namespace sictm {

// Row-major float64 GEMM descriptor without problems (add them with add()).
inline GemmBatch gemm_of(int M, int N, int K, long lda, long ldb, long ldc) {
  GemmBatch g{};
  g.count = 0;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  gemm_set_rowmajor_c(g, ldc);
  g.nbatch = 1;
  g.alpha = 1.0;
  return g;
}

inline void add(GemmBatch& g, const double* A, const double* B, double* C, int transA = 0) {
  g.A[g.count] = A;
  g.B[g.count] = B;
  g.C[g.count] = C;
  g.transA[g.count] = transA;
  ++g.count;
}

// the turned cell
inline int width(const ctm_cell* c, int d) { return (d & 1) ? c->Ly : c->Lx; }
inline int height(const ctm_cell* c, int d) { return (d & 1) ? c->Lx : c->Ly; }

// Site of the cell at (x', y') of the cell turned d times (one turn maps
// site (x, y) of a cell of width w to (y, w - 1 - x)).
inline int site_of(const ctm_cell* c, int d, int xt, int yt) {
  int x = imod(xt, width(c, d)), y = imod(yt, height(c, d));
  for (int t = d; t >= 1; --t) {
    const int w_prev = ((t - 1) & 1) ? c->Ly : c->Lx;
    const int xp = w_prev - 1 - y, yp = x;
    x = xp;
    y = yp;
  }
  return y * c->Lx + x;
}

}  // namespace sictm
