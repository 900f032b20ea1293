// Tall-skinny Householder QR with explicit Q (QR-based projector section,
// step 1: the isometries are re-orthonormalised by a QR decomposition after
// the power update).
//
// Communication-avoiding layout for N x k blocks with N >> k:
//  * the rows are split into `nb` leaves of at most kLeafRows rows (leaf 0
//    holds at least k rows); the columns are processed in panels of width
//    kPanel;
//  * per panel, every leaf factors its active rows of the panel with
//    Householder reflectors in LDS, forms the compact-WY factor T
//    (H_0...H_(w-1) = I - V T V^T) and updates its trailing columns with
//    C <- C - V T^T (V^T C), three small GEMMs on the FP64 matrix cores;
//  * the w x w triangles the leaves leave in their top rows are combined
//    pairwise up a binary tree; combining two upper triangles gives
//    reflectors [e_j; v] with v upper triangular, stored in the place of the
//    absorbed triangle, and their own WY factor updates the trailing columns
//    of the node's 2w rows;
//  * Q = prod_p L_p T_p [I; 0] is then formed by applying the tree and leaf
//    WY factors (C <- C - V T (V^T C)) in reverse order to [I_k; 0], on the
//    columns that can be non-trivial, and each column c is multiplied by
//    sign(R_cc) so that R has a non-negative diagonal.
// Reflectors follow the LAPACK dlarfg convention: beta = -sign(alpha) * norm,
// tau = (beta - alpha) / beta, and tau = 0 (H = I) when the part below the
// diagonal is exactly zero, so rank-deficient blocks never divide by zero.

#include "common.h"

namespace sictm {
namespace {

constexpr int kPanel = 32;
constexpr int kLeafRows = 256;
constexpr int kLR = kLeafRows + 1;   // odd row length: fragment reads hit distinct banks
constexpr int kT = kPanel + 1;   // padded row length of the small LDS matrices
constexpr int kTrail = 64;       // trailing columns per LDS chunk in the tree kernels

struct QrPlan {
  int N, k, nb, P, depth;
};

__host__ __device__ inline int leaf_start(int i, int N, int nb) {
  return (int)(((long)i * N) / nb);
}

__device__ __forceinline__ double wave_sum(double x) { return wave_sum64(x); }

// C(M x N) = sum_k A(m, k) B(k, n) for operands in LDS, on the FP64 matrix
// cores (v_mfma_f64_16x16x4: operand lane l -> (row l%16, k l/16), result
// element r -> (row l/16 + 4r, column l%16)).  16x16 blocks are dealt to the
// four wavefronts; `store(m, n, value)` receives every result element once.
template <typename FA, typename FB, typename FS>
__device__ __forceinline__ void lds_mm(int M, int N, int K, FA A, FB B, FS store, int wave,
                                       int lane) {
  const int bm = (M + 15) >> 4, bn = (N + 15) >> 4;
  for (int blk = wave; blk < bm * bn; blk += 4) {
    const int i0 = (blk / bn) << 4, j0 = (blk % bn) << 4;
    const int ar = i0 + (lane & 15), bc = j0 + (lane & 15);
    v4d acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    int k0 = 0;
    for (; k0 + 8 <= K; k0 += 8) {
      const int ka = k0 + (lane >> 4), kb = ka + 4;
      const double a0 = ar < M ? A(ar, ka) : 0.0;
      const double b0 = bc < N ? B(ka, bc) : 0.0;
      const double a1 = ar < M ? A(ar, kb) : 0.0;
      const double b1 = bc < N ? B(kb, bc) : 0.0;
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
    }
    for (; k0 < K; k0 += 4) {
      const int ka = k0 + (lane >> 4);
      const double a0 = (ar < M && ka < K) ? A(ar, ka) : 0.0;
      const double b0 = (bc < N && ka < K) ? B(ka, bc) : 0.0;
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + (lane >> 4) + 4 * r, col = j0 + (lane & 15);
      if (row < M && col < N) store(row, col, acc0[r] + acc1[r]);
    }
  }
}

// Global -> LDS copy with kInFlight independent loads per thread before the
// LDS stores: one workgroup per CU leaves nothing else to hide the latency.
constexpr int kInFlight = 8;
template <typename FL, typename FS>
__device__ __forceinline__ void g2l(int count, int tid, FL load, FS store) {
  for (int base = tid; base < count; base += 256 * kInFlight) {
    double t[kInFlight];
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      const int i = base + u * 256;
      t[u] = i < count ? load(i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      const int i = base + u * 256;
      if (i < count) store(i, t[u]);
    }
  }
}

struct QrArgs {
  double* A[kMaxProb];   // matrices being factored (in place)
  double* E[kMaxProb];   // explicit Q being formed
  double* O[kMaxProb];   // destination of Q
  double* tau;           // [count][P][nb][kPanel] leaf taus
  double* Tl;            // [count][P][nb][kPanel*kPanel] leaf WY factors
  double* Tn;            // [count][P][nb][kPanel*kPanel] tree WY factors (by right child)
  double* sgn;           // [count][k] signs of the diagonal of R
  int count, N, k, nb, P;
};

__device__ __forceinline__ long slot(int mat, int p, int leaf, int nb, int P) {
  return ((long)mat * P + p) * nb + leaf;
}

// T (w x w, upper) of H_0...H_(w-1) = I - V T V^T from the Gram matrix
// G = V^T V and the taus (forward, columnwise): T_jj = tau_j,
// T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].  One wavefront, lane i = row i.
__device__ __forceinline__ void build_T(double (*T)[kT], double (*G)[kT], const double* tau,
                                        int w, int lane) {
  for (int j = 0; j < w; ++j) {
    double t = 0.0;
    if (lane < j) {
      for (int l = lane; l < j; ++l) t += T[lane][l] * G[l][j];
      t *= -tau[j];
      T[lane][j] = t;
    }
    if (lane == j) T[j][j] = tau[j];
    if (lane > j && lane < kPanel) T[lane][j] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// leaf factorisation of panel p + WY update of its trailing columns
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void qr_leaf_factor(QrArgs q, int p) {
  __shared__ double V[kPanel][kLR];           // panel, column-major
  __shared__ double Cc[kPanel][kLR];          // trailing chunk, column-major
  __shared__ double T[kPanel][kT], G[kPanel][kT], W1[kPanel][kT];
  __shared__ double tau_s[kPanel];
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  double* A = q.A[mat];

  g2l(kPanel * kLeafRows, tid,
      [&](int idx) {
        const int r = idx / kPanel, c = idx % kPanel;
        return (r < m && c < w) ? A[(long)(a0 + r) * k + c0 + c] : 0.0;
      },
      [&](int idx, double v) { V[idx % kPanel][idx / kPanel] = v; });
  __syncthreads();

  for (int j = 0; j < w; ++j) {
    if (wave == 0) {
      double ss = 0.0;
      for (int r = j + 1 + lane; r < m; r += 64) ss += V[j][r] * V[j][r];
      ss = wave_sum(ss);
      const double alpha = V[j][j];
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      for (int r = j + 1 + lane; r < m; r += 64) V[j][r] *= scal;
      if (lane == 0) { V[j][j] = beta; tau_s[j] = tau; }
    }
    __syncthreads();
    const double tau = tau_s[j];
    if (tau != 0.0) {
      // all columns of this wavefront at once: the cross-lane reductions of
      // the (up to 8) dot products are independent and overlap
      double d[kPanel / 4];
#pragma unroll
      for (int t = 0; t < kPanel / 4; ++t) {
        const int c = j + 1 + wave + 4 * t;
        double acc = 0.0;
        if (c < w)
          for (int r = j + 1 + lane; r < m; r += 64) acc += V[j][r] * V[c][r];
        d[t] = acc;
      }
#pragma unroll
      for (int t = 0; t < kPanel / 4; ++t) d[t] = wave_sum64(d[t]);
#pragma unroll
      for (int t = 0; t < kPanel / 4; ++t) {
        const int c = j + 1 + wave + 4 * t;
        if (c < w) {
          const double f = tau * (d[t] + V[c][j]);
          for (int r = j + 1 + lane; r < m; r += 64) V[c][r] -= f * V[j][r];
          if (lane == 0) V[c][j] -= f;
        }
      }
    }
    __syncthreads();
  }

  for (int idx = tid; idx < m * w; idx += 256) {
    const int r = idx / w, c = idx % w;
    A[(long)(a0 + r) * k + c0 + c] = V[c][r];
  }
  const long sl = slot(mat, p, leaf, nb, q.P);
  if (tid < w) q.tau[sl * kPanel + tid] = tau_s[tid];

  // unit lower-trapezoidal V (implicit ones, zeros above) of the WY factor
  auto Veff = [&](int r, int a) -> double {
    return r > a ? V[a][r] : (r == a ? 1.0 : 0.0);
  };
  lds_mm(w, w, m, [&](int a, int r) { return Veff(r, a); }, Veff,
         [&](int i, int j, double x) { G[i][j] = x; }, wave, lane);
  __syncthreads();
  if (wave == 0) build_T(T, G, tau_s, w, lane);
  __syncthreads();
  for (int idx = tid; idx < kPanel * kPanel; idx += 256)
    q.Tl[sl * kPanel * kPanel + idx] = T[idx / kPanel][idx % kPanel];

  for (int cb = c0 + w; cb < k; cb += kPanel) {
    const int nc = min(kPanel, k - cb);
    __syncthreads();
    g2l(m * kPanel, tid,
        [&](int idx) {
          const int r = idx / kPanel, c = idx % kPanel;
          return c < nc ? A[(long)(a0 + r) * k + cb + c] : 0.0;
        },
        [&](int idx, double v) { Cc[idx % kPanel][idx / kPanel] = v; });
    __syncthreads();
    // W1 = V^T C  (w x nc)
    lds_mm(w, nc, m, [&](int a, int r) { return Veff(r, a); },
           [&](int r, int c) { return Cc[c][r]; }, [&](int i, int j, double x) { W1[i][j] = x; },
           wave, lane);
    __syncthreads();
    // G <- T^T W1   (G reused as scratch)
    lds_mm(w, nc, w, [&](int i, int l) { return T[l][i]; }, [&](int l, int c) { return W1[l][c]; },
           [&](int i, int j, double x) { G[i][j] = x; }, wave, lane);
    __syncthreads();
    // C -= V G
    lds_mm(m, nc, w, Veff, [&](int l, int c) { return G[l][c]; },
           [&](int r, int c, double x) { Cc[c][r] -= x; }, wave, lane);
    __syncthreads();
    for (int idx = tid; idx < m * kPanel; idx += 256) {
      const int r = idx / kPanel, c = idx % kPanel;
      if (c < nc) A[(long)(a0 + r) * k + cb + c] = Cc[c][r];
    }
  }
}

// Top row of the w x w triangle a leaf holds during panel p.
__device__ __forceinline__ int top_row(int leaf, int c0, int N, int nb) {
  return leaf == 0 ? c0 : leaf_start(leaf, N, nb);
}

// ---------------------------------------------------------------------------
// tree combine at level L of panel p: node = right child b, left child b-2^L
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void qr_tree_factor(QrArgs q, int p, int L) {
  __shared__ double Ra[kPanel][kT];   // [row][col]
  __shared__ double Rb[kPanel][kT];
  __shared__ double T[kPanel][kT], G[kPanel][kT];
  __shared__ double Ca[kPanel][kTrail + 1], Cb[kPanel][kTrail + 1];
  __shared__ double W1[kPanel][kTrail + 1], W2[kPanel][kTrail + 1];
  __shared__ double tau_s[kPanel];
  const int step = 1 << (L + 1);
  const int b = blockIdx.x * step + (1 << L);
  const int mat = blockIdx.y;
  const int N = q.N, k = q.k, nb = q.nb;
  if (b >= nb) return;
  const int a = b - (1 << L);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int ta = top_row(a, c0, N, nb), tb = top_row(b, c0, N, nb);
  double* A = q.A[mat];
  g2l(2 * kPanel * kPanel, tid,
      [&](int idx) {
        const int h = idx / (kPanel * kPanel), rc = idx % (kPanel * kPanel);
        const int r = rc / kPanel, c = rc % kPanel;
        const bool up = r <= c && r < w && c < w;
        return up ? A[(long)((h ? tb : ta) + r) * k + c0 + c] : 0.0;
      },
      [&](int idx, double v) {
        const int h = idx / (kPanel * kPanel), rc = idx % (kPanel * kPanel);
        (h ? Rb : Ra)[rc / kPanel][rc % kPanel] = v;
      });
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (wave == 0) {
      double ss = 0.0;
      if (lane <= j) ss = Rb[lane][j] * Rb[lane][j];
      ss = row_sum16(ss);
      ss = readlane_f64(ss, 0) + readlane_f64(ss, 16);
      const double alpha = Ra[j][j];
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      if (lane <= j) Rb[lane][j] *= scal;
      if (lane == 0) { Ra[j][j] = beta; tau_s[j] = tau; }
    }
    __syncthreads();
    const double tau = tau_s[j];
    if (tau != 0.0) {
      double d[kPanel / 4];
#pragma unroll
      for (int t = 0; t < kPanel / 4; ++t) {
        const int c = j + 1 + wave + 4 * t;
        d[t] = (c < w && lane <= j) ? Rb[lane][j] * Rb[lane][c] : 0.0;
      }
      // rows live in lanes 0..j <= 31: a 32-lane reduction suffices
#pragma unroll
      for (int t = 0; t < kPanel / 4; ++t) {
        d[t] = row_sum16(d[t]);
        d[t] = readlane_f64(d[t], 0) + readlane_f64(d[t], 16);
      }
#pragma unroll
      for (int t = 0; t < kPanel / 4; ++t) {
        const int c = j + 1 + wave + 4 * t;
        if (c < w) {
          const double f = tau * (d[t] + Ra[j][c]);
          if (lane <= j) Rb[lane][c] -= f * Rb[lane][j];
          if (lane == 0) Ra[j][c] -= f;
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < w * w; idx += 256) {
    const int r = idx / w, c = idx % w;
    if (r <= c) {
      A[(long)(ta + r) * k + c0 + c] = Ra[r][c];
      A[(long)(tb + r) * k + c0 + c] = Rb[r][c];
    }
  }
  // Vb = upper triangle of Rb (lower parts of the node's reflectors);
  // G = I + Vb^T Vb, then T
  auto Vb = [&](int r, int c) -> double { return r <= c ? Rb[r][c] : 0.0; };
  lds_mm(w, w, w, [&](int i, int r) { return Vb(r, i); }, Vb,
         [&](int i, int j, double x) { G[i][j] = x + (i == j ? 1.0 : 0.0); }, wave, lane);
  __syncthreads();
  if (wave == 0) build_T(T, G, tau_s, w, lane);
  __syncthreads();
  const long sl = slot(mat, p, b, nb, q.P);
  for (int idx = tid; idx < kPanel * kPanel; idx += 256)
    q.Tn[sl * kPanel * kPanel + idx] = T[idx / kPanel][idx % kPanel];
  // trailing columns [c0+w, k) of the 2w rows: W1 = Ca + Vb^T Cb;
  // W2 = T^T W1; Ca -= W2; Cb -= Vb W2
  for (int cb = c0 + w; cb < k; cb += kTrail) {
    const int nc = min(kTrail, k - cb);
    __syncthreads();
    g2l(2 * w * kTrail, tid,
        [&](int idx) {
          const int h = idx / (w * kTrail), rc = idx % (w * kTrail);
          const int r = rc / kTrail, c = rc % kTrail;
          return c < nc ? A[(long)((h ? tb : ta) + r) * k + cb + c] : 0.0;
        },
        [&](int idx, double v) {
          const int h = idx / (w * kTrail), rc = idx % (w * kTrail);
          (h ? Cb : Ca)[rc / kTrail][rc % kTrail] = v;
        });
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int r) { return Vb(r, i); }, [&](int r, int c) { return Cb[r][c]; },
           [&](int i, int j, double x) { W1[i][j] = x + Ca[i][j]; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int l) { return T[l][i]; }, [&](int l, int c) { return W1[l][c]; },
           [&](int i, int j, double x) { W2[i][j] = x; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, Vb, [&](int l, int c) { return W2[l][c]; },
           [&](int r, int c, double x) { Cb[r][c] -= x; }, wave, lane);
    for (int idx = tid; idx < w * kTrail; idx += 256) {
      const int r = idx / kTrail, c = idx % kTrail;
      if (c < nc) Ca[r][c] -= W2[r][c];
    }
    __syncthreads();
    for (int idx = tid; idx < w * kTrail; idx += 256) {
      const int r = idx / kTrail, c = idx % kTrail;
      if (c < nc) {
        A[(long)(ta + r) * k + cb + c] = Ca[r][c];
        A[(long)(tb + r) * k + cb + c] = Cb[r][c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Q formation
// ---------------------------------------------------------------------------
__global__ void qr_init_e(QrArgs q) {
  const int mat = blockIdx.y;
  const long total = (long)q.N * q.k;
  double* E = q.E[mat];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const long r = i / q.k, c = i % q.k;
    E[i] = (r == c) ? 1.0 : 0.0;
  }
}

// E rows of the node <- Q_node E on columns [c0, k): W1 = Ea + Vb^T Eb;
// W2 = T W1; Ea -= W2; Eb -= Vb W2.
__global__ __launch_bounds__(256) void qr_tree_apply(QrArgs q, int p, int L) {
  __shared__ double Vs[kPanel][kT], T[kPanel][kT];
  __shared__ double Ca[kPanel][kTrail + 1], Cb[kPanel][kTrail + 1];
  __shared__ double W1[kPanel][kTrail + 1], W2[kPanel][kTrail + 1];
  const int step = 1 << (L + 1);
  const int b = blockIdx.x * step + (1 << L);
  const int mat = blockIdx.y;
  const int N = q.N, k = q.k, nb = q.nb;
  if (b >= nb) return;
  const int a = b - (1 << L);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int ta = top_row(a, c0, N, nb), tb = top_row(b, c0, N, nb);
  const double* A = q.A[mat];
  double* E = q.E[mat];
  const long sl = slot(mat, p, b, nb, q.P);
  g2l(2 * kPanel * kPanel, tid,
      [&](int idx) {
        const int h = idx / (kPanel * kPanel), rc = idx % (kPanel * kPanel);
        const int r = rc / kPanel, c = rc % kPanel;
        if (h) return q.Tn[sl * kPanel * kPanel + rc];
        return (r <= c && r < w && c < w) ? A[(long)(tb + r) * k + c0 + c] : 0.0;
      },
      [&](int idx, double v) {
        const int h = idx / (kPanel * kPanel), rc = idx % (kPanel * kPanel);
        (h ? T : Vs)[rc / kPanel][rc % kPanel] = v;
      });
  for (int cb = c0; cb < k; cb += kTrail) {
    const int nc = min(kTrail, k - cb);
    __syncthreads();
    g2l(2 * w * kTrail, tid,
        [&](int idx) {
          const int h = idx / (w * kTrail), rc = idx % (w * kTrail);
          const int r = rc / kTrail, c = rc % kTrail;
          return c < nc ? E[(long)((h ? tb : ta) + r) * k + cb + c] : 0.0;
        },
        [&](int idx, double v) {
          const int h = idx / (w * kTrail), rc = idx % (w * kTrail);
          (h ? Cb : Ca)[rc / kTrail][rc % kTrail] = v;
        });
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int r) { return Vs[r][i]; }, [&](int r, int c) { return Cb[r][c]; },
           [&](int i, int j, double x) { W1[i][j] = x + Ca[i][j]; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int l) { return T[i][l]; }, [&](int l, int c) { return W1[l][c]; },
           [&](int i, int j, double x) { W2[i][j] = x; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, [&](int r, int l) { return Vs[r][l]; }, [&](int l, int c) { return W2[l][c]; },
           [&](int r, int c, double x) { Cb[r][c] -= x; }, wave, lane);
    for (int idx = tid; idx < w * kTrail; idx += 256) {
      const int r = idx / kTrail, c = idx % kTrail;
      if (c < nc) Ca[r][c] -= W2[r][c];
    }
    __syncthreads();
    for (int idx = tid; idx < w * kTrail; idx += 256) {
      const int r = idx / kTrail, c = idx % kTrail;
      if (c < nc) {
        E[(long)(ta + r) * k + cb + c] = Ca[r][c];
        E[(long)(tb + r) * k + cb + c] = Cb[r][c];
      }
    }
  }
}

// E rows of the leaf <- Q_leaf E on columns [c0, k): C -= V T (V^T C).
__global__ __launch_bounds__(256) void qr_leaf_apply(QrArgs q, int p) {
  __shared__ double V[kPanel][kLR];
  __shared__ double Cc[kPanel][kLR];
  __shared__ double T[kPanel][kT], W1[kPanel][kT], W2[kPanel][kT];
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  const double* A = q.A[mat];
  double* E = q.E[mat];
  const long sl = slot(mat, p, leaf, nb, q.P);
  g2l(kPanel * kLeafRows, tid,
      [&](int idx) {
        const int r = idx / kPanel, c = idx % kPanel;
        if (r >= m || c >= w) return 0.0;
        return r > c ? A[(long)(a0 + r) * k + c0 + c] : (r == c ? 1.0 : 0.0);
      },
      [&](int idx, double v) { V[idx % kPanel][idx / kPanel] = v; });
  g2l(kPanel * kPanel, tid, [&](int idx) { return q.Tl[sl * kPanel * kPanel + idx]; },
      [&](int idx, double v) { T[idx / kPanel][idx % kPanel] = v; });
  for (int cb = c0; cb < k; cb += kPanel) {
    const int nc = min(kPanel, k - cb);
    __syncthreads();
    g2l(m * kPanel, tid,
        [&](int idx) {
          const int r = idx / kPanel, c = idx % kPanel;
          return c < nc ? E[(long)(a0 + r) * k + cb + c] : 0.0;
        },
        [&](int idx, double v) { Cc[idx % kPanel][idx / kPanel] = v; });
    __syncthreads();
    lds_mm(w, nc, m, [&](int a, int r) { return V[a][r]; }, [&](int r, int c) { return Cc[c][r]; },
           [&](int i, int j, double x) { W1[i][j] = x; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int l) { return T[i][l]; }, [&](int l, int c) { return W1[l][c]; },
           [&](int i, int j, double x) { W2[i][j] = x; }, wave, lane);
    __syncthreads();
    lds_mm(m, nc, w, [&](int r, int l) { return V[l][r]; }, [&](int l, int c) { return W2[l][c]; },
           [&](int r, int c, double x) { Cc[c][r] -= x; }, wave, lane);
    __syncthreads();
    for (int idx = tid; idx < m * kPanel; idx += 256) {
      const int r = idx / kPanel, c = idx % kPanel;
      if (c < nc) E[(long)(a0 + r) * k + cb + c] = Cc[c][r];
    }
  }
}

// sgn[mat][c] = sign(R_cc) (R_cc read from the factored block).  A separate
// pass, because the destination of Q may be the factored block itself.
__global__ void qr_diag_sign(QrArgs q) {
  const int mat = blockIdx.y;
  const double* A = q.A[mat];
  for (int c = threadIdx.x; c < q.k; c += blockDim.x)
    q.sgn[(long)mat * q.k + c] = A[(long)c * q.k + c] < 0.0 ? -1.0 : 1.0;
}

// Q_out[:, c] = sgn[c] * E[:, c]
__global__ void qr_sign_copy(QrArgs q) {
  const int mat = blockIdx.y;
  const long total = (long)q.N * q.k;
  const double* E = q.E[mat];
  const double* sg = q.sgn + (long)mat * q.k;
  double* O = q.O[mat];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x)
    O[i] = sg[i % q.k] * E[i];
}

QrPlan make_plan(int N, int k) {
  QrPlan pl;
  pl.N = N;
  pl.k = k;
  int nb = N / (k > 128 ? k : 128);
  if (nb < 1) nb = 1;
  const int need = (N + kLeafRows - 1) / kLeafRows;
  if (nb < need) nb = need;
  if (nb > 1 && N / nb < k) nb = N / k;  // leaf 0 must hold k rows
  pl.nb = nb;
  pl.P = (k + kPanel - 1) / kPanel;
  int depth = 0;
  while ((1 << depth) < nb) ++depth;
  pl.depth = depth;
  return pl;
}

}  // namespace

size_t qr_workspace_bytes(int count, int N, int k) {
  const QrPlan pl = make_plan(N, k);
  const size_t slots = (size_t)count * pl.P * pl.nb;
  const size_t n = slots * kPanel + 2 * slots * kPanel * kPanel + (size_t)count * N * k +
                   (size_t)count * k;
  return n * sizeof(double);
}

int launch_qr(int count, double* const* W, int N, int k, void* ws, hipStream_t s) {
  if (count <= 0 || k <= 0) return 0;
  if (count > kMaxProb || N < k || k > kLeafRows) {
    set_thread_error("launch_qr: need k <= N, k <= 256 and at most 8 matrices per launch");
    return 1;
  }
  const QrPlan pl = make_plan(N, k);
  if ((N + pl.nb - 1) / pl.nb > kLeafRows) {
    set_thread_error("launch_qr: N too large for the leaf size (N/k too large)");
    return 1;
  }
  QrArgs q{};
  q.count = count;
  q.N = N;
  q.k = k;
  q.nb = pl.nb;
  q.P = pl.P;
  const size_t slots = (size_t)count * pl.P * pl.nb;
  double* base = (double*)ws;
  q.tau = base;
  q.Tl = q.tau + slots * kPanel;
  q.Tn = q.Tl + slots * kPanel * kPanel;
  double* e = q.Tn + slots * kPanel * kPanel;
  for (int i = 0; i < count; ++i) {
    q.A[i] = W[i];
    q.E[i] = e + (size_t)i * N * k;
    q.O[i] = W[i];
  }
  q.sgn = e + (size_t)count * N * k;

  for (int p = 0; p < pl.P; ++p) {
    qr_leaf_factor<<<dim3(pl.nb, count), 256, 0, s>>>(q, p);
    for (int L = 0; L < pl.depth; ++L) {
      const int nodes = (pl.nb + (1 << (L + 1)) - 1) >> (L + 1);
      qr_tree_factor<<<dim3(nodes, count), 256, 0, s>>>(q, p, L);
    }
  }
  const long total = (long)N * k;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  qr_init_e<<<dim3(blocks, count), 256, 0, s>>>(q);
  for (int p = pl.P - 1; p >= 0; --p) {
    for (int L = pl.depth - 1; L >= 0; --L) {
      const int nodes = (pl.nb + (1 << (L + 1)) - 1) >> (L + 1);
      qr_tree_apply<<<dim3(nodes, count), 256, 0, s>>>(q, p, L);
    }
    qr_leaf_apply<<<dim3(pl.nb, count), 256, 0, s>>>(q, p);
  }
  qr_diag_sign<<<dim3(1, count), 256, 0, s>>>(q);
  qr_sign_copy<<<dim3(blocks, count), 256, 0, s>>>(q);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace sictm
