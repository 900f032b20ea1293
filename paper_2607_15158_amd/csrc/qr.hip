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
//    four at a time up a reduction tree (depth log4 of the leaf count);
//    combining stacked upper triangles gives reflectors [e_j; v] with v
//    upper triangular in each absorbed triangle, stored in its place, and
//    their own WY factor updates the trailing columns of the node's rows;
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
constexpr int kLeafRows = 192;   // three rows per lane of one wavefront
constexpr int kLR = kLeafRows + 1;   // odd row length: fragment reads hit distinct banks
constexpr int kT = kPanel + 1;   // padded row length of the small LDS matrices

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
// G = V^T V (strict upper part) and the taus, forward columnwise:
// T_jj = tau_j, T[i, j] = -tau_j sum_{l=i}^{j-1} T[i, l] G[l, j] for i < j.
// Row i depends only on itself, so lane i builds row i in registers.
__device__ __forceinline__ void build_T(double (*T)[kT], double (*G)[kT], const double* tau,
                                        int w, int lane) {
  double t[kPanel];
#pragma unroll
  for (int j = 0; j < kPanel; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < j; ++l) acc += t[l] * G[l][j];   // t[l] = 0 for l < lane
    const double tj = j < w ? tau[j] : 0.0;
    t[j] = lane < j ? -tj * acc : (lane == j ? tj : 0.0);
  }
  if (lane < kPanel) {
#pragma unroll
    for (int j = 0; j < kPanel; ++j) T[lane][j] = t[j];
  }
}

// ---------------------------------------------------------------------------
// Householder factorisation of one panel by a single wavefront, with the
// panel in registers: x[r][c] is row (lane + 64 r), column c.  The pivot of
// column j is row j (lane j, r = 0); below(j, r) selects the rows that carry
// reflector j under the pivot.  Per column the wavefront forms the reflector
// (dlarfg convention); one reduction then gives both v_j^T x_s for the later
// columns s > j (applied at once) and v_s^T v_j for the earlier ones (the
// Gram column of the WY factor T).  The 32 per-lane partial sums of a step
// are reduced through LDS: every lane writes its row of partials, lane l
// adds column l % 32 over one half of the rows, and the halves meet in one
// cross-lane exchange; the scaled sums are read back as LDS broadcasts.
// The wavefront's LDS traffic is ordered by itself, so no barrier is needed.
// ---------------------------------------------------------------------------
struct PanelScratch {
  double P[64][kT];   // per-lane partial sums
  double F[kPanel];   // tau * v_j^T x_s
};

// 1/x to full double precision from the hardware estimate (two Newton
// steps); x is never zero where it is used.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Step J of the panel factorisation (J is a template parameter so that every
// register of the panel is addressed statically).  Branch-free when FULL
// (w == 32), so consecutive steps form one block the scheduler can overlap.
template <int J, bool FULL, int RPL, typename Below>
__device__ __forceinline__ void panel_step(double (&x)[RPL][kPanel], int w, int lane,
                                           const Below& below, double* tau_out, double (*G)[kT],
                                           PanelScratch& ps) {
  if (FULL || J < w) {
    bool bl[RPL];
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      bl[r] = below(J, r);
      ss += bl[r] ? x[r][J] * x[r][J] : 0.0;
    }
    ss = wave_sum64(ss);
    const double alpha = readlane_f64(x[0][J], J);
    // dlarfg: beta = -sign(alpha) |(alpha, x)|, tau = (beta - alpha) / beta,
    // v = x / (alpha - beta); H = I (tau = 0) when x is exactly zero
    const bool live = ss > 0.0;
    const double nrm = sqrt(alpha * alpha + ss);
    const double beta = live ? (alpha >= 0.0 ? -nrm : nrm) : alpha;
    const double tau = live ? (beta - alpha) * fast_rcp(beta) : 0.0;
    const double scal = live ? fast_rcp(alpha - beta) : 0.0;
    double vj[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      vj[r] = bl[r] ? x[r][J] * scal : ((r == 0 && lane == J) ? 1.0 : 0.0);
      if (bl[r]) x[r][J] = vj[r];
    }
    if (lane == J) x[0][J] = beta;
    if (lane == 0) tau_out[J] = tau;
#pragma unroll
    for (int s = 0; s < kPanel; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc += vj[r] * x[r][s];
      ps.P[lane][s] = acc;
    }
    const int col = lane & 31, h = (lane >> 5) * 32;
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < 32; ++i) tot += ps.P[h + i][col];
    tot += __shfl_xor(tot, 32, 64);
    if (lane < 32) {
      ps.F[lane] = tau * tot;
      if (lane < J) G[lane][J] = tot;
    }
#pragma unroll
    for (int s = J + 1; s < kPanel; ++s) {
      if (FULL || s < w) {
        const double f = ps.F[s];
#pragma unroll
        for (int r = 0; r < RPL; ++r) x[r][s] -= f * vj[r];
      }
    }
  }
  if constexpr (J + 1 < kPanel) panel_step<J + 1, FULL>(x, w, lane, below, tau_out, G, ps);
}

template <int RPL, typename Below>
__device__ __forceinline__ void wave_panel_qr(double (&x)[RPL][kPanel], int w, int lane, Below below,
                                              double* tau_out, double (*G)[kT], PanelScratch& ps) {
  if (w == kPanel)
    panel_step<0, true>(x, w, lane, below, tau_out, G, ps);
  else
    panel_step<0, false>(x, w, lane, below, tau_out, G, ps);
}

// ---------------------------------------------------------------------------
// leaf factorisation of panel p + WY update of its trailing columns
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void qr_leaf_factor(QrArgs q, int p) {
  __shared__ double V[kPanel][kLR];           // panel, column-major
  __shared__ double Cc[kPanel][kLR];          // trailing chunk, column-major
  __shared__ double T[kPanel][kT], G[kPanel][kT], W1[kPanel][kT];
  __shared__ double tau_s[kPanel];
  __shared__ PanelScratch ps;
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  double* A = q.A[mat];

  if (wave == 0) {
    constexpr int RPL = kLeafRows / 64;
    double x[RPL][kPanel];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      const double* src = A + (long)(a0 + row) * k + c0;
#pragma unroll
      for (int c = 0; c < kPanel; ++c) x[r][c] = (row < m && c < w) ? src[c] : 0.0;
    }
    wave_panel_qr<RPL>(
        x, w, lane,
        [&](int j, int r) {
          const int row = lane + 64 * r;
          return row > j && row < m;
        },
        tau_s, G, ps);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      double* dst = A + (long)(a0 + row) * k + c0;
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        if (row < m && c < w) dst[c] = x[r][c];
        if (row < kLR) V[c][row] = x[r][c];
      }
    }
    build_T(T, G, tau_s, w, lane);
  }
  __syncthreads();
  const long sl = slot(mat, p, leaf, nb, q.P);
  if (tid < w) q.tau[sl * kPanel + tid] = tau_s[tid];
  for (int idx = tid; idx < kPanel * kPanel; idx += 256)
    q.Tl[sl * kPanel * kPanel + idx] = T[idx / kPanel][idx % kPanel];

  // unit lower-trapezoidal V (implicit ones, zeros above) of the WY factor
  auto Veff = [&](int r, int a) -> double {
    return r > a ? V[a][r] : (r == a ? 1.0 : 0.0);
  };
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
// Reduction tree: a node at stride s combines the triangles of the leaves
// a, a + s, ..., a + (kArity - 1) s (those below nb), a = node * s * kArity;
// the first child keeps R, the others receive the reflector parts.  Row
// (lane + 64 r) of the node's wavefront is row (lane & 31) of child
// (lane >> 5) + 2 r.  The node's WY factor is stored in the slot of child 1,
// s (4 i + 1), which no other node at any stride shares.
// ---------------------------------------------------------------------------
constexpr int kArity = 4;
constexpr int kNodeRPL = kArity / 2;
constexpr int kTrailN = 32;   // trailing columns per LDS chunk in the tree kernels

__device__ __forceinline__ int node_children(int a, int s, int nb) {
  return min(kArity, (nb - a + s - 1) / s);
}

// Wavefront 0 factors the stacked triangles [R_0; R_1; ...]; the reflectors
// are [e_j; v_j] with v_j in the upper triangles of the children after the
// first.  Trailing columns [c0 + w, k) of the node's rows:
// W1 = C_0 + sum_h V_h^T C_h; W2 = T^T W1; C_0 -= W2; C_h -= V_h W2.
__global__ __launch_bounds__(256) void qr_tree_factor(QrArgs q, int p, int s) {
  __shared__ double Vs[kArity - 1][kPanel][kT];
  __shared__ double T[kPanel][kT], G[kPanel][kT];
  __shared__ double Cs[kArity][kPanel][kTrailN + 1];
  __shared__ double W1[kPanel][kTrailN + 1], W2[kPanel][kTrailN + 1];
  __shared__ double tau_s[kPanel];
  __shared__ PanelScratch ps;
  const int a = blockIdx.x * s * kArity;
  const int mat = blockIdx.y;
  const int N = q.N, k = q.k, nb = q.nb;
  if (a + s >= nb) return;
  const int nch = node_children(a, s, nb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  // top rows of the children, computed once (leaf_start divides in 64 bits)
  __shared__ int tops[kArity];
  if (tid < kArity) tops[tid] = tid < nch ? top_row(a + tid * s, c0, N, nb) : 0;
  __syncthreads();
  auto top = [&](int h) { return tops[h]; };
  double* A = q.A[mat];
  if (wave == 0) {
    const int rr = lane & 31;
    double x[kNodeRPL][kPanel];
#pragma unroll
    for (int r = 0; r < kNodeRPL; ++r) {
      const int h = (lane >> 5) + 2 * r;
      const bool live = h < nch;
      const double* src = A + (long)(live ? top(h) + rr : 0) * k + c0;
#pragma unroll
      for (int c = 0; c < kPanel; ++c) x[r][c] = (live && rr <= c && c < w) ? src[c] : 0.0;
    }
    wave_panel_qr<kNodeRPL>(
        x, w, lane,
        [&](int j, int r) {
          const int h = (lane >> 5) + 2 * r;
          return h > 0 && h < nch && rr <= j;
        },
        tau_s, G, ps);
#pragma unroll
    for (int r = 0; r < kNodeRPL; ++r) {
      const int h = (lane >> 5) + 2 * r;
      if (h < nch) {
        double* dst = A + (long)(top(h) + rr) * k + c0;
#pragma unroll
        for (int c = 0; c < kPanel; ++c) {
          const bool in = rr <= c && c < w;
          if (in) dst[c] = x[r][c];
          if (h > 0) Vs[h - 1][rr][c] = in ? x[r][c] : 0.0;
        }
      }
    }
    build_T(T, G, tau_s, w, lane);
  }
  __syncthreads();
  const long sl = slot(mat, p, a + s, nb, q.P);
  for (int idx = tid; idx < kPanel * kPanel; idx += 256)
    q.Tn[sl * kPanel * kPanel + idx] = T[idx / kPanel][idx % kPanel];
  // children after the first stacked along one index: u = (h - 1) * kPanel + r
  const int nv = (nch - 1) * kPanel;
  auto V = [&](int u, int c) -> double { return Vs[u >> 5][u & 31][c]; };
  for (int cb = c0 + w; cb < k; cb += kTrailN) {
    const int nc = min(kTrailN, k - cb);
    __syncthreads();
    // rows r >= w of every child are loaded as zeros, so that the stacked
    // products may run over full kPanel-row blocks
    g2l(nch * kPanel * kTrailN, tid,
        [&](int idx) {
          const int h = idx / (kPanel * kTrailN), rc = idx % (kPanel * kTrailN);
          const int r = rc / kTrailN, c = rc % kTrailN;
          return (r < w && c < nc) ? A[(long)(top(h) + r) * k + cb + c] : 0.0;
        },
        [&](int idx, double v) {
          const int h = idx / (kPanel * kTrailN), rc = idx % (kPanel * kTrailN);
          Cs[h][rc / kTrailN][rc % kTrailN] = v;
        });
    __syncthreads();
    lds_mm(w, nc, nv, [&](int i, int u) { return V(u, i); },
           [&](int u, int c) { return Cs[1 + (u >> 5)][u & 31][c]; },
           [&](int i, int j, double x) { W1[i][j] = x + Cs[0][i][j]; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int l) { return T[l][i]; }, [&](int l, int c) { return W1[l][c]; },
           [&](int i, int j, double x) { W2[i][j] = x; }, wave, lane);
    __syncthreads();
    lds_mm(nv, nc, w, V, [&](int l, int c) { return W2[l][c]; },
           [&](int u, int c, double x) { Cs[1 + (u >> 5)][u & 31][c] -= x; }, wave, lane);
    for (int idx = tid; idx < w * kTrailN; idx += 256) {
      const int r = idx / kTrailN, c = idx % kTrailN;
      if (c < nc) Cs[0][r][c] -= W2[r][c];
    }
    __syncthreads();
    for (int idx = tid; idx < nch * w * kTrailN; idx += 256) {
      const int h = idx / (w * kTrailN), rc = idx % (w * kTrailN);
      const int r = rc / kTrailN, c = rc % kTrailN;
      if (c < nc) A[(long)(top(h) + r) * k + cb + c] = Cs[h][r][c];
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

// E rows of the node <- Q_node E on columns [c0, k):
// W1 = E_0 + sum_h V_h^T E_h; W2 = T W1; E_0 -= W2; E_h -= V_h W2.
__global__ __launch_bounds__(256) void qr_tree_apply(QrArgs q, int p, int s) {
  __shared__ double Vs[kArity - 1][kPanel][kT], T[kPanel][kT];
  __shared__ double Cs[kArity][kPanel][kTrailN + 1];
  __shared__ double W1[kPanel][kTrailN + 1], W2[kPanel][kTrailN + 1];
  const int a = blockIdx.x * s * kArity;
  const int mat = blockIdx.y;
  const int N = q.N, k = q.k, nb = q.nb;
  if (a + s >= nb) return;
  const int nch = node_children(a, s, nb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  __shared__ int tops[kArity];
  if (tid < kArity) tops[tid] = tid < nch ? top_row(a + tid * s, c0, N, nb) : 0;
  __syncthreads();
  auto top = [&](int h) { return tops[h]; };
  const double* A = q.A[mat];
  double* E = q.E[mat];
  const long sl = slot(mat, p, a + s, nb, q.P);
  const int nv = (nch - 1) * kPanel;
  g2l(nv * kPanel, tid,
      [&](int idx) {
        const int u = idx / kPanel, c = idx % kPanel;
        const int h = 1 + (u >> 5), r = u & 31;
        return (r <= c && c < w) ? A[(long)(top(h) + r) * k + c0 + c] : 0.0;
      },
      [&](int idx, double v) {
        const int u = idx / kPanel;
        Vs[u >> 5][u & 31][idx % kPanel] = v;
      });
  g2l(kPanel * kPanel, tid, [&](int idx) { return q.Tn[sl * kPanel * kPanel + idx]; },
      [&](int idx, double v) { T[idx / kPanel][idx % kPanel] = v; });
  auto V = [&](int u, int c) -> double { return Vs[u >> 5][u & 31][c]; };
  for (int cb = c0; cb < k; cb += kTrailN) {
    const int nc = min(kTrailN, k - cb);
    __syncthreads();
    g2l(nch * kPanel * kTrailN, tid,
        [&](int idx) {
          const int h = idx / (kPanel * kTrailN), rc = idx % (kPanel * kTrailN);
          const int r = rc / kTrailN, c = rc % kTrailN;
          return (r < w && c < nc) ? E[(long)(top(h) + r) * k + cb + c] : 0.0;
        },
        [&](int idx, double v) {
          const int h = idx / (kPanel * kTrailN), rc = idx % (kPanel * kTrailN);
          Cs[h][rc / kTrailN][rc % kTrailN] = v;
        });
    __syncthreads();
    lds_mm(w, nc, nv, [&](int i, int u) { return V(u, i); },
           [&](int u, int c) { return Cs[1 + (u >> 5)][u & 31][c]; },
           [&](int i, int j, double x) { W1[i][j] = x + Cs[0][i][j]; }, wave, lane);
    __syncthreads();
    lds_mm(w, nc, w, [&](int i, int l) { return T[i][l]; }, [&](int l, int c) { return W1[l][c]; },
           [&](int i, int j, double x) { W2[i][j] = x; }, wave, lane);
    __syncthreads();
    lds_mm(nv, nc, w, V, [&](int l, int c) { return W2[l][c]; },
           [&](int u, int c, double x) { Cs[1 + (u >> 5)][u & 31][c] -= x; }, wave, lane);
    for (int idx = tid; idx < w * kTrailN; idx += 256) {
      const int r = idx / kTrailN, c = idx % kTrailN;
      if (c < nc) Cs[0][r][c] -= W2[r][c];
    }
    __syncthreads();
    for (int idx = tid; idx < nch * w * kTrailN; idx += 256) {
      const int h = idx / (w * kTrailN), rc = idx % (w * kTrailN);
      const int r = rc / kTrailN, c = rc % kTrailN;
      if (c < nc) E[(long)(top(h) + r) * k + cb + c] = Cs[h][r][c];
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
  for (long span = 1; span < nb; span *= kArity) ++depth;
  pl.depth = depth;
  return pl;
}

}  // namespace

bool qr_plan_ok(int N, int k) {
  if (k <= 0 || N < k || k > kLeafRows) return false;
  const QrPlan pl = make_plan(N, k);
  return (N + pl.nb - 1) / pl.nb <= kLeafRows;
}

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
    set_thread_error("launch_qr: need k <= N, k <= 192 and at most 8 matrices per launch");
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
    for (int L = 0, st = 1; L < pl.depth; ++L, st *= kArity) {
      const int nodes = (pl.nb + st * kArity - 1) / (st * kArity);
      qr_tree_factor<<<dim3(nodes, count), 256, 0, s>>>(q, p, st);
    }
  }
  const long total = (long)N * k;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  qr_init_e<<<dim3(blocks, count), 256, 0, s>>>(q);
  for (int p = pl.P - 1; p >= 0; --p) {
    for (int L = pl.depth - 1; L >= 0; --L) {
      int st = 1;
      for (int i = 0; i < L; ++i) st *= kArity;
      const int nodes = (pl.nb + st * kArity - 1) / (st * kArity);
      qr_tree_apply<<<dim3(nodes, count), 256, 0, s>>>(q, p, st);
    }
    qr_leaf_apply<<<dim3(pl.nb, count), 256, 0, s>>>(q, p);
  }
  qr_diag_sign<<<dim3(1, count), 256, 0, s>>>(q);
  qr_sign_copy<<<dim3(blocks, count), 256, 0, s>>>(q);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace sictm
