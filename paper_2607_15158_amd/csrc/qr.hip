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
// The operands of kMmStage k-steps are read into registers before their
// products issue, so that one LDS latency covers kMmStage products, and the
// products rotate over four accumulators.  Indices outside the operands are
// clamped to element (0, 0) for the read and their values replaced by zero,
// so every LDS read stays inside the caller's arrays.
constexpr int kMmStage = 8;
template <typename FA, typename FB, typename FS>
__device__ __forceinline__ void lds_mm(int M, int N, int K, FA A, FB B, FS store, int wave,
                                       int lane) {
  const int bm = (M + 15) >> 4, bn = (N + 15) >> 4;
  for (int blk = wave; blk < bm * bn; blk += 4) {
    const int i0 = (blk / bn) << 4, j0 = (blk % bn) << 4;
    const int ar = i0 + (lane & 15), bc = j0 + (lane & 15);
    const bool ain = ar < M, bin = bc < N;
    const int arc = ain ? ar : 0, bcc = bin ? bc : 0;
    v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int k0 = 0; k0 < K; k0 += 4 * kMmStage) {
      double a[kMmStage], b[kMmStage];
#pragma unroll
      for (int u = 0; u < kMmStage; ++u) {
        const int ka = k0 + 4 * u + (lane >> 4);
        const bool kin = ka < K;
        const int kc = kin ? ka : 0;
        const double av = A(arc, kc), bv = B(kc, bcc);
        a[u] = (ain && kin) ? av : 0.0;
        b[u] = (bin && kin) ? bv : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kMmStage; ++u)
        acc[u & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc[u & 3], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + (lane >> 4) + 4 * r, col = j0 + (lane & 15);
      if (row < M && col < N) store(row, col, (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]));
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
// Householder factorisation of one panel by the four wavefronts of a
// workgroup, each holding 64 rows of the panel in registers: x[c] is column
// c of the lane's row.  The pivot of column j is row j, held by lane j of
// wavefront 0; on(j) says whether the lane's row carries reflector j (lies
// below the pivot).  Rows and columns outside the panel are held as zeros,
// so they take part in every sum without changing it.  Per column every
// wavefront reduces its share of the squared norm and wavefront 0 publishes
// the pivot; after a barrier all wavefronts form the same reflector (dlarfg
// convention); one transpose-reduction per wavefront (wave_xsum32) of the
// products v_j^T x_s, a barrier, and the four shares summed in a fixed
// order give every wavefront the same v_j^T x_s for the later columns s > j
// (applied at once from scalar registers) and v_s^T v_j for the earlier
// ones (the Gram column of the WY factor T, written by wavefront 0).  The
// shared sums are double-buffered by column parity, so two barriers per
// column order all reads and writes.
// ---------------------------------------------------------------------------

// 1/x to full double precision from the hardware estimate (two Newton
// steps); x is never zero where it is used.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

struct PanelShare {
  double ss[2][4];          // squared norms below the pivot, per wavefront
  double alpha[2];          // pivot value
  double dot[2][4][kPanel]; // v_j^T x_s per wavefront
};

// Squared norm below the pivot of column j (this wavefront's share) and the
// pivot value, published for the step that factors column j.
template <int J, typename On>
__device__ __forceinline__ void publish_norm(const double (&x)[kPanel], int lane, int wave,
                                             const On& on, PanelShare& sh) {
  constexpr int b = J & 1;
  const double ssw = wave_sum64(on(J) ? x[J] * x[J] : 0.0);
  if (lane == 0) sh.ss[b][wave] = ssw;
  if (wave == 0 && lane == J) sh.alpha[b] = x[J];
}

// Step J of the panel factorisation (J is a template parameter so that every
// register of the panel is addressed statically); columns J >= w are absent.
// Column J + 1 is updated first and its norm published before the other
// columns are updated, so that its reduction overlaps their updates.
template <int J, typename On>
__device__ __forceinline__ void panel_step(double (&x)[kPanel], int w, int lane, int wave,
                                           const On& on, double* tau_out, double (*G)[kT],
                                           PanelShare& sh) {
  if (J < w) {
    constexpr int b = J & 1;
    const bool bj = on(J);
    const bool piv = wave == 0 && lane == J;
    __syncthreads();
    const double ss = (sh.ss[b][0] + sh.ss[b][1]) + (sh.ss[b][2] + sh.ss[b][3]);
    const double alpha = sh.alpha[b];
    // dlarfg: beta = -sign(alpha) |(alpha, x)|, tau = (beta - alpha) / beta,
    // v = x / (alpha - beta); H = I (tau = 0) when x is exactly zero
    const bool live = ss > 0.0;
    const double nrm = sqrt(alpha * alpha + ss);
    const double beta = live ? (alpha >= 0.0 ? -nrm : nrm) : alpha;
    const double tau = live ? (beta - alpha) * fast_rcp(beta) : 0.0;
    const double scal = live ? fast_rcp(alpha - beta) : 0.0;
    const double vj = bj ? x[J] * scal : (piv ? 1.0 : 0.0);
    x[J] = bj ? vj : (piv ? beta : x[J]);
    if (wave == 0 && lane == 0) tau_out[J] = tau;
    const double part = wave_xsum32([&](int s) { return s == J ? 0.0 : vj * x[s]; }, lane);
    const int col = lane >> 1;
    if (!(lane & 1)) sh.dot[b][wave][col] = part;
    __syncthreads();
    const double tot =
        (sh.dot[b][0][col] + sh.dot[b][1][col]) + (sh.dot[b][2][col] + sh.dot[b][3][col]);
    if (wave == 0 && !(lane & 1) && col < J) G[col][J] = tot;
    const double f = tau * tot;
    if constexpr (J + 1 < kPanel) {
      x[J + 1] -= readlane_f64(f, 2 * (J + 1)) * vj;
      publish_norm<J + 1>(x, lane, wave, on, sh);
    }
#pragma unroll
    for (int s = J + 2; s < kPanel; ++s) x[s] -= readlane_f64(f, 2 * s) * vj;
  }
  if constexpr (J + 1 < kPanel) panel_step<J + 1>(x, w, lane, wave, on, tau_out, G, sh);
}

// The whole panel; afterwards wavefront 0 forms T from the Gram columns.
template <typename On>
__device__ __forceinline__ void block_panel_qr(double (&x)[kPanel], int w, int lane, int wave,
                                               On on, double* tau_s, double (*G)[kT],
                                               double (*T)[kT], PanelShare& sh) {
  publish_norm<0>(x, lane, wave, on, sh);
  panel_step<0>(x, w, lane, wave, on, tau_s, G, sh);
  if (wave == 0) build_T(T, G, tau_s, w, lane);
}

// ---------------------------------------------------------------------------
// leaf factorisation of panel p (the trailing columns: qr_leaf_wy)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void qr_leaf_factor(QrArgs q, int p) {
  __shared__ double T[kPanel][kT], G[kPanel][kT];
  __shared__ double tau_s[kPanel];
  __shared__ PanelShare sh;
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  double* A = q.A[mat];
  // row (lane + 64 wave) of the leaf's active rows; rows at or beyond m are
  // held as zeros
  const int row = lane + 64 * wave;
  double x[kPanel];
  {
    const double* src = A + (long)(a0 + (row < m ? row : 0)) * k + c0;
#pragma unroll
    for (int c = 0; c < kPanel; ++c) x[c] = (row < m && c < w) ? src[c] : 0.0;
  }
  block_panel_qr(x, w, lane, wave, [&](int j) { return row > j; }, tau_s, G, T, sh);
  if (row < m) {
    double* dst = A + (long)(a0 + row) * k + c0;
#pragma unroll
    for (int c = 0; c < kPanel; ++c)
      if (c < w) dst[c] = x[c];
  }
  __syncthreads();
  const long sl = slot(mat, p, leaf, nb, q.P);
  if (tid < w) q.tau[sl * kPanel + tid] = tau_s[tid];
  for (int idx = tid; idx < kPanel * kPanel; idx += 256)
    q.Tl[sl * kPanel * kPanel + idx] = T[idx / kPanel][idx % kPanel];
}

// Top row of the w x w triangle a leaf holds during panel p.
__device__ __forceinline__ int top_row(int leaf, int c0, int N, int nb) {
  return leaf == 0 ? c0 : leaf_start(leaf, N, nb);
}

// ---------------------------------------------------------------------------
// Reduction tree: a node at stride s combines the triangles of the leaves
// a, a + s, ..., a + (kArity - 1) s (those below nb), a = node * s * kArity;
// the first child keeps R, the others receive the reflector parts.  Lane l
// of wavefront v holds row (l & 31) of child 2 v + (l >> 5).  The node's WY
// factor is stored in the slot of child 1, s (kArity i + 1), which no other
// node at any stride shares (its odd part times a power of kArity).
// ---------------------------------------------------------------------------
constexpr int kArity = 8;
static_assert(kArity == 2 * 4, "two children per wavefront, four wavefronts");
constexpr int kTrailN = 32;   // columns per workgroup in the block-reflector kernels
static_assert(kTrailN == kPanel, "the leaf and tree block-reflector chunks share one launch width");

__device__ __forceinline__ int node_children(int a, int s, int nb) {
  return min(kArity, (nb - a + s - 1) / s);
}

// The workgroup factors the stacked triangles [R_0; R_1; ...]; the
// reflectors are [e_j; v_j] with v_j in the upper triangles of the children
// after the first (the node's trailing columns: qr_tree_wy).
__global__ __launch_bounds__(256) void qr_tree_factor(QrArgs q, int p, int s) {
  __shared__ double T[kPanel][kT], G[kPanel][kT];
  __shared__ double tau_s[kPanel];
  __shared__ PanelShare sh;
  const int a = blockIdx.x * s * kArity;
  const int mat = blockIdx.y;
  const int N = q.N, k = q.k, nb = q.nb;
  if (a + s >= nb) return;
  const int nch = node_children(a, s, nb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  double* A = q.A[mat];
  const int rr = lane & 31, h = 2 * wave + (lane >> 5);
  const bool live = h < nch;
  const long rowoff = live ? (long)(top_row(a + h * s, c0, N, nb) + rr) * k + c0 : 0;
  double x[kPanel];
#pragma unroll
  for (int c = 0; c < kPanel; ++c) x[c] = (live && rr <= c && c < w) ? A[rowoff + c] : 0.0;
  // the reflectors live in the children after the first; their rows below
  // the triangles and absent children are held as zeros
  block_panel_qr(x, w, lane, wave, [&](int) { return h > 0; }, tau_s, G, T, sh);
  if (live) {
#pragma unroll
    for (int c = 0; c < kPanel; ++c)
      if (rr <= c && c < w) A[rowoff + c] = x[c];
  }
  __syncthreads();
  const long sl = slot(mat, p, a + s, nb, q.P);
  for (int idx = tid; idx < kPanel * kPanel; idx += 256)
    q.Tn[sl * kPanel * kPanel + idx] = T[idx / kPanel][idx % kPanel];
}

// ---------------------------------------------------------------------------
// Block reflectors applied to 32-column chunks, one chunk per workgroup
// (blockIdx.z), so that the chunks of a leaf or node run side by side.
// FORM = false: the trailing update of the factorisation, A <- H^T A on the
// columns [c0 + w, k) (H = I - V T V^T, so H^T uses T^T); FORM = true: the
// Q formation, E <- H E on the columns [c0, k).
// ---------------------------------------------------------------------------

// Node rows: W1 = C_0 + sum_h V_h^T C_h; W2 = op(T) W1; C_0 -= W2;
// C_h -= V_h W2.  The children are stacked with V_0 = I, so that the node is
// one product of the leaf kernel's form over kArity x 32 rows: wavefront w
// owns children 2w and 2w + 1 (64 rows) and reads their rows of V and C
// straight into the MFMA operand layout; rows r >= w of a child are zero.
template <bool FORM>
__global__ __launch_bounds__(256, 2) void qr_tree_wy(QrArgs q, int p, int s) {
  constexpr int RW = kArity * kPanel / 4;   // rows per wavefront (two children)
  constexpr int KS = RW / 4;
  constexpr int RB = RW / 16;
  static_assert(kPanel == 32 && kTrailN == kPanel && kArity == 8, "fragment shapes");
  __shared__ double Wp[4][kPanel][kT];
  __shared__ double T[kPanel][kT], W2[kPanel][kT];
  __shared__ int tops[kArity];
  const int a = blockIdx.x * s * kArity;
  const int mat = blockIdx.y;
  const int N = q.N, k = q.k, nb = q.nb;
  if (a + s >= nb) return;
  const int nch = node_children(a, s, nb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int cb = (FORM ? c0 : c0 + w) + blockIdx.z * kTrailN;
  if (cb >= k) return;
  const int nc = min(kTrailN, k - cb);
  if (tid < kArity) tops[tid] = tid < nch ? top_row(a + tid * s, c0, N, nb) : 0;
  const double* A = q.A[mat];
  double* M = FORM ? q.E[mat] : q.A[mat];
  const long sl = slot(mat, p, a + s, nb, q.P);
  for (int idx = tid; idx < kPanel * kPanel; idx += 256) {
    const int i = idx / kPanel, l = idx % kPanel;
    T[i][l] = (i < w && l < w) ? q.Tn[sl * kPanel * kPanel + idx] : 0.0;
  }
  __syncthreads();
  // stacked row u = 32 h + r of child h
  auto vval = [&](int u, int c) -> double {
    const int h = u >> 5, r = u & 31;
    if (h >= nch || r >= w || c >= w) return 0.0;
    if (h == 0) return r == c ? 1.0 : 0.0;
    return r <= c ? A[(long)(tops[h] + r) * k + c0 + c] : 0.0;
  };
  auto cval = [&](int u, int c) -> double {
    const int h = u >> 5, r = u & 31;
    return (h < nch && r < w && c < nc) ? M[(long)(tops[h] + r) * k + cb + c] : 0.0;
  };
  const int r0 = RW * wave, li = lane & 15, lk = lane >> 4;
  {
    double vf[KS][2], cf[KS][2];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const int rr = r0 + 4 * t + lk;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        vf[t][i] = vval(rr, 16 * i + li);
        cf[t][i] = cval(rr, 16 * i + li);
      }
    }
    v4d acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(vf[t][i], cf[t][j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) Wp[wave][16 * i + lk + 4 * r][16 * j + li] = acc[i][j][r];
  }
  __syncthreads();
  {
    const int bi = wave >> 1, bj = wave & 1;
    v4d a2 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < kPanel / 4; ++t) {
      const int l = 4 * t + lk, i = 16 * bi + li, c = 16 * bj + li;
      const double tv = FORM ? T[i][l] : T[l][i];
      const double w1 = (Wp[0][l][c] + Wp[1][l][c]) + (Wp[2][l][c] + Wp[3][l][c]);
      a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(tv, w1, a2, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) W2[16 * bi + lk + 4 * r][16 * bj + li] = a2[r];
  }
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int rr0 = r0 + 16 * rb;
    if ((rr0 >> 5) >= nch) break;
    v4d u[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int t = 0; t < kPanel / 4; ++t) {
      const double av = vval(rr0 + li, 4 * t + lk);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        u[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, W2[4 * t + lk][16 * j + li], u[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int uu = rr0 + lk + 4 * r, col = 16 * j + li;
        const int h = uu >> 5, rw = uu & 31;
        if (h < nch && rw < w && col < nc) {
          double* pc = M + (long)(tops[h] + rw) * k + cb + col;
          *pc = *pc - u[j][r];
        }
      }
  }
}

// Leaf rows: C -= V op(T) (V^T C), V unit lower-trapezoidal (implicit ones,
// zeros above).  Wavefront w owns rows 48 w .. 48 w + 47 of the leaf and
// reads its rows of V and C from global memory straight into the operand
// layout of v_mfma_f64_16x16x4 (lane l: row l/16 of a 4-row k-step, column
// l%16 of a 16-column block), so neither block is staged in LDS: the
// wavefronts' partial products V_w^T C_w meet in LDS, every wavefront forms
// one 16 x 16 block of W2 = op(T) W1 from their sum, and each then updates
// its own rows, C_w -= V_w W2.  About 50 KB of LDS lets several workgroups
// share a CU.
template <bool FORM>
__global__ __launch_bounds__(256, 2) void qr_leaf_wy(QrArgs q, int p) {
  constexpr int RW = kLeafRows / 4;   // rows per wavefront
  constexpr int KS = RW / 4;          // k-steps over a wavefront's rows
  constexpr int RB = RW / 16;         // 16-row blocks of a wavefront's rows
  static_assert(kPanel == 32 && kTrailN == kPanel && RW % 16 == 0, "fragment shapes");
  __shared__ double Wp[4][kPanel][kT];
  __shared__ double T[kPanel][kT], W2[kPanel][kT];
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int cb = (FORM ? c0 : c0 + w) + blockIdx.z * kPanel;
  if (cb >= k) return;
  const int nc = min(kPanel, k - cb);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  const double* A = q.A[mat];
  double* M = FORM ? q.E[mat] : q.A[mat];
  const long sl = slot(mat, p, leaf, nb, q.P);
  auto vval = [&](int r, int c) -> double {
    if (r >= m || c >= w) return 0.0;
    return r > c ? A[(long)(a0 + r) * k + c0 + c] : (r == c ? 1.0 : 0.0);
  };
  auto cval = [&](int r, int c) -> double {
    return (r < m && c < nc) ? M[(long)(a0 + r) * k + cb + c] : 0.0;
  };
  // T (w x w; entries outside it are never read)
  for (int idx = tid; idx < kPanel * kPanel; idx += 256) {
    const int i = idx / kPanel, l = idx % kPanel;
    T[i][l] = (i < w && l < w) ? q.Tl[sl * kPanel * kPanel + idx] : 0.0;
  }
  const int r0 = RW * wave, li = lane & 15, lk = lane >> 4;
  {
    double vf[KS][2], cf[KS][2];
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const int rr = r0 + 4 * t + lk;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        vf[t][i] = vval(rr, 16 * i + li);
        cf[t][i] = cval(rr, 16 * i + li);
      }
    }
    v4d acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(vf[t][i], cf[t][j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) Wp[wave][16 * i + lk + 4 * r][16 * j + li] = acc[i][j][r];
  }
  __syncthreads();
  {
    // W2 block (bi, bj) = op(T) W1 with W1 the sum of the partials in wave order
    const int bi = wave >> 1, bj = wave & 1;
    v4d a2 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < kPanel / 4; ++t) {
      const int l = 4 * t + lk, i = 16 * bi + li, c = 16 * bj + li;
      const double tv = FORM ? T[i][l] : T[l][i];
      const double w1 = (Wp[0][l][c] + Wp[1][l][c]) + (Wp[2][l][c] + Wp[3][l][c]);
      a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(tv, w1, a2, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) W2[16 * bi + lk + 4 * r][16 * bj + li] = a2[r];
  }
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int rr0 = r0 + 16 * rb;
    if (rr0 >= m) break;
    v4d u[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int t = 0; t < kPanel / 4; ++t) {
      const double av = vval(rr0 + li, 4 * t + lk);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        u[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, W2[4 * t + lk][16 * j + li], u[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rr0 + lk + 4 * r, col = 16 * j + li;
        if (row < m && col < nc) {
          double* pc = M + (long)(a0 + row) * k + cb + col;
          *pc = *pc - u[j][r];
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

  // factorisation: per panel the leaves, then the tree levels; each factor
  // launch is followed by the update of the trailing columns it leaves
  for (int p = 0; p < pl.P; ++p) {
    const int c0 = p * kPanel, w = std::min(kPanel, k - c0);
    const int trail = (k - c0 - w + kTrailN - 1) / kTrailN;
    qr_leaf_factor<<<dim3(pl.nb, count), 256, 0, s>>>(q, p);
    if (trail) qr_leaf_wy<false><<<dim3(pl.nb, count, trail), 256, 0, s>>>(q, p);
    for (int L = 0, st = 1; L < pl.depth; ++L, st *= kArity) {
      const int nodes = (pl.nb + st * kArity - 1) / (st * kArity);
      qr_tree_factor<<<dim3(nodes, count), 256, 0, s>>>(q, p, st);
      if (trail) qr_tree_wy<false><<<dim3(nodes, count, trail), 256, 0, s>>>(q, p, st);
    }
  }
  const long total = (long)N * k;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  qr_init_e<<<dim3(blocks, count), 256, 0, s>>>(q);
  for (int p = pl.P - 1; p >= 0; --p) {
    const int chunks = (k - p * kPanel + kTrailN - 1) / kTrailN;
    for (int L = pl.depth - 1; L >= 0; --L) {
      int st = 1;
      for (int i = 0; i < L; ++i) st *= kArity;
      const int nodes = (pl.nb + st * kArity - 1) / (st * kArity);
      qr_tree_wy<true><<<dim3(nodes, count, chunks), 256, 0, s>>>(q, p, st);
    }
    qr_leaf_wy<true><<<dim3(pl.nb, count, chunks), 256, 0, s>>>(q, p);
  }
  qr_diag_sign<<<dim3(1, count), 256, 0, s>>>(q);
  qr_sign_copy<<<dim3(blocks, count), 256, 0, s>>>(q);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace sictm
