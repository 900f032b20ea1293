// Tall-skinny Householder QR with explicit Q (QR-based projector section,
// step 1: the isometries are re-orthonormalised by a QR decomposition after
// every power update).
//
// Communication-avoiding layout for N x k blocks with N >> k:
//  * the rows are split into `nb` leaves of at most kLeafRows rows (leaf 0
//    holds at least k rows); the columns are processed in panels of width
//    kPanel;
//  * per panel, every leaf factors its active rows of the panel with
//    Householder reflectors held in LDS and applies them to its trailing
//    columns (one workgroup per leaf);
//  * the w x w triangles that the leaves leave in their top rows are then
//    combined pairwise up a binary tree; a combine of two upper triangles has
//    reflectors [e_j; v] whose lower part v is itself upper triangular, so it
//    is stored in the place of the absorbed triangle; the tree node applies
//    its reflectors to the trailing columns of its 2w rows;
//  * Q = prod_p L_p T_p [I; 0] is then formed by applying the tree and leaf
//    reflectors in reverse order to [I_k; 0], restricted to the columns that
//    can be non-trivial, and each column c is multiplied by sign(R_cc) so
//    that R has a non-negative diagonal.
// Reflectors follow the LAPACK dlarfg convention: beta = -sign(alpha) * norm,
// tau = (beta - alpha) / beta, and tau = 0 (H = I) when the part below the
// diagonal is exactly zero, so rank-deficient blocks never divide by zero.
// A wavefront owns one column at a time; rows are spread over its 64 lanes
// and reductions use cross-lane shuffles, so no workgroup barrier is needed
// inside the reflector application to a column.

#include "common.h"

namespace sictm {
namespace {

constexpr int kPanel = 32;
constexpr int kLeafRows = 256;
constexpr int kRowsPerLane = kLeafRows / 64;

struct QrPlan {
  int N, k, nb, P, depth;
};

__host__ __device__ inline int leaf_start(int i, int N, int nb) {
  return (int)(((long)i * N) / nb);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

struct QrArgs {
  double* A[kMaxProb];   // matrices being factored (in place)
  double* E[kMaxProb];   // explicit Q being formed
  double* O[kMaxProb];   // destination of Q
  double* tau;           // [count][P][nb][kPanel] leaf taus
  double* tau_node;      // [count][P][nb][kPanel] tree taus, indexed by right child
  double* sgn;           // [count][k] signs of the diagonal of R
  int count, N, k, nb, P;
};

__device__ __forceinline__ double* tau_at(double* base, int mat, int p, int leaf, int nb, int P) {
  return base + (((long)mat * P + p) * nb + leaf) * kPanel;
}

// Applies the w reflectors of a leaf panel (unit diagonal implicit, V[j][r]
// for r > j) to one column x held in LDS, in order (Q^T) or reversed (Q).
// Lane l owns rows l, l+64, ... for the whole call.
__device__ __forceinline__ void apply_panel(const double (*V)[kLeafRows], const double* tau_s,
                                            double* x_lds, int m, int w, int lane, bool reverse) {
  double x[kRowsPerLane];
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int r = lane + 64 * t;
    x[t] = r < m ? x_lds[r] : 0.0;
  }
  for (int jj = 0; jj < w; ++jj) {
    const int j = reverse ? w - 1 - jj : jj;
    const double tau = tau_s[j];
    if (tau == 0.0) continue;
    double v[kRowsPerLane];
    double d = 0.0;
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) {
      const int r = lane + 64 * t;
      v[t] = (r > j && r < m) ? V[j][r] : (r == j ? 1.0 : 0.0);
      d += v[t] * x[t];
    }
    const double f = tau * wave_sum(d);
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) x[t] -= f * v[t];
  }
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int r = lane + 64 * t;
    if (r < m) x_lds[r] = x[t];
  }
}

// ---------------------------------------------------------------------------
// leaf factorisation of panel p + update of its trailing columns
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void qr_leaf_factor(QrArgs q, int p) {
  __shared__ double V[kPanel][kLeafRows];     // panel, column-major
  __shared__ double Cc[kPanel][kLeafRows];    // trailing chunk, column-major
  __shared__ double tau_s[kPanel];
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  double* A = q.A[mat];

  // load panel rows [a0, e) x columns [c0, c0+w)
  for (int idx = tid; idx < kPanel * kLeafRows; idx += 256) {
    const int r = idx / kPanel, c = idx % kPanel;
    double v = 0.0;
    if (r < m && c < w) v = A[(long)(a0 + r) * k + c0 + c];
    V[c][r] = v;
  }
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
      for (int c = j + 1 + wave; c < w; c += 4) {
        double d = 0.0;
        for (int r = j + 1 + lane; r < m; r += 64) d += V[j][r] * V[c][r];
        d = wave_sum(d) + V[c][j];
        const double f = tau * d;
        for (int r = j + 1 + lane; r < m; r += 64) V[c][r] -= f * V[j][r];
        if (lane == 0) V[c][j] -= f;
      }
    }
    __syncthreads();
  }

  // write back R (upper) and V (below the diagonal), and the taus
  for (int idx = tid; idx < m * w; idx += 256) {
    const int r = idx / w, c = idx % w;
    A[(long)(a0 + r) * k + c0 + c] = V[c][r];
  }
  if (tid < w) tau_at(q.tau, mat, p, leaf, nb, q.P)[tid] = tau_s[tid];

  // trailing columns [c0+w, k) in chunks of kPanel
  for (int cb = c0 + w; cb < k; cb += kPanel) {
    const int nc = min(kPanel, k - cb);
    __syncthreads();
    for (int idx = tid; idx < m * kPanel; idx += 256) {
      const int r = idx / kPanel, c = idx % kPanel;
      if (c < nc) Cc[c][r] = A[(long)(a0 + r) * k + cb + c];
    }
    __syncthreads();
    for (int c = wave; c < nc; c += 4) apply_panel(V, tau_s, Cc[c], m, w, lane, false);
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
  __shared__ double Ra[kPanel][kPanel + 1];   // [row][col]
  __shared__ double Rb[kPanel][kPanel + 1];
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
  for (int idx = tid; idx < kPanel * kPanel; idx += 256) {
    const int r = idx / kPanel, c = idx % kPanel;
    const bool up = r <= c && r < w && c < w;
    Ra[r][c] = up ? A[(long)(ta + r) * k + c0 + c] : 0.0;
    Rb[r][c] = up ? A[(long)(tb + r) * k + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (wave == 0) {
      double ss = 0.0;
      if (lane <= j) ss = Rb[lane][j] * Rb[lane][j];
      ss = wave_sum(ss);
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
      for (int c = j + 1 + wave; c < w; c += 4) {
        double d = (lane <= j) ? Rb[lane][j] * Rb[lane][c] : 0.0;
        d = wave_sum(d) + Ra[j][c];
        const double f = tau * d;
        if (lane <= j) Rb[lane][c] -= f * Rb[lane][j];
        if (lane == 0) Ra[j][c] -= f;
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
  if (tid < w) tau_at(q.tau_node, mat, p, b, nb, q.P)[tid] = tau_s[tid];
  // trailing columns: rows ta..ta+w and tb..tb+w; one wavefront per column,
  // lane r < w holds row r of both blocks
  for (int c = c0 + w + wave; c < k; c += 4) {
    double xa = (lane < w) ? A[(long)(ta + lane) * k + c] : 0.0;
    double xb = (lane < w) ? A[(long)(tb + lane) * k + c] : 0.0;
    for (int j = 0; j < w; ++j) {
      const double tau = tau_s[j];
      if (tau == 0.0) continue;
      const double vb = (lane <= j) ? Rb[lane][j] : 0.0;
      double d = wave_sum(vb * xb) + __shfl(xa, j, 64);
      const double f = tau * d;
      xb -= f * vb;
      if (lane == j) xa -= f;
    }
    if (lane < w) {
      A[(long)(ta + lane) * k + c] = xa;
      A[(long)(tb + lane) * k + c] = xb;
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

__global__ __launch_bounds__(256) void qr_tree_apply(QrArgs q, int p, int L) {
  __shared__ double Vb[kPanel][kPanel + 1];
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
  const double* A = q.A[mat];
  double* E = q.E[mat];
  for (int idx = tid; idx < kPanel * kPanel; idx += 256) {
    const int r = idx / kPanel, c = idx % kPanel;
    Vb[r][c] = (r <= c && r < w && c < w) ? A[(long)(tb + r) * k + c0 + c] : 0.0;
  }
  if (tid < kPanel) tau_s[tid] = tid < w ? tau_at(q.tau_node, mat, p, b, nb, q.P)[tid] : 0.0;
  __syncthreads();
  for (int c = c0 + wave; c < k; c += 4) {
    double xa = (lane < w) ? E[(long)(ta + lane) * k + c] : 0.0;
    double xb = (lane < w) ? E[(long)(tb + lane) * k + c] : 0.0;
    for (int j = w - 1; j >= 0; --j) {
      const double tau = tau_s[j];
      if (tau == 0.0) continue;
      const double vb = (lane <= j) ? Vb[lane][j] : 0.0;
      double d = wave_sum(vb * xb) + __shfl(xa, j, 64);
      const double f = tau * d;
      xb -= f * vb;
      if (lane == j) xa -= f;
    }
    if (lane < w) {
      E[(long)(ta + lane) * k + c] = xa;
      E[(long)(tb + lane) * k + c] = xb;
    }
  }
}

__global__ __launch_bounds__(256) void qr_leaf_apply(QrArgs q, int p) {
  __shared__ double V[kPanel][kLeafRows];
  __shared__ double Cc[kPanel][kLeafRows];
  __shared__ double tau_s[kPanel];
  const int leaf = blockIdx.x, mat = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = q.N, k = q.k, nb = q.nb;
  const int c0 = p * kPanel, w = min(kPanel, k - c0);
  const int s = leaf_start(leaf, N, nb), e = leaf_start(leaf + 1, N, nb);
  const int a0 = (leaf == 0) ? c0 : s;
  const int m = e - a0;
  const double* A = q.A[mat];
  double* E = q.E[mat];
  for (int idx = tid; idx < kPanel * kLeafRows; idx += 256) {
    const int r = idx / kPanel, c = idx % kPanel;
    double v = 0.0;
    if (r < m && c < w && r > c) v = A[(long)(a0 + r) * k + c0 + c];
    V[c][r] = v;
  }
  if (tid < kPanel) tau_s[tid] = tid < w ? tau_at(q.tau, mat, p, leaf, nb, q.P)[tid] : 0.0;
  for (int cb = c0; cb < k; cb += kPanel) {
    const int nc = min(kPanel, k - cb);
    __syncthreads();
    for (int idx = tid; idx < m * kPanel; idx += 256) {
      const int r = idx / kPanel, c = idx % kPanel;
      if (c < nc) Cc[c][r] = E[(long)(a0 + r) * k + cb + c];
    }
    __syncthreads();
    for (int c = wave; c < nc; c += 4) apply_panel(V, tau_s, Cc[c], m, w, lane, true);
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
  const size_t taus = 2ull * count * pl.P * pl.nb * kPanel;
  const size_t e = (size_t)count * N * k + (size_t)count * k;
  return (taus + e) * sizeof(double);
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
  double* base = (double*)ws;
  q.tau = base;
  q.tau_node = base + (size_t)count * pl.P * pl.nb * kPanel;
  double* e = q.tau_node + (size_t)count * pl.P * pl.nb * kPanel;
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
