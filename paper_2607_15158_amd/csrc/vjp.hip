// Adjoint of one SI-CTMRG move: the vector-Jacobian product
//   (C, T, X, Y^T, A) -> (C', T', X', Y^T')
// that the paper's differentiation of CTMRG is built from (Differentiable
// fixed point passage, eq. implicit: the fixed-point gradient needs only
// VJPs of the single move; the timing figure unrolls the moves instead).
//
// The move is recomputed from the caller's input state with its
// intermediates kept in a caller-owned workspace (the "tape"), then the
// cotangents are propagated back through every step on the GPU:
//   - unit-norm scaling:  x_bar = (y_bar - y <y, y_bar>) / |x|;
//   - renormalisation (Fig. 1): the GEMM chain of C' = P_r Ct P_l and
//     T' = P_r (T a) P_l, with the a-absorption's permutations inverted;
//   - projectors (eq. projectors_diag) with the pseudo-inverse mask and the
//     signs of the sign rule held constant;
//   - the small SVD of rho (eq. rho_hat_diag): for rho = u s v^T (square,
//     full u, v),  rho_bar = u [F o (u^T u_bar - u_bar^T u) s + diag(s_bar)
//     + s F o (v^T v_bar - v_bar^T v)] v^T,  F_ij = 1 / (s_j^2 - s_i^2);
//   - the QRs of the subspace steps (eq. xy_iter, stabilised): for H = Q R
//     with only Q used,  H_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T;
//   - every application of an enlarged corner: the block cotangent goes
//     back through op(Ct)^T, the corner cotangent gains a rank-k term;
//   - enlarged corners (eq. rho_M_diag) and the double layer (eq.
//     double_layer).
// Discrete choices (QR diagonal signs, sign rule, pseudo-inverse mask) are
// piecewise constant in the input and are held fixed, as in any
// reverse-mode treatment of the move.

#include "../../include/ctm.h"

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <string>
#include <vector>

#include "common.h"
#include "elem.h"
#include "vjp.h"

using namespace sictm;

namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// dst[i] (=, or += when acc) alpha * src[i0 s0 + i1 s1 + i2 s2 + i3 s3] over
// the index box n0 x n1 x n2 x n3 (row-major in dst).  I is the type of the
// flat index and its decomposition: 32-bit unsigned when the box holds fewer
// than 2^31 elements (the integer divisions are the kernel's main cost),
// 64-bit otherwise.
template <typename I>
__global__ __launch_bounds__(256) void k_gather4(const double* __restrict__ src,
                                                 double* __restrict__ dst, int n0, int n1,
                                                 int n2, int n3, long s0, long s1, long s2,
                                                 long s3, double alpha, int acc) {
  const I total = (I)n0 * (I)n1 * (I)n2 * (I)n3;
  for (I i = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x; i < total;
       i += (I)gridDim.x * (I)blockDim.x) {
    I r = i;
    const I i3 = r % (I)n3;
    r /= (I)n3;
    const I i2 = r % (I)n2;
    r /= (I)n2;
    const I i1 = r % (I)n1;
    const I i0 = r / (I)n1;
    const double v =
        alpha * src[(long)i0 * s0 + (long)i1 * s1 + (long)i2 * s2 + (long)i3 * s3];
    dst[i] = acc ? dst[i] + v : v;
  }
}

// The transposing case of k_gather4 (n0 = n1 = 1, s2 = 1):
// dst[i2, i3] (=|+=) alpha * src[i2 + i3 s3], through 32 x 32 LDS tiles so
// that the reads (along i2) and the writes (along i3) are both unit-stride.
// One workgroup per tile; the padded row length 33 keeps the column reads of
// the tile on distinct banks.
__global__ __launch_bounds__(256) void k_transpose_tiles(const double* __restrict__ src,
                                                         double* __restrict__ dst, int n2,
                                                         int n3, long s3, double alpha, int acc) {
  __shared__ double t[32][33];
  const int tiles2 = (n2 + 31) / 32;
  const int b2 = blockIdx.x % tiles2, b3 = blockIdx.x / tiles2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int i3 = b3 * 32 + ty + k, i2 = b2 * 32 + tx;
    if (i3 < n3 && i2 < n2) t[ty + k][tx] = src[(long)i3 * s3 + i2];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int i2 = b2 * 32 + ty + k, i3 = b3 * 32 + tx;
    if (i2 < n2 && i3 < n3) {
      const double v = alpha * t[tx][ty + k];
      double* p = dst + (long)i2 * n3 + i3;
      *p = acc ? *p + v : v;
    }
  }
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ x, long n, double v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = v;
}

__device__ __forceinline__ double block_sum256(double x, double* sh) {
  x = wave_sum64(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

struct DotArgs {
  const double* x[8];
  const double* y[8];
  long n[8];
  double* out;
};

// out[t] = <x_t, y_t> for up to 8 pairs.  Block (b, t) adds the products
// b * 256 + j + m * kDotParts * 256 of pair t into part[t * kDotParts + b];
// k_dots_final adds a pair's partial sums in block order, so the result does
// not depend on scheduling.
constexpr int kDotParts = 128;

__global__ __launch_bounds__(256) void k_dots_part(DotArgs a, double* part) {
  __shared__ double sh[4];
  const int t = blockIdx.y;
  const double* x = a.x[t];
  const double* y = a.y[t];
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n[t]; i += (long)kDotParts * 256)
    acc += x[i] * y[i];
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[(long)t * kDotParts + blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_dots_final(DotArgs a, const double* part) {
  __shared__ double sh[4];
  const int t = blockIdx.x;
  double acc = threadIdx.x < kDotParts ? part[(long)t * kDotParts + threadIdx.x] : 0.0;
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) a.out[t] = acc;
}

int launch_dots(const DotArgs& a, int count, double* part, hipStream_t s) {
  k_dots_part<<<dim3(kDotParts, count), 256, 0, s>>>(a, part);
  CTM_HIP_TRY(hipGetLastError());
  k_dots_final<<<count, 256, 0, s>>>(a, part);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

struct NormBwdArgs {
  const double* y[8];    // unit-norm outputs
  const double* yb[8];   // their cotangents
  double* xb[8];         // cotangents of the unscaled tensors
  long n[8];
  const double* dot;     // <y_t, yb_t>
  const double* nrm;     // |x_t|
};

__global__ __launch_bounds__(256) void k_norm_bwd(NormBwdArgs a) {
  const int t = blockIdx.y;
  const double dt = a.dot[t], inv = 1.0 / a.nrm[t];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n[t]; i += (long)gridDim.x * 256)
    a.xb[t][i] = (a.yb[t][i] - a.y[t][i] * dt) * inv;
}

struct SmallArgs {
  const double* in[8];
  double* out[8];
  int n;
};

// out = tril(in) + tril(in, -1)^T (the lower triangle mirrored up).
__global__ __launch_bounds__(256) void k_copyltu(SmallArgs a) {
  const int b = blockIdx.y, n = a.n;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n * n; idx += gridDim.x * 256) {
    const int i = idx / n, j = idx % n;
    a.out[b][idx] = i >= j ? a.in[b][idx] : a.in[b][j * n + i];
  }
}

// Inverse of an upper-triangular n x n matrix (n <= 256), one block per
// matrix, thread j owns column j: back substitution row by row.  A zero
// diagonal entry (a rank-deficient block) gives a zero row.
__global__ __launch_bounds__(256) void k_tri_inv(SmallArgs a) {
  const int b = blockIdx.x, n = a.n, j = threadIdx.x;
  const double* R = a.in[b];
  double* X = a.out[b];
  if (j >= n) return;
  for (int i = n - 1; i >= 0; --i) {
    double v = 0.0;
    if (j >= i) {
      double acc = i == j ? 1.0 : 0.0;
      for (int l = i + 1; l <= j; ++l) acc -= R[(long)i * n + l] * X[(long)l * n + j];
      const double d = R[(long)i * n + i];
      v = d != 0.0 ? acc / d : 0.0;
    }
    X[(long)i * n + j] = v;
  }
}

// Same result as k_tri_inv, operation for operation, for n <= kTriLds: the
// upper triangle of X lives in LDS, row-packed (row l starts at
// l n - l (l - 1) / 2, so the threads of a row step read consecutive words),
// and row i of R is staged in LDS for step i.  Every thread takes part in
// the two barriers of each step.
constexpr int kTriLds = 192;

__global__ __launch_bounds__(256) void k_tri_inv_lds(SmallArgs a) {
  __shared__ double Xs[kTriLds * (kTriLds + 1) / 2];
  __shared__ double Rrow[kTriLds];
  const int b = blockIdx.x, n = a.n, j = threadIdx.x;
  const double* R = a.in[b];
  double* X = a.out[b];
  auto at = [n](int l, int c) { return l * n - l * (l - 1) / 2 + (c - l); };   // l <= c
  for (int i = n - 1; i >= 0; --i) {
    __syncthreads();
    if (j < n) Rrow[j] = R[(long)i * n + j];
    __syncthreads();
    if (j < n && j >= i) {
      double acc = i == j ? 1.0 : 0.0;
      // unrolled so that the LDS loads of later terms issue while earlier
      // terms are accumulated; the accumulation order is unchanged
#pragma unroll 4
      for (int l = i + 1; l <= j; ++l) acc -= Rrow[l] * Xs[at(l, j)];
      const double d = Rrow[i];
      Xs[at(i, j)] = d != 0.0 ? acc / d : 0.0;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e % n;
    X[e] = c >= r ? Xs[at(r, c)] : 0.0;
  }
}

struct PrepArgs {
  const double* u[4];
  const double* v[4];
  const double* s[4];
  const double* sg[4];
  double* us[4];
  double* vs[4];
  double* sinv[4];
  double* vsc[4];
  double* usc[4];
  int k, keep;
  double rtol;
};

// Signed singular vectors, s^-1/2 with the cut s_i <= rtol s_1 (and beyond
// keep) set to 0, and the scaled kept columns v_s sinv, u_s sinv.
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  const int b = blockIdx.y, k = a.k, keep = a.keep;
  const double s0 = a.s[b][0];
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < k * k; idx += gridDim.x * 256) {
    const int r = idx / k, c = idx % k;
    const double sc = c < keep && s0 > 0.0 && a.s[b][c] > a.rtol * s0 ? 1.0 / sqrt(a.s[b][c]) : 0.0;
    const double us = a.u[b][idx] * a.sg[b][c], vs = a.v[b][idx] * a.sg[b][c];
    a.us[b][idx] = us;
    a.vs[b][idx] = vs;
    if (c < keep) {
      a.vsc[b][r * keep + c] = vs * sc;
      a.usc[b][r * keep + c] = us * sc;
    }
    if (r == 0) a.sinv[b][c] = sc;
  }
}

struct ProjBwdArgs {
  const double* us[4];
  const double* vs[4];
  const double* sinv[4];
  const double* vscb[4];   // A^T P_l_bar    (k x keep)
  const double* uscb[4];   // B^T P_rT_bar   (k x keep)
  double* ub[4];           // in: recycle term Y^T Y'_bar; out: full u_bar
  double* vb[4];
  double* sb[4];
  int k, keep;
};

// Adds the projector terms to u_bar, v_bar and forms s_bar from
// d(s^-1/2)/ds = -s^-3/2 / 2 = -sinv^3 / 2 (zero where the cut applies).
__global__ __launch_bounds__(256) void k_proj_bwd(ProjBwdArgs a) {
  const int b = blockIdx.x, k = a.k, keep = a.keep;
  for (int c = threadIdx.x; c < k; c += 256) {
    if (c >= keep) {
      a.sb[b][c] = 0.0;
      continue;
    }
    const double si = a.sinv[b][c];
    double acc = 0.0;
    for (int r = 0; r < k; ++r) {
      const double vq = a.vscb[b][r * keep + c], uq = a.uscb[b][r * keep + c];
      a.vb[b][r * k + c] += vq * si;
      a.ub[b][r * k + c] += uq * si;
      acc += vq * a.vs[b][r * k + c] + uq * a.us[b][r * k + c];
    }
    a.sb[b][c] = si > 0.0 ? -0.5 * acc * si * si * si : 0.0;
  }
}

struct KmatArgs {
  const double* Ju[4];   // u^T u_bar
  const double* Jv[4];   // v^T v_bar
  const double* s[4];
  const double* sb[4];
  double* K[4];
  int n;
};

// Inner matrix of the SVD adjoint.  The inverse gaps 1 / (s_j^2 - s_i^2)
// carry a Lorentzian broadening relative to the pair, (1e-14 (s_i^2 +
// s_j^2))^2, which only changes pairs degenerate to rounding: the kept
// singular values of rho span many orders of magnitude, so a broadening on
// the scale of s_1^2 would suppress the gaps among the small ones.
// Singular values at or below the forward SVD's zero cut (1e-15 of the
// Frobenius norm) count as exact zeros: their vectors are a completion
// chosen by the forward pass, a rotation among them changes no output, and
// the terms of a pair of them vanish (both carry a factor s = 0).
__global__ __launch_bounds__(256) void k_svd_kmat(KmatArgs a) {
  const int b = blockIdx.y, n = a.n;
  const double* s = a.s[b];
  double f2 = 0.0;
  for (int t = 0; t < n; ++t) f2 += s[t] * s[t];
  const double cut = 1e-15 * sqrt(f2);
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n * n; idx += gridDim.x * 256) {
    const int i = idx / n, j = idx % n;
    double v;
    if (i == j) {
      v = a.sb[b][i];
    } else {
      const double si = s[i] > cut ? s[i] : 0.0, sj = s[j] > cut ? s[j] : 0.0;
      if (si == 0.0 && sj == 0.0) {
        v = 0.0;
      } else {
        const double dl = sj * sj - si * si;
        const double e2 = 1e-14 * (si * si + sj * sj);
        const double F = dl / (dl * dl + e2 * e2);
        v = F * (a.Ju[b][idx] - a.Ju[b][j * n + i]) * sj +
            si * F * (a.Jv[b][idx] - a.Jv[b][j * n + i]);
      }
    }
    a.K[b][idx] = v;
  }
}

// msym[ket, bra] = ab[ket, bra] + ab[bra, ket] with ab in the double-layer
// order [(uU),(lL),(dD),(rR)] and ket = (u,l,d,r), bra = (U,L,D,R).
__global__ __launch_bounds__(256) void k_dl_sym(const double* __restrict__ ab,
                                                double* __restrict__ out, int D) {
  const long D4 = (long)D * D * D * D, Dl = (long)D * D;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < D4 * D4; idx += (long)gridDim.x * 256) {
    long p = idx / D4, q = idx % D4;
    const long r0 = p % D, d0 = (p / D) % D, l0 = (p / Dl) % D, u0 = p / (Dl * D);
    const long r1 = q % D, d1 = (q / D) % D, l1 = (q / Dl) % D, u1 = q / (Dl * D);
    const long i1 = (((u0 * D + u1) * Dl + (l0 * D + l1)) * Dl + (d0 * D + d1)) * Dl + (r0 * D + r1);
    const long i2 = (((u1 * D + u0) * Dl + (l1 * D + l0)) * Dl + (d1 * D + d0)) * Dl + (r1 * D + r0);
    out[idx] = ab[i1] + ab[i2];
  }
}

// ---------------------------------------------------------------------------
// buffers of one adjoint call, carved from the caller's workspace
// ---------------------------------------------------------------------------
struct Dims {
  int d, D, Dl, x, N, k, nsi;
};

struct Bufs {
  double *Ct[4], *Ctb[4], *CT[4], *Wc[4], *apT[4];
  std::vector<double*> tape[8];           // 10 n_si blocks per side
  double *W1[4], *Ab[4], *W2[4], *Bt[4];
  double *rho[4], *u[4], *v[4], *us[4], *vs[4], *s[4], *sg[4], *sinv[4], *vsc[4], *usc[4];
  double *Pl[4], *Prt[4], *Zc[4], *Z1[4], *Z2[4];
  double *Cn[4], *Tn[4], *Ch[4], *Th[4];
  double *nrm, *dots;
  double *Chb[4], *Thb[4], *Plb[4], *Prtb[4], *Zcb;
  double *Sa, *Sb, *St;                   // N x N scratch, and a transposition buffer
  double *ab, *apb, *msym;
  double *Qb[8], *Hb[8], *Yq[8], *tr[8];
  double *R[8], *Rinv[8], *RinvT[8], *Mm[8], *Mc[8];
  double *Ju[4], *Jv[4], *Km[4], *uK[4], *vsT[4], *usT[4], *rhob[4], *rhobT[4];
  double *vscb[4], *uscb[4], *vscT[4], *uscT[4], *ub[4], *vb[4], *sb[4];
  double *smallT;                         // x x x / k x k transposes
  double *fp_v[2], *fp_dot;               // fixed-point iteration: cotangent ping-pong
  double* dpart;                          // partial sums of the dot products (8 * kDotParts)
  double *PTs[4], *QTs[4];                // per corner: 8 transposed blocks stacked along K
  double *Ga[4], *Gb[4];                  // per corner / edge N x N scratch (batched launches)
  double *apb4[4];                        // per corner / edge cotangents of the permuted a
  void *qr_ws, *svd_ws;
};

struct Carver {
  char* base = nullptr;
  size_t off = 0;
  std::vector<std::pair<uintptr_t, uintptr_t>>* reg = nullptr;
  double* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    if (base && reg) reg->push_back({(uintptr_t)p, (uintptr_t)p + count * sizeof(double)});
    off += count * sizeof(double);
    return p;
  }
  void* bytes(size_t n) {
    off = (off + 255) & ~size_t(255);
    void* p = base ? base + off : nullptr;
    if (base && reg) reg->push_back({(uintptr_t)p, (uintptr_t)p + n});
    off += n;
    return p;
  }
};

size_t carve(const Dims& m, Bufs* b, char* base, std::vector<std::pair<uintptr_t, uintptr_t>>* reg) {
  Carver cv;
  cv.base = base;
  cv.reg = reg;
  const size_t N = m.N, k = m.k, x = m.x, Dl = m.Dl, NN = N * N, Nk = N * k;
  const size_t D4 = (size_t)m.D * m.D * m.D * m.D;
  for (int i = 0; i < 4; ++i) {
    b->Ct[i] = cv.take(NN);
    b->Ctb[i] = cv.take(NN);
    b->CT[i] = cv.take(x * Dl * x);
    b->Wc[i] = cv.take(NN);
    b->apT[i] = cv.take(Dl * Dl * Dl * Dl);
  }
  for (int j = 0; j < 8; ++j) {
    b->tape[j].resize(10 * m.nsi);
    for (int t = 0; t < 10 * m.nsi; ++t) b->tape[j][t] = cv.take(Nk);
  }
  for (int i = 0; i < 4; ++i) {
    b->W1[i] = cv.take(Nk);
    b->Ab[i] = cv.take(Nk);
    b->W2[i] = cv.take(Nk);
    b->Bt[i] = cv.take(Nk);
    b->rho[i] = cv.take(k * k);
    b->u[i] = cv.take(k * k);
    b->v[i] = cv.take(k * k);
    b->us[i] = cv.take(k * k);
    b->vs[i] = cv.take(k * k);
    b->s[i] = cv.take(k);
    b->sg[i] = cv.take(k);
    b->sinv[i] = cv.take(k);
    b->vsc[i] = cv.take(k * x);
    b->usc[i] = cv.take(k * x);
    b->Pl[i] = cv.take(N * x);
    b->Prt[i] = cv.take(N * x);
    b->Zc[i] = cv.take(N * x);
    b->Z1[i] = cv.take(NN);
    b->Z2[i] = cv.take(NN);
    b->Cn[i] = cv.take(x * x);
    b->Tn[i] = cv.take(x * Dl * x);
    b->Ch[i] = cv.take(x * x);
    b->Th[i] = cv.take(x * Dl * x);
    b->Chb[i] = cv.take(x * x);
    b->Thb[i] = cv.take(x * Dl * x);
    b->Plb[i] = cv.take(N * x);
    b->Prtb[i] = cv.take(N * x);
    b->Ju[i] = cv.take(k * k);
    b->Jv[i] = cv.take(k * k);
    b->Km[i] = cv.take(k * k);
    b->uK[i] = cv.take(k * k);
    b->vsT[i] = cv.take(k * k);
    b->usT[i] = cv.take(k * k);
    b->rhob[i] = cv.take(k * k);
    b->rhobT[i] = cv.take(k * k);
    b->vscb[i] = cv.take(k * x);
    b->uscb[i] = cv.take(k * x);
    b->vscT[i] = cv.take(k * x);
    b->uscT[i] = cv.take(k * x);
    b->ub[i] = cv.take(k * k);
    b->vb[i] = cv.take(k * k);
    b->sb[i] = cv.take(k);
  }
  b->nrm = cv.take(8);
  b->dots = cv.take(8);
  b->Zcb = cv.take(N * x);
  b->Sa = cv.take(NN);
  b->Sb = cv.take(NN);
  b->St = cv.take(std::max(NN, Nk));
  b->ab = cv.take(Dl * Dl * Dl * Dl);
  b->apb = cv.take(Dl * Dl * Dl * Dl);
  b->msym = cv.take(D4 * D4);
  for (int j = 0; j < 8; ++j) {
    b->Qb[j] = cv.take(Nk);
    b->Hb[j] = cv.take(Nk);
    b->Yq[j] = cv.take(Nk);
    b->tr[j] = cv.take(Nk);
    b->R[j] = cv.take(k * k);
    b->Rinv[j] = cv.take(k * k);
    b->RinvT[j] = cv.take(k * k);
    b->Mm[j] = cv.take(k * k);
    b->Mc[j] = cv.take(k * k);
  }
  b->smallT = cv.take(std::max(x * x, k * k));
  const size_t nstate = 4 * x * x + 4 * x * Dl * x + 8 * Nk + 4;
  b->fp_v[0] = cv.take(nstate);
  b->fp_v[1] = cv.take(nstate);
  b->fp_dot = cv.take(8);
  b->dpart = cv.take((size_t)8 * kDotParts);
  for (int i = 0; i < 4; ++i) {
    b->PTs[i] = cv.take(8 * Nk);
    b->QTs[i] = cv.take(8 * Nk);
    b->Ga[i] = cv.take(NN);
    b->Gb[i] = cv.take(NN);
    b->apb4[i] = cv.take(Dl * Dl * Dl * Dl);
  }
  b->qr_ws = cv.bytes(qr_workspace_bytes(8, m.N, m.k));
  b->svd_ws = cv.bytes(svd_workspace_bytes(4, m.k));
  return cv.off + 256;
}

// ---------------------------------------------------------------------------
// launch helpers with host-side bounds checks
// ---------------------------------------------------------------------------
struct Run {
  ctm_ctx* c;
  hipStream_t st;
  double* sk_part = nullptr;
  int sk_cus = 0;
  std::vector<std::pair<uintptr_t, uintptr_t>> reg;

  bool inside(const void* p, size_t bytes) const {
    const uintptr_t a = (uintptr_t)p;
    for (const auto& r : reg)
      if (a >= r.first && a + bytes <= r.second) return true;
    return false;
  }
  int fail(const std::string& msg) { return vjp_fail(c, CTM_E_SHAPE, msg); }
};

long extent(int n, int div, long s1, long s0) {
  if (n <= 0) return 0;
  return (long)((n - 1) / div) * s1 + (long)std::min(div - 1, n - 1) * s0;
}

GemmBatch rowmajor(int count, int M, int N, int K, long lda, long ldb, long ldc) {
  GemmBatch g{};
  g.count = count;
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

// Float64 GEMM after checking every operand against the registered buffers.
int gemm(Run& r, const GemmBatch& g, bool si = false) {
  if (g.M <= 0 || g.N <= 0) return 0;
  for (int i = 0; i < g.count; ++i) {
    const long ea = g.K <= 0 ? 0
                    : (g.transA[i] ? (long)(g.K - 1) * g.lda + (g.M - 1)
                                   : (long)(g.M - 1) * g.lda + (g.K - 1)) +
                          (long)(g.nbatch - 1) * g.a_bs;
    const long eb = g.K <= 0 ? 0 : (long)(g.K - 1) * g.ldb + (g.N - 1) + (long)(g.nbatch - 1) * g.b_bs;
    const long ec = extent(g.M, g.cdiv_m, g.cs_m1, g.cs_m0) +
                    extent(g.N, g.cdiv_n, g.cs_n1, g.cs_n0) + (long)(g.nbatch - 1) * g.c_bs;
    if (!(g.K <= 0 || r.inside(g.A[i], (size_t)(ea + 1) * 8)) ||
        !(g.K <= 0 || r.inside(g.B[i], (size_t)(eb + 1) * 8)) || !r.inside(g.C[i], (size_t)(ec + 1) * 8))
      return r.fail("adjoint GEMM operand out of its buffer (M=" + std::to_string(g.M) + " N=" +
                    std::to_string(g.N) + " K=" + std::to_string(g.K) + ", problem " +
                    std::to_string(i) + "); launch refused");
  }
  const int rc = si ? launch_gemm_si_balanced(g, r.sk_part, r.sk_cus, r.st)
                     : launch_gemm(g, DT::F64, DT::F64, DT::F64, r.st);
  if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
  return 0;
}

// dst (n0 x n1 x n2 x n3, row-major) (=|+=) alpha * src[strided].
int gather(Run& r, const double* src, double* dst, int n0, int n1, int n2, int n3, long s0,
           long s1, long s2, long s3, bool acc = false, double alpha = 1.0) {
  const long total = (long)n0 * n1 * n2 * n3;
  if (total <= 0) return 0;
  const long es = (long)(n0 - 1) * s0 + (long)(n1 - 1) * s1 + (long)(n2 - 1) * s2 + (long)(n3 - 1) * s3;
  if (!r.inside(src, (size_t)(es + 1) * 8) || !r.inside(dst, (size_t)total * 8))
    return r.fail("adjoint permutation out of its buffer; launch refused");
  const int blocks = (int)std::min<long>(4096, (total + 255) / 256);
  if (n0 == 1 && n1 == 1 && s2 == 1 && n2 >= 32 && n3 >= 32) {
    const long tiles = (long)((n2 + 31) / 32) * ((n3 + 31) / 32);
    k_transpose_tiles<<<(unsigned)tiles, 256, 0, r.st>>>(src, dst, n2, n3, s3, alpha,
                                                         acc ? 1 : 0);
    CTM_HIP_TRY(hipGetLastError());
    return 0;
  }
  // the grid stride is at most 4096 * 256 = 2^20, so a 32-bit index below
  // 2^31 never wraps
  if (total < (1L << 31))
    k_gather4<unsigned><<<blocks, 256, 0, r.st>>>(src, dst, n0, n1, n2, n3, s0, s1, s2, s3,
                                                   alpha, acc ? 1 : 0);
  else
    k_gather4<long><<<blocks, 256, 0, r.st>>>(src, dst, n0, n1, n2, n3, s0, s1, s2, s3, alpha,
                                               acc ? 1 : 0);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

// dst (cols x rows) = src (rows x cols)^T
int transpose(Run& r, const double* src, double* dst, long rows, long cols) {
  return gather(r, src, dst, 1, 1, (int)cols, (int)rows, 0, 0, 1, cols);
}

int fill(Run& r, double* x, long n, double v) {
  if (n <= 0) return 0;
  if (!r.inside(x, (size_t)n * 8)) return r.fail("adjoint fill out of its buffer; launch refused");
  k_fill<<<(int)std::min<long>(2048, (n + 255) / 256), 256, 0, r.st>>>(x, n, v);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int copy(Run& r, const double* src, double* dst, long n) {
  if (!r.inside(src, (size_t)n * 8) || !r.inside(dst, (size_t)n * 8))
    return r.fail("adjoint copy out of its buffer; refused");
  CTM_HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n * 8, hipMemcpyDeviceToDevice, r.st));
  return 0;
}

#define VTRY(expr)              \
  do {                          \
    const int _r = (expr);      \
    if (_r) return _r;          \
  } while (0)

inline int md(int i) { return ((i % 4) + 4) % 4; }

// Corner index and orientation of application t of half h for side j
// (sides 0..3: X of bond j; 4..7: Y^T of bond j-4).  X: M then M^T;
// Y^T: M^T then M.  M X applies Ct[b+2], Ct[b+1], Ct[b], Ct[b-1] in turn.
void app(int j, int h, int t, int* ci, int* trans) {
  const int b = j & 3;
  const bool x_side = j < 4;
  const bool with_M = (h == 0) == x_side;
  const int mseq[4] = {md(b + 2), md(b + 1), md(b), md(b - 1)};
  const int tseq[4] = {md(b - 1), md(b), md(b + 1), md(b + 2)};
  *ci = with_M ? mseq[t] : tseq[t];
  *trans = with_M ? 0 : 1;
}

// ---------------------------------------------------------------------------
// forward with the tape
// ---------------------------------------------------------------------------
struct State {
  const double* C[4];
  const double* T[4];
  const double* X[4];
  const double* Yt[4];
};

int forward(Run& r, const VjpView& v, const Dims& m, Bufs& b, const State& in, double rtol) {
  const int x = m.x, Dl = m.Dl, N = m.N, k = m.k;
  // enlarged corners: CT = C T, W = T_(i-1) (C T), Ct = W ap_i
  {
    GemmBatch g = rowmajor(4, x, Dl * x, x, x, (long)Dl * x, (long)Dl * x);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = in.C[i];
      g.B[i] = in.T[i];
      g.C[i] = b.CT[i];
    }
    VTRY(gemm(r, g));
  }
  {
    GemmBatch g = rowmajor(4, x * Dl, Dl * x, x, x, (long)Dl * x, 0);
    g.cdiv_m = Dl;
    g.cs_m1 = (long)x * Dl * Dl;
    g.cs_m0 = Dl;
    g.cdiv_n = x;
    g.cs_n1 = 1;
    g.cs_n0 = (long)Dl * Dl;
    for (int i = 0; i < 4; ++i) {
      g.A[i] = in.T[md(i - 1)];
      g.B[i] = b.CT[i];
      g.C[i] = b.Wc[i];
    }
    VTRY(gemm(r, g));
  }
  {
    GemmBatch g = rowmajor(4, x * x, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
    g.cdiv_m = x;
    g.cs_m1 = (long)Dl * N;
    g.cs_m0 = Dl;
    g.cdiv_n = Dl;
    g.cs_n1 = N;
    g.cs_n0 = 1;
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Wc[i];
      g.B[i] = v.ap[i];
      g.C[i] = b.Ct[i];
    }
    VTRY(gemm(r, g));
  }
  // subspace steps of all 8 sides, every product and every Q on the tape
  const double* cur[8];
  for (int j = 0; j < 8; ++j) cur[j] = j < 4 ? in.X[j] : in.Yt[j - 4];
  for (int s = 0; s < m.nsi; ++s) {
    for (int h = 0; h < 2; ++h) {
      const int base = (s * 2 + h) * 5;
      for (int t = 0; t < 4; ++t) {
        GemmBatch g = rowmajor(8, N, k, N, N, k, k);
        for (int j = 0; j < 8; ++j) {
          int ci, tr;
          app(j, h, t, &ci, &tr);
          g.A[j] = b.Ct[ci];
          g.transA[j] = tr;
          g.B[j] = t == 0 ? cur[j] : b.tape[j][base + t - 1];
          g.C[j] = b.tape[j][base + t];
        }
        VTRY(gemm(r, g, true));
      }
      double* q[8];
      for (int j = 0; j < 8; ++j) {
        VTRY(copy(r, b.tape[j][base + 3], b.tape[j][base + 4], (long)N * k));
        q[j] = b.tape[j][base + 4];
      }
      const int rc = launch_qr(8, q, N, k, b.qr_ws, r.st);
      if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
      for (int j = 0; j < 8; ++j) cur[j] = q[j];
    }
  }
  // A = Ct[b+1] (Ct[b+2] X),  B^T = Ct[b]^T (Ct[b-1]^T Y^T)
  {
    GemmBatch g = rowmajor(8, N, k, N, N, k, k);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Ct[md(i + 2)];
      g.B[i] = cur[i];
      g.C[i] = b.W1[i];
      g.A[4 + i] = b.Ct[md(i - 1)];
      g.transA[4 + i] = 1;
      g.B[4 + i] = cur[4 + i];
      g.C[4 + i] = b.W2[i];
    }
    VTRY(gemm(r, g, true));
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Ct[md(i + 1)];
      g.B[i] = b.W1[i];
      g.C[i] = b.Ab[i];
      g.A[4 + i] = b.Ct[i];
      g.B[4 + i] = b.W2[i];
      g.C[4 + i] = b.Bt[i];
    }
    VTRY(gemm(r, g, true));
  }
  {
    GemmBatch g = rowmajor(4, k, k, N, k, k, k);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Bt[i];
      g.transA[i] = 1;
      g.B[i] = b.Ab[i];
      g.C[i] = b.rho[i];
    }
    VTRY(gemm(r, g));
  }
  {
    const double* rho[4] = {b.rho[0], b.rho[1], b.rho[2], b.rho[3]};
    const int rc = launch_svd(4, rho, b.u, b.s, b.v, k, b.svd_ws, r.st);
    if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
  }
  // signs from Y^T u (the sign rule), then the signed factors and s^-1/2
  {
    GemmBatch g = rowmajor(4, N, k, k, k, k, k);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = cur[4 + i];
      g.B[i] = b.u[i];
      g.C[i] = b.Hb[i];
    }
    VTRY(gemm(r, g));
    SignArgs sa{};
    sa.N = N;
    sa.k = k;
    sa.ld = k;
    for (int i = 0; i < 4; ++i) {
      sa.Y[i] = b.Hb[i];
      sa.sg[i] = b.sg[i];
    }
    const int rc = elem_col_sign(sa, 4, r.st);
    if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
    PrepArgs pa{};
    for (int i = 0; i < 4; ++i) {
      pa.u[i] = b.u[i];
      pa.v[i] = b.v[i];
      pa.s[i] = b.s[i];
      pa.sg[i] = b.sg[i];
      pa.us[i] = b.us[i];
      pa.vs[i] = b.vs[i];
      pa.sinv[i] = b.sinv[i];
      pa.vsc[i] = b.vsc[i];
      pa.usc[i] = b.usc[i];
    }
    pa.k = k;
    pa.keep = x;
    pa.rtol = rtol;
    k_prep<<<dim3((k * k + 255) / 256, 4), 256, 0, r.st>>>(pa);
    CTM_HIP_TRY(hipGetLastError());
  }
  // P_l = A v_s sinv, P_r^T = B^T u_s sinv
  {
    GemmBatch g = rowmajor(8, N, x, k, k, x, x);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Ab[i];
      g.B[i] = b.vsc[i];
      g.C[i] = b.Pl[i];
      g.A[4 + i] = b.Bt[i];
      g.B[4 + i] = b.usc[i];
      g.C[4 + i] = b.Prt[i];
    }
    VTRY(gemm(r, g));
  }
  // renormalisation (unscaled), then the unit-norm outputs
  {
    GemmBatch g = rowmajor(4, N, x, N, N, x, x);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Ct[i];
      g.B[i] = b.Pl[i];
      g.C[i] = b.Zc[i];
    }
    VTRY(gemm(r, g));
    GemmBatch g2 = rowmajor(4, x, x, N, x, x, x);
    for (int i = 0; i < 4; ++i) {
      g2.A[i] = b.Prt[md(i - 1)];
      g2.transA[i] = 1;
      g2.B[i] = b.Zc[i];
      g2.C[i] = b.Ch[i];
    }
    VTRY(gemm(r, g2));
  }
  {
    // Z1[(b,g'),(u,r)] = sum_g T_j[(b,u),g] P_l[(g,r),g']   (batched over r)
    GemmBatch g = rowmajor(4, x * Dl, x, x, x, (long)Dl * x, 0);
    g.cdiv_m = Dl;
    g.cs_m1 = (long)x * Dl * Dl;
    g.cs_m0 = Dl;
    g.cdiv_n = 1 << 30;
    g.cs_n1 = 0;
    g.cs_n0 = (long)Dl * Dl;
    g.nbatch = Dl;
    g.a_bs = 0;
    g.b_bs = x;
    g.c_bs = 1;
    for (int j = 0; j < 4; ++j) {
      g.A[j] = in.T[j];
      g.B[j] = b.Pl[j];
      g.C[j] = b.Z1[j];
    }
    VTRY(gemm(r, g));
    // Z2[(b,l),(d,g')] = Z1[(b,g'),(u,r)] ap_(j+1)[(u,r),(l,d)]
    GemmBatch g2 = rowmajor(4, x * x, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
    g2.cdiv_m = x;
    g2.cs_m1 = (long)Dl * Dl * x;
    g2.cs_m0 = 1;
    g2.cdiv_n = Dl;
    g2.cs_n1 = (long)Dl * x;
    g2.cs_n0 = x;
    for (int j = 0; j < 4; ++j) {
      g2.A[j] = b.Z1[j];
      g2.B[j] = v.ap[md(j + 1)];
      g2.C[j] = b.Z2[j];
    }
    VTRY(gemm(r, g2));
    // T'[b',(d,g')] = sum_(b,l) P_r^T[(b,l),b'] Z2[(b,l),(d,g')]
    GemmBatch g3 = rowmajor(4, x, Dl * x, x * Dl, x, (long)Dl * x, (long)Dl * x);
    for (int j = 0; j < 4; ++j) {
      g3.A[j] = b.Prt[j];
      g3.transA[j] = 1;
      g3.B[j] = b.Z2[j];
      g3.C[j] = b.Th[j];
    }
    VTRY(gemm(r, g3));
  }
  {
    NormArgs na{};
    for (int i = 0; i < 4; ++i) {
      na.x[i] = b.Ch[i];
      na.n[i] = (long)x * x;
      na.x[4 + i] = b.Th[i];
      na.n[4 + i] = (long)x * Dl * x;
    }
    na.out = b.nrm;
    na.bad = nullptr;
    DotArgs da{};
    for (int t = 0; t < 8; ++t) {
      da.x[t] = na.x[t];
      da.y[t] = na.x[t];
      da.n[t] = na.n[t];
    }
    da.out = b.dots;   // squared norms; the square roots are taken below
    VTRY(launch_dots(da, 8, b.dpart, r.st));
  }
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// kernels that need the forward norms: sqrt of the squared norms, then scale
// ---------------------------------------------------------------------------
namespace {

__global__ void k_sqrt8(const double* sq, double* nrm) {
  if (threadIdx.x < 8) nrm[threadIdx.x] = sqrt(sq[threadIdx.x]);
}

struct ScaleArgs {
  const double* x[8];
  double* y[8];
  long n[8];
  const double* nrm;
};

__global__ __launch_bounds__(256) void k_scale_out(ScaleArgs a) {
  const int t = blockIdx.y;
  const double inv = 1.0 / a.nrm[t];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n[t]; i += (long)gridDim.x * 256)
    a.y[t][i] = a.x[t][i] * inv;
}

// inverse strides of a corner permutation: ab[u,l,d,r] gathers from apb
void inverse_strides(const long s[4], long Dl, long out[4]) {
  const long pw[4] = {Dl * Dl * Dl, Dl * Dl, Dl, 1};
  for (int p = 0; p < 4; ++p)
    for (int j = 0; j < 4; ++j)
      if (s[j] == pw[p]) out[p] = pw[j];
}

int backward(Run& r, const VjpView& v, const Dims& m, Bufs& b, const State& in,
             const State& bar, double* const* Cb_out, double* const* Tb_out,
             double* const* Xb_out, double* const* Yb_out, double* site_bar) {
  const int x = m.x, Dl = m.Dl, N = m.N, k = m.k;
  const long NN = (long)N * N, Nk = (long)N * k;
  for (int i = 0; i < 4; ++i) {
    VTRY(fill(r, b.Ctb[i], NN, 0.0));
    VTRY(fill(r, b.Plb[i], (long)N * x, 0.0));
    VTRY(fill(r, b.Prtb[i], (long)N * x, 0.0));
    VTRY(fill(r, Tb_out[i], (long)x * Dl * x, 0.0));
  }
  VTRY(fill(r, b.ab, (long)Dl * Dl * Dl * Dl, 0.0));
  for (int i = 0; i < 4; ++i) VTRY(transpose(r, v.ap[i], b.apT[i], (long)Dl * Dl, (long)Dl * Dl));
  // unit-norm scaling
  {
    DotArgs da{};
    NormBwdArgs nb{};
    for (int i = 0; i < 4; ++i) {
      da.x[i] = b.Cn[i];
      da.y[i] = bar.C[i];
      da.n[i] = (long)x * x;
      da.x[4 + i] = b.Tn[i];
      da.y[4 + i] = bar.T[i];
      da.n[4 + i] = (long)x * Dl * x;
    }
    da.out = b.dots;
    VTRY(launch_dots(da, 8, b.dpart, r.st));
    for (int t = 0; t < 8; ++t) {
      nb.y[t] = da.x[t];
      nb.yb[t] = da.y[t];
      nb.n[t] = da.n[t];
      nb.xb[t] = t < 4 ? b.Chb[t] : b.Thb[t - 4];
    }
    nb.dot = b.dots;
    nb.nrm = b.nrm;
    const long mx = (long)x * Dl * x;
    k_norm_bwd<<<dim3((int)std::min<long>(512, (mx + 255) / 256), 8), 256, 0, r.st>>>(nb);
    CTM_HIP_TRY(hipGetLastError());
  }
  // C_i' = P_r^(i-1)T Zc_i, Zc_i = Ct_i P_l^(i)
  for (int i = 0; i < 4; ++i) {
    const int ip = md(i - 1);
    VTRY(transpose(r, b.Chb[i], b.smallT, x, x));
    GemmBatch g = rowmajor(1, N, x, x, x, x, x);
    g.A[0] = b.Zc[i];
    g.B[0] = b.smallT;
    g.C[0] = b.Prtb[ip];
    g.accumulate = 1;
    VTRY(gemm(r, g));
    GemmBatch g2 = rowmajor(1, N, x, x, x, x, x);
    g2.A[0] = b.Prt[ip];
    g2.B[0] = b.Chb[i];
    g2.C[0] = b.Zcb;
    VTRY(gemm(r, g2));
    VTRY(transpose(r, b.Pl[i], b.St, N, x));
    GemmBatch g3 = rowmajor(1, N, N, x, x, N, N);
    g3.A[0] = b.Zcb;
    g3.B[0] = b.St;
    g3.C[0] = b.Ctb[i];
    g3.accumulate = 1;
    VTRY(gemm(r, g3));
    GemmBatch g4 = rowmajor(1, N, x, N, N, x, x);
    g4.A[0] = b.Ct[i];
    g4.transA[0] = 1;
    g4.B[0] = b.Zcb;
    g4.C[0] = b.Plb[i];
    g4.accumulate = 1;
    VTRY(gemm(r, g4));
  }
  // T_j' = P_r^T Z2,  Z2 = perm(Z1 ap_(j+1)),  Z1 = T_j P_l; the four edges
  // go through each step in one launch
  {
    const long D2 = (long)Dl * Dl;
    for (int j = 0; j < 4; ++j) VTRY(transpose(r, b.Thb[j], b.Gb[j], x, (long)Dl * x));
    GemmBatch g = rowmajor(4, N, x, Dl * x, (long)Dl * x, x, x);
    g.accumulate = 1;
    for (int j = 0; j < 4; ++j) {
      g.A[j] = b.Z2[j];
      g.B[j] = b.Gb[j];
      g.C[j] = b.Prtb[j];
    }
    VTRY(gemm(r, g));
    GemmBatch g2 = rowmajor(4, N, Dl * x, x, x, (long)Dl * x, (long)Dl * x);
    for (int j = 0; j < 4; ++j) {
      g2.A[j] = b.Prt[j];
      g2.B[j] = b.Thb[j];
      g2.C[j] = b.Ga[j];                                   // Z2_bar [(b,l)][(d,g')]
    }
    VTRY(gemm(r, g2));
    for (int j = 0; j < 4; ++j)                            // -> [(b,g')][(l,d)]
      VTRY(gather(r, b.Ga[j], b.Gb[j], x, x, Dl, Dl, D2 * x, 1, (long)Dl * x, x));
    GemmBatch g3 = rowmajor(4, (int)D2, (int)D2, x * x, D2, D2, D2);
    for (int j = 0; j < 4; ++j) {
      g3.A[j] = b.Z1[j];
      g3.transA[j] = 1;
      g3.B[j] = b.Gb[j];
      g3.C[j] = b.apb4[j];
    }
    VTRY(gemm(r, g3));
    for (int j = 0; j < 4; ++j) {
      long inv[4];
      inverse_strides(v.ap_strides[md(j + 1)], Dl, inv);
      VTRY(gather(r, b.apb4[j], b.ab, Dl, Dl, Dl, Dl, inv[0], inv[1], inv[2], inv[3], true));
    }
    GemmBatch g4 = rowmajor(4, x * x, (int)D2, (int)D2, D2, D2, D2);
    for (int j = 0; j < 4; ++j) {
      g4.A[j] = b.Gb[j];
      g4.B[j] = b.apT[md(j + 1)];
      g4.C[j] = b.Ga[j];                                   // Z1_bar [(b,g')][(u,r)]
    }
    VTRY(gemm(r, g4));
    for (int j = 0; j < 4; ++j) {                          // -> [(b,u)][(r,g')]
      VTRY(gather(r, b.Ga[j], b.Gb[j], x, Dl, Dl, x, (long)x * D2, Dl, 1, D2));
      VTRY(transpose(r, b.Pl[j], b.Ga[j], x, (long)Dl * x));
    }
    GemmBatch g5 = rowmajor(4, x * Dl, x, Dl * x, (long)Dl * x, x, x);
    g5.accumulate = 1;
    for (int j = 0; j < 4; ++j) {
      g5.A[j] = b.Gb[j];
      g5.B[j] = b.Ga[j];
      g5.C[j] = Tb_out[j];
    }
    VTRY(gemm(r, g5));
    GemmBatch g6 = rowmajor(4, x, Dl * x, x * Dl, x, (long)Dl * x, (long)Dl * x);
    g6.accumulate = 1;
    for (int j = 0; j < 4; ++j) {
      g6.A[j] = in.T[j];
      g6.transA[j] = 1;
      g6.B[j] = b.Gb[j];
      g6.C[j] = b.Plb[j];
    }
    VTRY(gemm(r, g6));
  }
  // projectors, recycled blocks, rho and its SVD, per bond (batched over 4)
  double* Xf[4];
  double* Yf[4];
  for (int i = 0; i < 4; ++i) {
    Xf[i] = m.nsi > 0 ? b.tape[i][10 * m.nsi - 1] : (double*)in.X[i];
    Yf[i] = m.nsi > 0 ? b.tape[4 + i][10 * m.nsi - 1] : (double*)in.Yt[i];
  }
  for (int i = 0; i < 4; ++i) {
    VTRY(transpose(r, b.vsc[i], b.vscT[i], k, x));
    VTRY(transpose(r, b.usc[i], b.uscT[i], k, x));
    VTRY(transpose(r, b.vs[i], b.vsT[i], k, k));
    VTRY(transpose(r, b.us[i], b.usT[i], k, k));
  }
  {
    // A_bar = P_l_bar vsc^T -> Hb[i];  B^T_bar = P_rT_bar usc^T -> Hb[4+i]
    GemmBatch g = rowmajor(8, N, k, x, x, k, k);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Plb[i];
      g.B[i] = b.vscT[i];
      g.C[i] = b.Hb[i];
      g.A[4 + i] = b.Prtb[i];
      g.B[4 + i] = b.uscT[i];
      g.C[4 + i] = b.Hb[4 + i];
    }
    VTRY(gemm(r, g));
    GemmBatch g2 = rowmajor(8, k, x, N, k, x, x);
    for (int i = 0; i < 4; ++i) {
      g2.A[i] = b.Ab[i];
      g2.transA[i] = 1;
      g2.B[i] = b.Plb[i];
      g2.C[i] = b.vscb[i];
      g2.A[4 + i] = b.Bt[i];
      g2.transA[4 + i] = 1;
      g2.B[4 + i] = b.Prtb[i];
      g2.C[4 + i] = b.uscb[i];
    }
    VTRY(gemm(r, g2));
    // recycled blocks X' = Xf v_s, Y^T' = Yf u_s
    GemmBatch g3 = rowmajor(8, N, k, k, k, k, k);
    for (int i = 0; i < 4; ++i) {
      g3.A[i] = bar.X[i];
      g3.B[i] = b.vsT[i];
      g3.C[i] = b.Qb[i];
      g3.A[4 + i] = bar.Yt[i];
      g3.B[4 + i] = b.usT[i];
      g3.C[4 + i] = b.Qb[4 + i];
    }
    VTRY(gemm(r, g3));
    GemmBatch g4 = rowmajor(8, k, k, N, k, k, k);
    for (int i = 0; i < 4; ++i) {
      g4.A[i] = Xf[i];
      g4.transA[i] = 1;
      g4.B[i] = bar.X[i];
      g4.C[i] = b.vb[i];
      g4.A[4 + i] = Yf[i];
      g4.transA[4 + i] = 1;
      g4.B[4 + i] = bar.Yt[i];
      g4.C[4 + i] = b.ub[i];
    }
    VTRY(gemm(r, g4));
  }
  {
    ProjBwdArgs pb{};
    KmatArgs ka{};
    for (int i = 0; i < 4; ++i) {
      pb.us[i] = b.us[i];
      pb.vs[i] = b.vs[i];
      pb.sinv[i] = b.sinv[i];
      pb.vscb[i] = b.vscb[i];
      pb.uscb[i] = b.uscb[i];
      pb.ub[i] = b.ub[i];
      pb.vb[i] = b.vb[i];
      pb.sb[i] = b.sb[i];
    }
    pb.k = k;
    pb.keep = x;
    k_proj_bwd<<<4, 256, 0, r.st>>>(pb);
    CTM_HIP_TRY(hipGetLastError());
    GemmBatch g = rowmajor(8, k, k, k, k, k, k);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.us[i];
      g.transA[i] = 1;
      g.B[i] = b.ub[i];
      g.C[i] = b.Ju[i];
      g.A[4 + i] = b.vs[i];
      g.transA[4 + i] = 1;
      g.B[4 + i] = b.vb[i];
      g.C[4 + i] = b.Jv[i];
    }
    VTRY(gemm(r, g));
    for (int i = 0; i < 4; ++i) {
      ka.Ju[i] = b.Ju[i];
      ka.Jv[i] = b.Jv[i];
      ka.s[i] = b.s[i];
      ka.sb[i] = b.sb[i];
      ka.K[i] = b.Km[i];
    }
    ka.n = k;
    k_svd_kmat<<<dim3((k * k + 255) / 256, 4), 256, 0, r.st>>>(ka);
    CTM_HIP_TRY(hipGetLastError());
    GemmBatch g2 = rowmajor(4, k, k, k, k, k, k);
    for (int i = 0; i < 4; ++i) {
      g2.A[i] = b.us[i];
      g2.B[i] = b.Km[i];
      g2.C[i] = b.uK[i];
    }
    VTRY(gemm(r, g2));
    for (int i = 0; i < 4; ++i) {
      g2.A[i] = b.uK[i];
      g2.B[i] = b.vsT[i];
      g2.C[i] = b.rhob[i];
    }
    VTRY(gemm(r, g2));
    for (int i = 0; i < 4; ++i) VTRY(transpose(r, b.rhob[i], b.rhobT[i], k, k));
    // rho = B A:  A_bar += B^T rho_bar,  B^T_bar += A rho_bar^T
    GemmBatch g3 = rowmajor(8, N, k, k, k, k, k);
    g3.accumulate = 1;
    for (int i = 0; i < 4; ++i) {
      g3.A[i] = b.Bt[i];
      g3.B[i] = b.rhob[i];
      g3.C[i] = b.Hb[i];
      g3.A[4 + i] = b.Ab[i];
      g3.B[4 + i] = b.rhobT[i];
      g3.C[4 + i] = b.Hb[4 + i];
    }
    VTRY(gemm(r, g3));
  }
  // A = Ct[b+1] W1, W1 = Ct[b+2] Xf;  B^T = Ct[b]^T W2, W2 = Ct[b-1]^T Yf
  {
    // rank-k terms of the outer applications (A and B^T)
    for (int i = 0; i < 4; ++i) VTRY(transpose(r, b.W1[i], b.tr[i], N, k));
    for (int i = 0; i < 4; ++i) VTRY(transpose(r, b.Hb[4 + i], b.tr[4 + i], N, k));
    GemmBatch g = rowmajor(4, N, N, k, k, N, N);
    g.accumulate = 1;
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Hb[i];
      g.B[i] = b.tr[i];
      g.C[i] = b.Ctb[md(i + 1)];
    }
    VTRY(gemm(r, g));
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.W2[i];
      g.B[i] = b.tr[4 + i];
      g.C[i] = b.Ctb[i];
    }
    VTRY(gemm(r, g));
    // W1_bar = Ct[b+1]^T A_bar,  W2_bar = Ct[b] B^T_bar
    GemmBatch g2 = rowmajor(8, N, k, N, N, k, k);
    for (int i = 0; i < 4; ++i) {
      g2.A[i] = b.Ct[md(i + 1)];
      g2.transA[i] = 1;
      g2.B[i] = b.Hb[i];
      g2.C[i] = b.Yq[i];
      g2.A[4 + i] = b.Ct[i];
      g2.B[4 + i] = b.Hb[4 + i];
      g2.C[4 + i] = b.Yq[4 + i];
    }
    VTRY(gemm(r, g2, true));
    for (int i = 0; i < 4; ++i) VTRY(transpose(r, Xf[i], b.tr[i], N, k));
    for (int i = 0; i < 4; ++i) VTRY(transpose(r, b.Yq[4 + i], b.tr[4 + i], N, k));
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Yq[i];
      g.B[i] = b.tr[i];
      g.C[i] = b.Ctb[md(i + 2)];
    }
    VTRY(gemm(r, g));
    for (int i = 0; i < 4; ++i) {
      g.A[i] = Yf[i];
      g.B[i] = b.tr[4 + i];
      g.C[i] = b.Ctb[md(i - 1)];
    }
    VTRY(gemm(r, g));
    // Xf_bar += Ct[b+2]^T W1_bar,  Yf_bar += Ct[b-1] W2_bar
    GemmBatch g3 = rowmajor(8, N, k, N, N, k, k);
    g3.accumulate = 1;
    for (int i = 0; i < 4; ++i) {
      g3.A[i] = b.Ct[md(i + 2)];
      g3.transA[i] = 1;
      g3.B[i] = b.Yq[i];
      g3.C[i] = b.Qb[i];
      g3.A[4 + i] = b.Ct[md(i - 1)];
      g3.B[4 + i] = b.Yq[4 + i];
      g3.C[4 + i] = b.Qb[4 + i];
    }
    VTRY(gemm(r, g3, true));
  }
  // subspace steps in reverse: QR adjoint, then the four applications
  for (int s = m.nsi - 1; s >= 0; --s) {
    for (int h = 1; h >= 0; --h) {
      const int base = (s * 2 + h) * 5;
      // R = Q^T H, M = -Q_bar^T Q, Y = Q_bar + Q copyltu(M), H_bar = Y R^-T
      GemmBatch g = rowmajor(8, k, k, N, k, k, k);
      for (int j = 0; j < 8; ++j) {
        g.A[j] = b.tape[j][base + 4];
        g.transA[j] = 1;
        g.B[j] = b.tape[j][base + 3];
        g.C[j] = b.R[j];
      }
      VTRY(gemm(r, g));
      GemmBatch gm = rowmajor(8, k, k, N, k, k, k);
      gm.alpha = -1.0;
      for (int j = 0; j < 8; ++j) {
        gm.A[j] = b.Qb[j];
        gm.transA[j] = 1;
        gm.B[j] = b.tape[j][base + 4];
        gm.C[j] = b.Mm[j];
      }
      VTRY(gemm(r, gm));
      SmallArgs sa{};
      for (int j = 0; j < 8; ++j) {
        sa.in[j] = b.Mm[j];
        sa.out[j] = b.Mc[j];
      }
      sa.n = k;
      k_copyltu<<<dim3((k * k + 255) / 256, 8), 256, 0, r.st>>>(sa);
      CTM_HIP_TRY(hipGetLastError());
      for (int j = 0; j < 8; ++j) {
        sa.in[j] = b.R[j];
        sa.out[j] = b.Rinv[j];
      }
      if (k <= kTriLds)
        k_tri_inv_lds<<<8, 256, 0, r.st>>>(sa);
      else
        k_tri_inv<<<8, 256, 0, r.st>>>(sa);
      CTM_HIP_TRY(hipGetLastError());
      for (int j = 0; j < 8; ++j) {
        VTRY(transpose(r, b.Rinv[j], b.RinvT[j], k, k));
        VTRY(copy(r, b.Qb[j], b.Yq[j], Nk));
      }
      GemmBatch gy = rowmajor(8, N, k, k, k, k, k);
      gy.accumulate = 1;
      for (int j = 0; j < 8; ++j) {
        gy.A[j] = b.tape[j][base + 4];
        gy.B[j] = b.Mc[j];
        gy.C[j] = b.Yq[j];
      }
      VTRY(gemm(r, gy));
      for (int j = 0; j < 8; ++j) {
        gy.A[j] = b.Yq[j];
        gy.B[j] = b.RinvT[j];
        gy.C[j] = b.Hb[j];
      }
      gy.accumulate = 0;
      VTRY(gemm(r, gy));
      // applications t = 3 .. 0
      for (int t = 3; t >= 0; --t) {
        const double* hin[8];
        int ci[8], trn[8];
        for (int j = 0; j < 8; ++j) {
          app(j, h, t, &ci[j], &trn[j]);
          if (t > 0) {
            hin[j] = b.tape[j][base + t - 1];
          } else if (h == 1) {
            hin[j] = b.tape[j][base - 1];            // Q of the first half
          } else if (s > 0) {
            hin[j] = b.tape[j][base - 1];            // Q of the previous step
          } else {
            hin[j] = j < 4 ? in.X[j] : in.Yt[j - 4];
          }
        }
        // corner cotangents: plain H_out = Ct H_in gives Ct_bar += H_bar H_in^T;
        // transposed H_out = Ct^T H_in gives Ct_bar += H_in H_bar^T.  Both
        // factors go transposed into the corner's K-stacks (slot 2t for the X
        // side, 2t+1 for the Y side: each corner meets one of each per t);
        // the stacks are contracted once per half step below.
        for (int j = 0; j < 8; ++j) {
          const long slot = (2 * t + (j >= 4 ? 1 : 0)) * Nk;
          VTRY(transpose(r, trn[j] ? hin[j] : b.Hb[j], b.PTs[ci[j]] + slot, N, k));
          VTRY(transpose(r, trn[j] ? b.Hb[j] : hin[j], b.QTs[ci[j]] + slot, N, k));
        }
        GemmBatch gb = rowmajor(8, N, k, N, N, k, k);
        for (int j = 0; j < 8; ++j) {
          gb.A[j] = b.Ct[ci[j]];
          gb.transA[j] = trn[j] ? 0 : 1;
          gb.B[j] = b.Hb[j];
          gb.C[j] = b.Yq[j];
        }
        VTRY(gemm(r, gb, true));
        for (int j = 0; j < 8; ++j) std::swap(b.Hb[j], b.Yq[j]);
      }
      // Ct_bar[i] += sum over the 8 stacked pairs P Q^T = PTs^T QTs  (K = 8k)
      {
        GemmBatch gc = rowmajor(4, N, N, 8 * k, N, N, N);
        gc.accumulate = 1;
        for (int i = 0; i < 4; ++i) {
          gc.A[i] = b.PTs[i];
          gc.transA[i] = 1;
          gc.B[i] = b.QTs[i];
          gc.C[i] = b.Ctb[i];
        }
        VTRY(gemm(r, gc));
      }
      for (int j = 0; j < 8; ++j) std::swap(b.Qb[j], b.Hb[j]);
    }
  }
  for (int i = 0; i < 4; ++i) {
    VTRY(copy(r, b.Qb[i], Xb_out[i], Nk));
    VTRY(copy(r, b.Qb[4 + i], Yb_out[i], Nk));
  }
  // enlarged corners, the four corners batched in every step
  {
    const long D2 = (long)Dl * Dl;
    for (int i = 0; i < 4; ++i)   // Gp[(x_in,y),(o1,o2)] from Ct_bar[(x_in,o1),(y,o2)]
      VTRY(gather(r, b.Ctb[i], b.Ga[i], x, x, Dl, Dl, (long)Dl * N, Dl, N, 1));
    GemmBatch g = rowmajor(4, x * x, (int)D2, (int)D2, D2, D2, D2);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = b.Ga[i];
      g.B[i] = b.apT[i];
      g.C[i] = b.Gb[i];                                    // W_bar [(x_in,y)][(p,q)]
    }
    VTRY(gemm(r, g));
    GemmBatch g2 = rowmajor(4, (int)D2, (int)D2, x * x, D2, D2, D2);
    for (int i = 0; i < 4; ++i) {
      g2.A[i] = b.Wc[i];
      g2.transA[i] = 1;
      g2.B[i] = b.Ga[i];
      g2.C[i] = b.apb4[i];
    }
    VTRY(gemm(r, g2));
    for (int i = 0; i < 4; ++i) {
      long inv[4];
      inverse_strides(v.ap_strides[i], Dl, inv);
      VTRY(gather(r, b.apb4[i], b.ab, Dl, Dl, Dl, Dl, inv[0], inv[1], inv[2], inv[3], true));
      // Wbp[(x_in,p),(q,y)] from W_bar[(x_in,y),(p,q)]
      VTRY(gather(r, b.Gb[i], b.Ga[i], x, Dl, Dl, x, (long)x * D2, Dl, 1, D2));
      VTRY(transpose(r, b.CT[i], b.Gb[i], x, (long)Dl * x));
    }
    GemmBatch g3 = rowmajor(4, x * Dl, x, Dl * x, (long)Dl * x, x, x);
    g3.accumulate = 1;
    for (int i = 0; i < 4; ++i) {
      g3.A[i] = b.Ga[i];
      g3.B[i] = b.Gb[i];
      g3.C[i] = Tb_out[md(i - 1)];
    }
    VTRY(gemm(r, g3));
    GemmBatch g4 = rowmajor(4, x, Dl * x, x * Dl, x, (long)Dl * x, (long)Dl * x);
    for (int i = 0; i < 4; ++i) {
      g4.A[i] = in.T[md(i - 1)];
      g4.transA[i] = 1;
      g4.B[i] = b.Ga[i];
      g4.C[i] = b.Gb[i];                                   // CT_bar [a][(q,y)]
    }
    VTRY(gemm(r, g4));
    for (int i = 0; i < 4; ++i) VTRY(transpose(r, in.T[i], b.Ga[i], x, (long)Dl * x));
    GemmBatch g5 = rowmajor(4, x, x, Dl * x, (long)Dl * x, x, x);
    for (int i = 0; i < 4; ++i) {
      g5.A[i] = b.Gb[i];
      g5.B[i] = b.Ga[i];
      g5.C[i] = Cb_out[i];
    }
    VTRY(gemm(r, g5));
    GemmBatch g6 = rowmajor(4, x, Dl * x, x, x, (long)Dl * x, (long)Dl * x);
    g6.accumulate = 1;
    for (int i = 0; i < 4; ++i) {
      g6.A[i] = in.C[i];
      g6.transA[i] = 1;
      g6.B[i] = b.Gb[i];
      g6.C[i] = Tb_out[i];
    }
    VTRY(gemm(r, g6));
  }
  // double layer: A_bar[s, ket] += sum_bra (ab[ket,bra] + ab[bra,ket]) A[s, bra]
  if (site_bar) {
    const long D4 = (long)m.D * m.D * m.D * m.D;
    if (!r.inside(b.msym, (size_t)D4 * D4 * 8)) return r.fail("adjoint buffer too small");
    k_dl_sym<<<(int)std::min<long>(4096, (D4 * D4 + 255) / 256), 256, 0, r.st>>>(b.ab, b.msym, m.D);
    CTM_HIP_TRY(hipGetLastError());
    GemmBatch g = rowmajor(1, m.d, (int)D4, (int)D4, D4, D4, D4);
    g.A[0] = v.A_site;
    g.B[0] = b.msym;
    g.C[0] = site_bar;
    g.accumulate = 1;
    VTRY(gemm(r, g));
  }
  return 0;
}

Dims dims_of(const ctm_config& cfg) {
  Dims m{};
  m.d = cfg.d;
  m.D = cfg.D;
  m.Dl = cfg.d > 0 ? cfg.D * cfg.D : cfg.D;
  m.x = cfg.chi;
  m.N = m.x * m.Dl;
  m.k = std::min(cfg.chi + cfg.p, m.N);
  m.nsi = cfg.n_si;
  return m;
}

int check_cfg(const ctm_config* cfg) {
  if (!cfg) return CTM_E_ARG;
  size_t ws = 0;
  const ctm_status st = ctm_workspace_bytes(cfg, &ws);
  if (st != CTM_OK) return st;
  if (cfg->d < 1 || cfg->proj != CTM_PROJ_SI || cfg->prec != CTM_PREC_F64 || cfg->stabilized != 1 ||
      cfg->sym != CTM_SYM_NONE)
    return CTM_E_ARG;
  return CTM_OK;
}

}  // namespace

namespace {

// Validation, carving, buffer registration and the taped forward move from
// state_in (with its unit-norm outputs in b.Cn, b.Tn).
struct Prepared {
  VjpView v;
  Dims m;
  Bufs b;
  Run r;
  State in;
  size_t nstate;
};

int prepare(ctm_ctx* ctx, const double* state_in, void* ws, size_t ws_bytes, Prepared& P,
            std::initializer_list<std::pair<const double*, size_t>> extra) {
  const int rv = vjp_view(ctx, &P.v);
  if (rv) return rv;
  if (check_cfg(&P.v.cfg))
    return vjp_fail(ctx, CTM_E_ARG,
                    "the adjoint needs an iPEPS site (d >= 1), SI projectors, float64 "
                    "contractions, the stabilised update and no lattice symmetry");
  P.m = dims_of(P.v.cfg);
  const size_t need = carve(P.m, &P.b, nullptr, nullptr);
  if (ws_bytes < need)
    return vjp_fail(ctx, CTM_E_ARG, "adjoint workspace too small (need " + std::to_string(need) +
                                        " bytes)");
  P.r.c = ctx;
  P.r.st = P.v.st;
  P.r.sk_part = P.v.sk_part;
  P.r.sk_cus = P.v.sk_cus;
  const size_t x = P.m.x, Dl = P.m.Dl, N = P.m.N, k = P.m.k;
  P.nstate = 4 * x * x + 4 * x * Dl * x + 8 * N * k + 4;
  double chi_env = 0.0;
  if (hipMemcpyAsync(&chi_env, state_in + (P.nstate - 4), sizeof(double), hipMemcpyDeviceToHost,
                     P.v.st) != hipSuccess ||
      hipStreamSynchronize(P.v.st) != hipSuccess)
    return vjp_fail(ctx, CTM_E_DEVICE, "reading chi_env of the input state failed");
  if ((int)chi_env != P.m.x)
    return vjp_fail(ctx, CTM_E_STATE,
                    "the adjoint is defined for SI moves: the input state needs chi_env == chi");
  carve(P.m, &P.b, (char*)ws, &P.r.reg);
  const size_t D4 = (size_t)P.m.D * P.m.D * P.m.D * P.m.D;
  auto reg = [&](const double* p, size_t n) {
    if (p) P.r.reg.push_back({(uintptr_t)p, (uintptr_t)(p + n)});
  };
  reg(state_in, P.nstate);
  for (const auto& e : extra) reg(e.first, e.second == 0 ? P.nstate : e.second);
  reg(P.v.A_site, P.m.d * D4);
  reg(P.v.a, Dl * Dl * Dl * Dl);
  for (int i = 0; i < 4; ++i) reg(P.v.ap[i], Dl * Dl * Dl * Dl);
  const double* p = state_in;
  for (int i = 0; i < 4; ++i, p += x * x) P.in.C[i] = p;
  for (int i = 0; i < 4; ++i, p += x * Dl * x) P.in.T[i] = p;
  for (int i = 0; i < 4; ++i, p += N * k) P.in.X[i] = p;
  for (int i = 0; i < 4; ++i, p += N * k) P.in.Yt[i] = p;
  int rc = forward(P.r, P.v, P.m, P.b, P.in, P.v.cfg.pinv_rtol);
  if (rc) return rc;
  k_sqrt8<<<1, 64, 0, P.r.st>>>(P.b.dots, P.b.nrm);
  ScaleArgs sa{};
  for (int i = 0; i < 4; ++i) {
    sa.x[i] = P.b.Ch[i];
    sa.y[i] = P.b.Cn[i];
    sa.n[i] = (long)x * x;
    sa.x[4 + i] = P.b.Th[i];
    sa.y[4 + i] = P.b.Tn[i];
    sa.n[4 + i] = (long)x * Dl * x;
  }
  sa.nrm = P.b.nrm;
  k_scale_out<<<dim3((int)std::min<size_t>(512, (x * Dl * x + 255) / 256), 8), 256, 0, P.r.st>>>(sa);
  if (hipGetLastError() != hipSuccess) return vjp_fail(ctx, CTM_E_DEVICE, "scaling launch failed");
  return 0;
}

// Splits a state-layout buffer into its tensors.
void split(double* base, const Dims& m, double** C, double** T, double** X, double** Y) {
  const size_t x = m.x, Dl = m.Dl, N = m.N, k = m.k;
  double* p = base;
  for (int i = 0; i < 4; ++i, p += x * x) C[i] = p;
  for (int i = 0; i < 4; ++i, p += x * Dl * x) T[i] = p;
  for (int i = 0; i < 4; ++i, p += N * k) X[i] = p;
  for (int i = 0; i < 4; ++i, p += N * k) Y[i] = p;
}

// One reverse pass of the prepared move: bar (state layout) -> in_bar.
int reverse(Prepared& P, const double* bar, double* in_bar, double* site_bar) {
  State sb{};
  double *C[4], *T[4], *X[4], *Y[4];
  split(const_cast<double*>(bar), P.m, C, T, X, Y);
  for (int i = 0; i < 4; ++i) {
    sb.C[i] = C[i];
    sb.T[i] = T[i];
    sb.X[i] = X[i];
    sb.Yt[i] = Y[i];
  }
  double *Cb[4], *Tb[4], *Xb[4], *Yb[4];
  split(in_bar, P.m, Cb, Tb, Xb, Yb);
  VTRY(fill(P.r, in_bar + (P.nstate - 4), 4, 0.0));
  return backward(P.r, P.v, P.m, P.b, P.in, sb, Cb, Tb, Xb, Yb, site_bar);
}

}  // namespace

// ---------------------------------------------------------------------------
// bond energy <op>_H + <op>_V and its gradient (iPEPS section, observables:
// two-site reduced density matrices).  The horizontal pair is contracted
// column by column; the vertical pair is the horizontal pair of the network
// turned by 90 degrees (corner and edge i+1 in slot i, site legs
// (u,l,d,r) <- (r,u,l,d)), so one chain and its reverse serve both.
// ---------------------------------------------------------------------------
namespace {

// [ket][bra] matrix of an open double-layer cotangent in the order
// [(uU),(lL),(dD),(rR)]: out[ket, bra] = xb[pairs(ket, bra)].
__global__ __launch_bounds__(256) void k_open_reorder(const double* __restrict__ xb,
                                                      double* __restrict__ out, int D) {
  const long D4 = (long)D * D * D * D, Dl = (long)D * D;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < D4 * D4; idx += (long)gridDim.x * 256) {
    const long p = idx / D4, q = idx % D4;
    const long r0 = p % D, d0 = (p / D) % D, l0 = (p / Dl) % D, u0 = p / (Dl * D);
    const long r1 = q % D, d1 = (q / D) % D, l1 = (q / Dl) % D, u1 = q / (Dl * D);
    out[idx] = xb[(((u0 * D + u1) * Dl + (l0 * D + l1)) * Dl + (d0 * D + d1)) * Dl + (r0 * D + r1)];
  }
}

struct EBufs {
  int n;                                   // d^2 open-leg pairs (ket s, bra t)
  double *L0, *left, *R1, *Y1, *W1, *W1p, *R0, *right;
  std::vector<double*> xs, xb, x2p, Y2p, W2p;
  double *Y3s, *W3s, *E, *Eb;
  double *Y3b, *W3b, *T3Tb, *Y1b, *R1b, *leftb, *L0b, *W1pb, *W1b, *rightb, *R0b;
  double *Ta, *Tb, *Tc, *St;
  double *Ar, *Abr, *mopen;
  // diagonal pair (plaquette): stacks of n N x N matrices, then N x N scratch
  double *pCt0, *pCt2, *pY, *pZt, *pCt0b;
  double *pCt1, *pCt3, *pCt1b, *pCt3b, *pH, *pCt2b, *pRb;
  double *pW[4], *pWb[4], *pCT[4], *pCTb, *pCTt, *pTt;
  double *pSite, *pA, *pAb, *pDots;
  double *pSiteS, *pSiteTS, *pSiteBS;     // per open pair (n of them, or 2)
};

size_t ecarve(const Dims& m, EBufs* b, char* base, std::vector<std::pair<uintptr_t, uintptr_t>>* reg) {
  Carver cv;
  cv.base = base;
  cv.reg = reg;
  const size_t x = m.x, Dl = m.Dl, NN = (size_t)m.N * m.N, L = x * Dl * x;
  const size_t Dl4 = Dl * Dl * Dl * Dl, D4 = (size_t)m.D * m.D * m.D * m.D;
  const int n = m.d * m.d;
  b->n = n;
  b->L0 = cv.take(L);
  b->left = cv.take(L);
  b->R1 = cv.take(NN);
  b->Y1 = cv.take(NN);
  b->W1 = cv.take(NN);
  b->W1p = cv.take(NN);
  b->R0 = cv.take(L);
  b->right = cv.take(L);
  b->xs.resize(n);
  b->xb.resize(n);
  b->x2p.resize(n);
  b->Y2p.resize(n);
  b->W2p.resize(n);
  for (int i = 0; i < n; ++i) {
    b->xs[i] = cv.take(Dl4);
    b->xb[i] = cv.take(Dl4);
    b->x2p[i] = cv.take(Dl4);
    b->Y2p[i] = cv.take(NN);
    b->W2p[i] = cv.take(NN);
  }
  b->Y3s = cv.take(n * L);
  b->W3s = cv.take(n * L);
  b->E = cv.take(n * n);
  b->Eb = cv.take(n * n);
  b->Y3b = cv.take(n * L);
  b->W3b = cv.take(n * L);
  b->T3Tb = cv.take(L);
  b->Y1b = cv.take(NN);
  b->R1b = cv.take(NN);
  b->leftb = cv.take(L);
  b->L0b = cv.take(L);
  b->W1pb = cv.take(NN);
  b->W1b = cv.take(NN);
  b->rightb = cv.take(L);
  b->R0b = cv.take(L);
  b->Ta = cv.take(NN);
  b->Tb = cv.take(NN);
  b->Tc = cv.take(NN);
  b->St = cv.take(NN);
  b->Ar = cv.take(m.d * D4);
  b->Abr = cv.take(m.d * D4);
  b->mopen = cv.take(D4 * D4);
  b->pCt0 = cv.take(n * NN);
  b->pCt2 = cv.take(n * NN);
  b->pY = cv.take(n * NN);
  b->pZt = cv.take(n * NN);
  b->pCt0b = cv.take(n * NN);
  for (double** q : {&b->pCt1, &b->pCt3, &b->pCt1b, &b->pCt3b, &b->pH, &b->pCt2b, &b->pRb})
    *q = cv.take(NN);
  for (int i = 0; i < 4; ++i) {
    b->pW[i] = cv.take(NN);
    b->pWb[i] = cv.take(NN);
    b->pCT[i] = cv.take(L);
  }
  b->pCTb = cv.take(L);
  b->pCTt = cv.take(L);
  b->pTt = cv.take(L);
  for (double** q : {&b->pSite, &b->pA, &b->pAb}) *q = cv.take(Dl4);
  b->pDots = cv.take((size_t)kMaxDots * kDotBlocks);
  const size_t ns = (size_t)std::max(n, 2);
  b->pSiteS = cv.take(ns * Dl4);
  b->pSiteTS = cv.take(ns * Dl4);
  b->pSiteBS = cv.take(ns * Dl4);
  return cv.off + 256;
}

GemmBatch one(int M, int N, int K, const void* A, long lda, int transA, const void* B, long ldb,
              void* C, long ldc, bool acc = false) {
  GemmBatch g = rowmajor(1, M, N, K, lda, ldb, ldc);
  g.A[0] = A;
  g.transA[0] = transA;
  g.B[0] = B;
  g.C[0] = C;
  g.accumulate = acc ? 1 : 0;
  return g;
}

// Forward horizontal chain: E[st1, st2] = <Y3_st1, W3_st2> for the open
// site tensors xs (a-layout [(u,l)][(d,r)]), slots C[0..3], T[0..3].
int echain_fwd(Run& r, const Dims& m, EBufs& b, const double* const* C, const double* const* T) {
  const int x = m.x, Dl = m.Dl, n = b.n;
  const long L = (long)x * Dl * x, D2 = (long)Dl * Dl;
  VTRY(gemm(r, one(x, Dl * x, x, C[3], x, 0, T[3], (long)Dl * x, b.L0, (long)Dl * x)));       // [j][(l,a)]
  VTRY(gemm(r, one(x * Dl, x, x, b.L0, x, 0, C[0], x, b.left, x)));                            // [(j,l)][b]
  VTRY(gemm(r, one(x * Dl, Dl * x, x, b.left, x, 0, T[0], (long)Dl * x, b.R1, (long)Dl * x)));  // [(j,l)][(u,g)]
  VTRY(gather(r, b.R1, b.Y1, x, x, Dl, Dl, D2 * x, 1, x, (long)Dl * x));                       // [(j,g)][(u,l)]
  VTRY(transpose(r, T[2], b.St, x, (long)Dl * x));                                             // [(d,j)][i]
  for (int st = 0; st < n; ++st) {
    VTRY(gemm(r, one(x * x, D2, D2, b.Y1, D2, 0, b.xs[st], D2, b.Ta, D2)));                   // [(j,g)][(d,m)]
    VTRY(gather(r, b.Ta, b.Y2p[st], x, Dl, Dl, x, D2, 1, Dl, (long)x * D2));                  // [(g,m)][(d,j)]
    VTRY(gemm(r, one(x * Dl, x, Dl * x, b.Y2p[st], (long)Dl * x, 0, b.St, x, b.Y3s + st * L, x)));
  }
  VTRY(gemm(r, one(x, Dl * x, x, C[1], x, 0, T[1], (long)Dl * x, b.R0, (long)Dl * x)));       // [h][(w,e)]
  VTRY(gemm(r, one(x * Dl, x, x, b.R0, x, 0, C[2], x, b.right, x)));                           // [(h,w)][f]
  VTRY(gemm(r, one(x * Dl, Dl * x, x, T[0], x, 0, b.right, (long)Dl * x, b.W1, (long)Dl * x)));  // [(g,v)][(w,f)]
  VTRY(gather(r, b.W1, b.W1p, x, x, Dl, Dl, D2 * x, 1, (long)Dl * x, x));                      // [(g,f)][(v,w)]
  for (int st = 0; st < n; ++st) {
    VTRY(gather(r, b.xs[st], b.x2p[st], Dl, Dl, Dl, Dl, D2 * Dl, 1, D2, Dl));                  // [(v,w)][(m,y)]
    VTRY(gemm(r, one(x * x, D2, D2, b.W1p, D2, 0, b.x2p[st], D2, b.Ta, D2)));                 // [(g,f)][(m,y)]
    VTRY(gather(r, b.Ta, b.W2p[st], x, Dl, x, Dl, (long)x * D2, Dl, D2, 1));                  // [(g,m)][(f,y)]
    VTRY(gemm(r, one(x * Dl, x, x * Dl, b.W2p[st], (long)x * Dl, 0, T[2], x, b.W3s + st * L, x)));
  }
  // E[i, j] = <Y3_i, W3_j>: n^2 dot products over L = x Dl x, spread over the
  // chip (a GEMM with an n x n result would run on one workgroup)
  const double* w3[kMaxDots];
  if (n > kMaxDots) return r.fail("energy chain: more open-leg pairs than supported");
  for (int j = 0; j < n; ++j) w3[j] = b.W3s + j * L;
  for (int i = 0; i < n; ++i) {
    const int rc = elem_dots(b.Y3s + i * L, w3, n, L, b.pDots, b.E + i * n, r.st);
    if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
  }
  return 0;
}

// Reverse horizontal chain from Eb: accumulates into Cb, Tb (slots as C, T)
// and into the open-layer cotangents b.xb.
int echain_bwd(Run& r, const Dims& m, EBufs& b, const double* const* C, const double* const* T,
               double* const* Cb, double* const* Tb) {
  const int x = m.x, Dl = m.Dl, n = b.n;
  const long L = (long)x * Dl * x, D2 = (long)Dl * Dl, NN = (long)m.N * m.N;
  VTRY(gemm(r, one(n, (int)L, n, b.Eb, n, 0, b.W3s, L, b.Y3b, L)));
  VTRY(gemm(r, one(n, (int)L, n, b.Eb, n, 1, b.Y3s, L, b.W3b, L)));
  VTRY(fill(r, b.T3Tb, L, 0.0));
  VTRY(fill(r, b.Y1b, NN, 0.0));
  VTRY(fill(r, b.W1pb, NN, 0.0));
  // Y2b of every open pair into the plaquette stack (idle here), then the
  // D2 x D2 x (x x) products xb += Y1^T Y2b batched over the pairs
  for (int st = 0; st < n; ++st) {
    double* y2b = b.pCt2 + st * NN;
    VTRY(gemm(r, one(x * Dl, Dl * x, x, b.Y3b + st * L, x, 0, T[2], (long)Dl * x, b.Ta, (long)Dl * x)));
    VTRY(gemm(r, one(Dl * x, x, x * Dl, b.Y2p[st], (long)Dl * x, 1, b.Y3b + st * L, x, b.T3Tb, x, true)));
    VTRY(gather(r, b.Ta, y2b, x, x, Dl, Dl, 1, D2 * x, x, (long)Dl * x));                     // Y2b [(j,g)][(d,m)]
    VTRY(transpose(r, b.xs[st], b.Tc, D2, D2));
    VTRY(gemm(r, one(x * x, D2, D2, y2b, D2, 0, b.Tc, D2, b.Y1b, D2, true)));
  }
  for (int s0 = 0; s0 < n; s0 += kMaxProb) {
    const int cnt = std::min(kMaxProb, n - s0);
    GemmBatch g = rowmajor(cnt, (int)D2, (int)D2, x * x, D2, D2, D2);
    g.accumulate = 1;
    for (int i = 0; i < cnt; ++i) {
      g.A[i] = b.Y1;
      g.transA[i] = 1;
      g.B[i] = b.pCt2 + (s0 + i) * NN;
      g.C[i] = b.xb[s0 + i];
    }
    VTRY(gemm(r, g));
  }
  VTRY(gather(r, b.T3Tb, Tb[2], 1, 1, x, (int)(Dl * x), 0, 0, 1, x, true));                    // += T3Tb^T
  VTRY(gather(r, b.Y1b, b.R1b, x, Dl, Dl, x, (long)x * D2, 1, Dl, D2));                       // [(j,l)][(u,g)]
  VTRY(transpose(r, T[0], b.St, x, (long)Dl * x));
  VTRY(gemm(r, one(x * Dl, x, Dl * x, b.R1b, (long)Dl * x, 0, b.St, x, b.leftb, x)));
  VTRY(gemm(r, one(x, Dl * x, x * Dl, b.left, x, 1, b.R1b, (long)Dl * x, Tb[0], (long)Dl * x, true)));
  VTRY(transpose(r, C[0], b.St, x, x));
  VTRY(gemm(r, one(x * Dl, x, x, b.leftb, x, 0, b.St, x, b.L0b, x)));
  VTRY(gemm(r, one(x, x, x * Dl, b.L0, x, 1, b.leftb, x, Cb[0], x, true)));
  VTRY(transpose(r, T[3], b.St, x, (long)Dl * x));
  VTRY(gemm(r, one(x, x, Dl * x, b.L0b, (long)Dl * x, 0, b.St, x, Cb[3], x, true)));
  VTRY(gemm(r, one(x, Dl * x, x, C[3], x, 1, b.L0b, (long)Dl * x, Tb[3], (long)Dl * x, true)));
  // w chain
  VTRY(transpose(r, T[2], b.St, (long)x * Dl, x));                                            // [i][(f,y)]
  for (int st = 0; st < n; ++st) {
    double* w2b = b.pCt2 + st * NN;
    VTRY(gemm(r, one(x * Dl, x * Dl, x, b.W3b + st * L, x, 0, b.St, (long)x * Dl, b.Ta, (long)x * Dl)));
    VTRY(gemm(r, one(x * Dl, x, x * Dl, b.W2p[st], (long)x * Dl, 1, b.W3b + st * L, x, Tb[2], x, true)));
    VTRY(gather(r, b.Ta, w2b, x, x, Dl, Dl, D2 * x, Dl, (long)x * Dl, 1));                    // W2b [(g,f)][(m,y)]
    VTRY(transpose(r, b.x2p[st], b.Tc, D2, D2));
    VTRY(gemm(r, one(x * x, D2, D2, w2b, D2, 0, b.Tc, D2, b.W1pb, D2, true)));
  }
  // x2p_bar of every pair (D2 x D2 x (x x), batched), then into xb
  for (int s0 = 0; s0 < n; s0 += kMaxProb) {
    const int cnt = std::min(kMaxProb, n - s0);
    GemmBatch g = rowmajor(cnt, (int)D2, (int)D2, x * x, D2, D2, D2);
    for (int i = 0; i < cnt; ++i) {
      g.A[i] = b.W1p;
      g.transA[i] = 1;
      g.B[i] = b.pCt2 + (s0 + i) * NN;
      g.C[i] = b.pCt0 + (s0 + i) * NN;
    }
    VTRY(gemm(r, g));
  }
  for (int st = 0; st < n; ++st)
    VTRY(gather(r, b.pCt0 + st * NN, b.xb[st], Dl, Dl, Dl, Dl, D2 * Dl, Dl, 1, D2, true));
  VTRY(gather(r, b.W1pb, b.W1b, x, Dl, Dl, x, (long)x * D2, Dl, 1, D2));                      // [(g,v)][(w,f)]
  VTRY(transpose(r, b.right, b.St, x, (long)Dl * x));
  VTRY(gemm(r, one(x * Dl, x, Dl * x, b.W1b, (long)Dl * x, 0, b.St, x, Tb[0], x, true)));
  VTRY(gemm(r, one(x, Dl * x, x * Dl, T[0], x, 1, b.W1b, (long)Dl * x, b.rightb, (long)Dl * x)));
  VTRY(transpose(r, C[2], b.St, x, x));
  VTRY(gemm(r, one(x * Dl, x, x, b.rightb, x, 0, b.St, x, b.R0b, x)));
  VTRY(gemm(r, one(x, x, x * Dl, b.R0, x, 1, b.rightb, x, Cb[2], x, true)));
  VTRY(transpose(r, T[1], b.St, x, (long)Dl * x));
  VTRY(gemm(r, one(x, x, Dl * x, b.R0b, (long)Dl * x, 0, b.St, x, Cb[1], x, true)));
  VTRY(gemm(r, one(x, Dl * x, x, C[1], x, 1, b.R0b, (long)Dl * x, Tb[1], (long)Dl * x, true)));
  return 0;
}

// Open double layers of the site tensor `site` into b.xs (pairs (s,t)).
int open_layers(Run& r, const Dims& m, EBufs& b, const double* site) {
  for (int s = 0; s < m.d; ++s)
    for (int t = 0; t < m.d; ++t) {
      const int rc = elem_double_layer(site, nullptr, b.xs[s * m.d + t], m.d, m.D, r.st, s, t);
      if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
    }
  return 0;
}

// site_bar[s] += M_st site[t],  site_bar[t] += M_st^T site[s]  (M_st = [ket][bra] of xb_st)
int open_vjp(Run& r, const Dims& m, EBufs& b, const double* site, double* site_bar) {
  const long D4 = (long)m.D * m.D * m.D * m.D;
  for (int s = 0; s < m.d; ++s)
    for (int t = 0; t < m.d; ++t) {
      if (!r.inside(b.mopen, (size_t)D4 * D4 * 8)) return r.fail("adjoint buffer too small");
      k_open_reorder<<<(int)std::min<long>(4096, (D4 * D4 + 255) / 256), 256, 0, r.st>>>(
          b.xb[s * m.d + t], b.mopen, m.D);
      CTM_HIP_TRY(hipGetLastError());
      VTRY(gemm(r, one((int)D4, 1, (int)D4, b.mopen, D4, 0, site + t * D4, 1, site_bar + s * D4, 1, true)));
      VTRY(gemm(r, one((int)D4, 1, (int)D4, b.mopen, D4, 1, site + s * D4, 1, site_bar + t * D4, 1, true)));
    }
  return 0;
}

// value = sum E op' / sum_diag E and dvalue/dE (host, d^4 numbers)
double bond_value_and_bar(const std::vector<double>& E, const double* op, int d, std::vector<double>& Eb) {
  const int n = d * d;
  double num = 0.0, den = 0.0;
  for (int s1 = 0; s1 < d; ++s1)
    for (int t1 = 0; t1 < d; ++t1)
      for (int s2 = 0; s2 < d; ++s2)
        for (int t2 = 0; t2 < d; ++t2) {
          const double e = E[(s1 * d + t1) * n + (s2 * d + t2)];
          num += op[(t1 * d + t2) * n + (s1 * d + s2)] * e;
          if (s1 == t1 && s2 == t2) den += e;
        }
  const double val = num / den;
  Eb.assign(n * n, 0.0);
  for (int s1 = 0; s1 < d; ++s1)
    for (int t1 = 0; t1 < d; ++t1)
      for (int s2 = 0; s2 < d; ++s2)
        for (int t2 = 0; t2 < d; ++t2)
          Eb[(s1 * d + t1) * n + (s2 * d + t2)] =
              (op[(t1 * d + t2) * n + (s1 * d + s2)] - (s1 == t1 && s2 == t2 ? val : 0.0)) / den;
  return val;
}

}  // namespace

extern "C" {

ctm_status ctm_vjp_workspace_bytes(const ctm_config* cfg, size_t* bytes) {
  if (!bytes) return CTM_E_ARG;
  const int rc = check_cfg(cfg);
  if (rc) {
    set_thread_error("the adjoint needs an iPEPS site (d >= 1), SI projectors, float64 "
                     "contractions, the stabilised update and no lattice symmetry");
    return (ctm_status)rc;
  }
  Bufs b;
  EBufs eb;
  *bytes = std::max(carve(dims_of(*cfg), &b, nullptr, nullptr),
                    ecarve(dims_of(*cfg), &eb, nullptr, nullptr));
  return CTM_OK;
}

ctm_status ctm_move_vjp(ctm_ctx* ctx, const double* state_in, const double* state_out_bar,
                        double* state_in_bar, double* state_out, double* site_bar, void* ws,
                        size_t ws_bytes) {
  if (!ctx || !state_in || !state_out_bar || !state_in_bar || !ws) {
    set_thread_error("null argument");
    return CTM_E_ARG;
  }
  Prepared P;
  int rc = prepare(ctx, state_in, ws, ws_bytes, P,
                   {{state_out_bar, 0}, {state_in_bar, 0}, {state_out, 0}});
  if (!rc && site_bar) {
    const size_t D4 = (size_t)P.m.D * P.m.D * P.m.D * P.m.D;
    P.r.reg.push_back({(uintptr_t)site_bar, (uintptr_t)(site_bar + P.m.d * D4)});
  }
  if (!rc && state_out) {
    double *C[4], *T[4], *X[4], *Y[4];
    split(state_out, P.m, C, T, X, Y);
    const long x = P.m.x, Dl = P.m.Dl;
    for (int i = 0; i < 4 && !rc; ++i) {
      rc = copy(P.r, P.b.Cn[i], C[i], x * x);
      if (!rc) rc = copy(P.r, P.b.Tn[i], T[i], x * Dl * x);
    }
    if (!rc) {
      // recycled blocks X' = Xf v_s, Y^T' = Yf u_s
      const int N = P.m.N, k = P.m.k, last = 10 * P.m.nsi - 1;
      GemmBatch g = rowmajor(8, N, k, k, k, k, k);
      for (int i = 0; i < 4; ++i) {
        g.A[i] = P.m.nsi > 0 ? P.b.tape[i][last] : P.in.X[i];
        g.B[i] = P.b.vs[i];
        g.C[i] = X[i];
        g.A[4 + i] = P.m.nsi > 0 ? P.b.tape[4 + i][last] : P.in.Yt[i];
        g.B[4 + i] = P.b.us[i];
        g.C[4 + i] = Y[i];
      }
      rc = gemm(P.r, g);
    }
    if (!rc) rc = copy(P.r, state_in + (P.nstate - 4), state_out + (P.nstate - 4), 4);
  }
  if (!rc) rc = reverse(P, state_out_bar, state_in_bar, site_bar);
  if (rc) return (ctm_status)rc;
  if (hipStreamSynchronize(P.v.st) != hipSuccess)
    return (ctm_status)vjp_fail(ctx, CTM_E_DEVICE, "synchronisation failed");
  return CTM_OK;
}

ctm_status ctm_fixed_point_vjp(ctm_ctx* ctx, const double* state_star, const double* g_bar,
                               double tol, int max_iter, double* x_bar, double* site_bar,
                               void* ws, size_t ws_bytes, int* iters, double* rel_norm) {
  if (!ctx || !state_star || !g_bar || !site_bar || !ws || max_iter < 1 || !(tol >= 0.0)) {
    set_thread_error("invalid argument");
    return CTM_E_ARG;
  }
  Prepared P;
  int rc = prepare(ctx, state_star, ws, ws_bytes, P, {{g_bar, 0}, {x_bar, 0}});
  if (rc) return (ctm_status)rc;
  const size_t D4 = (size_t)P.m.D * P.m.D * P.m.D * P.m.D;
  P.r.reg.push_back({(uintptr_t)site_bar, (uintptr_t)(site_bar + P.m.d * D4)});
  const long n = (long)P.nstate - 4;
  // |v|^2 of the cotangent (counters excluded), read back to the host
  auto norm2 = [&](const double* v, double* out) -> int {
    DotArgs da{};
    da.x[0] = v;
    da.y[0] = v;
    da.n[0] = n;
    da.out = P.b.fp_dot;
    if (launch_dots(da, 1, P.b.dpart, P.r.st)) return 1;
    CTM_HIP_TRY(hipMemcpyAsync(out, P.b.fp_dot, sizeof(double), hipMemcpyDeviceToHost, P.r.st));
    CTM_HIP_TRY(hipStreamSynchronize(P.r.st));
    return 0;
  };
  double g2 = 0.0;
  rc = norm2(g_bar, &g2);
  if (rc) return (ctm_status)rc;
  rc = copy(P.r, g_bar, P.b.fp_v[0], (long)P.nstate);
  if (!rc && x_bar) rc = copy(P.r, g_bar, x_bar, (long)P.nstate);
  int it = 0, cur = 0;
  double rel = g2 > 0.0 ? 1.0 : 0.0;
  // x_bar = sum_n (J_x^T)^n g,  site_bar += sum_n J_A^T (J_x^T)^n g
  while (!rc && it < max_iter && rel > tol) {
    rc = reverse(P, P.b.fp_v[cur], P.b.fp_v[1 - cur], site_bar);
    if (rc) break;
    cur = 1 - cur;
    ++it;
    if (x_bar) {
      rc = gather(P.r, P.b.fp_v[cur], x_bar, 1, 1, 1, (int)n, 0, 0, 0, 1, true);
      if (rc) break;
    }
    double v2 = 0.0;
    rc = norm2(P.b.fp_v[cur], &v2);
    rel = g2 > 0.0 ? std::sqrt(v2 / g2) : 0.0;
  }
  if (iters) *iters = it;
  if (rel_norm) *rel_norm = rel;
  if (rc) return (ctm_status)rc;
  if (hipStreamSynchronize(P.v.st) != hipSuccess)
    return (ctm_status)vjp_fail(ctx, CTM_E_DEVICE, "synchronisation failed");
  return rel <= tol ? CTM_OK : CTM_E_NOT_CONVERGED;
}


}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Diagonal pair of the 2x2 plaquette (site 1 in corner 0, site 2 in corner 2):
// E[i, j] = Tr(Ct0(xs_i) Ct1 Ct2(xs_j) Ct3) with Ct_k = W_k site_k,
// W_k = T_(k-1) (C_k T_k), and its reverse pass.  The anti-diagonal is the
// diagonal of the network turned by 90 degrees (slots shifted by one, site
// legs rotated), as the vertical bond is the turned horizontal one.
// ---------------------------------------------------------------------------
const long kPerm[4][4] = {{2, 3, 1, 0}, {3, 0, 2, 1}, {0, 1, 3, 2}, {1, 2, 0, 3}};
// site_k[i0, i1, i2, i3] = a[sum_j i_j * Dl^kPerm[k][j]]: the a-leg strides
// (as powers of Dl: u = 3, l = 2, d = 1, r = 0) of the four site-tensor
// legs in the corner-k absorption.

long dl_pow(long Dl, int e) {
  long v = 1;
  for (int i = 0; i < e; ++i) v *= Dl;
  return v;
}

int pq_site(Run& r, const Dims& m, int k, const double* a_layout, double* out) {
  const long Dl = m.Dl;
  return gather(r, a_layout, out, (int)Dl, (int)Dl, (int)Dl, (int)Dl, dl_pow(Dl, kPerm[k][0]),
                dl_pow(Dl, kPerm[k][1]), dl_pow(Dl, kPerm[k][2]), dl_pow(Dl, kPerm[k][3]));
}

// out (N x N) = enlarged corner k with the site tensor xs (a-layout).
int pq_corner(Run& r, const Dims& m, EBufs& b, int k, const double* xs, double* out) {
  const int x = m.x, Dl = m.Dl;
  const long N = m.N;
  VTRY(pq_site(r, m, k, xs, b.pSite));
  GemmBatch g = one(x * x, Dl * Dl, Dl * Dl, b.pW[k], (long)Dl * Dl, 0, b.pSite, (long)Dl * Dl, out, 0);
  g.cdiv_m = x;
  g.cs_m1 = (long)Dl * N;
  g.cs_m0 = Dl;
  g.cdiv_n = Dl;
  g.cs_n1 = N;
  g.cs_n0 = 1;
  return gemm(r, g);
}

void transposed_out(GemmBatch& g, long N) {
  g.cdiv_m = 1 << 30;
  g.cs_m1 = 0;
  g.cs_m0 = 1;
  g.cdiv_n = 1 << 30;
  g.cs_n1 = 0;
  g.cs_n0 = N;
}

// Forward: fills b.E (n x n) from the open layers b.xs; keeps the tape.
int pq_fwd(Run& r, const Dims& m, EBufs& b, const double* const* C, const double* const* T) {
  const int x = m.x, Dl = m.Dl, n = b.n;
  const long N = m.N, NN = N * N, Dl4 = (long)Dl * Dl * Dl * Dl;
  for (int k = 0; k < 4; ++k) {
    VTRY(gemm(r, one(x, Dl * x, x, C[k], x, 0, T[k], (long)Dl * x, b.pCT[k], (long)Dl * x)));
    GemmBatch g = one(x * Dl, Dl * x, x, T[(k + 3) % 4], x, 0, b.pCT[k], (long)Dl * x, b.pW[k], 0);
    g.cdiv_m = Dl;
    g.cs_m1 = (long)x * Dl * Dl;
    g.cs_m0 = Dl;
    g.cdiv_n = x;
    g.cs_n1 = 1;
    g.cs_n0 = (long)Dl * Dl;
    VTRY(gemm(r, g));
  }
  // the closed double layer a = sum_s xs[(s, s)]
  VTRY(fill(r, b.pA, Dl4, 0.0));
  for (int s = 0; s < m.d; ++s)
    VTRY(gather(r, b.xs[s * m.d + s], b.pA, Dl, Dl, Dl, Dl, (long)Dl * Dl * Dl, (long)Dl * Dl, Dl, 1,
                true));
  VTRY(pq_corner(r, m, b, 1, b.pA, b.pCt1));
  VTRY(pq_corner(r, m, b, 3, b.pA, b.pCt3));
  const double* zt[kMaxDots];
  for (int j = 0; j < n; ++j) {
    double* c2 = b.pCt2 + j * NN;
    double* y = b.pY + j * NN;
    VTRY(pq_corner(r, m, b, 2, b.xs[j], c2));
    VTRY(gemm(r, one((int)N, (int)N, (int)N, b.pCt1, N, 0, c2, N, y, N)));
    GemmBatch g = one((int)N, (int)N, (int)N, y, N, 0, b.pCt3, N, b.pZt + j * NN, 0);
    transposed_out(g, N);
    VTRY(gemm(r, g));
    zt[j] = b.pZt + j * NN;
  }
  for (int i = 0; i < n; ++i) {
    double* c0 = b.pCt0 + i * NN;
    VTRY(pq_corner(r, m, b, 0, b.xs[i], c0));
    const int rc = elem_dots(c0, zt, n, NN, b.pDots, b.E + i * n, r.st);
    if (rc) return vjp_fail(r.c, rc == 1 ? CTM_E_ARG : rc, thread_error());
  }
  return 0;
}

// Reverse pass of the site absorptions of `cnt` corner instances: corner
// ks[i] with site tensor xs[i] (a-layout) and its cotangent regrouped as
// P_i[(x_in, y), (o1, o2)] (at b.pCt0 + i NN): pWb[ks[i]] += P_i site_i^T,
// and xbar[i] += (W^T P_i) returned to the a-layout; the W^T P products (a
// D2 x D2 result over K = x^2) run batched.
int pq_absorb_bwd(Run& r, const Dims& m, EBufs& b, const int* ks, const double* const* xs,
                  double* const* xbar, int cnt) {
  const int x = m.x, Dl = m.Dl;
  const long NN = (long)m.N * m.N, D2 = (long)Dl * Dl, Dl4 = D2 * D2;
  for (int i = 0; i < cnt; ++i) {
    double* site = b.pSiteS + i * Dl4;
    VTRY(pq_site(r, m, ks[i], xs[i], site));
    VTRY(transpose(r, site, b.pSiteTS + i * Dl4, D2, D2));
    VTRY(gemm(r, one(x * x, (int)D2, (int)D2, b.pCt0 + i * NN, D2, 0, b.pSiteTS + i * Dl4, D2,
                     b.pWb[ks[i]], D2, true)));
  }
  for (int s0 = 0; s0 < cnt; s0 += kMaxProb) {
    const int c = std::min(kMaxProb, cnt - s0);
    GemmBatch g = rowmajor(c, (int)D2, (int)D2, x * x, D2, D2, D2);
    for (int i = 0; i < c; ++i) {
      g.A[i] = b.pW[ks[s0 + i]];
      g.transA[i] = 1;
      g.B[i] = b.pCt0 + (s0 + i) * NN;
      g.C[i] = b.pSiteBS + (s0 + i) * Dl4;
    }
    VTRY(gemm(r, g));
  }
  // xbar[u, l, d, r] += siteB[i0..i3] where leg j of the site carries a-leg kPerm[k][j]
  for (int i = 0; i < cnt; ++i) {
    long st[4];
    for (int j = 0; j < 4; ++j) st[3 - kPerm[ks[i]][j]] = dl_pow(Dl, 3 - j);
    VTRY(gather(r, b.pSiteBS + i * Dl4, xbar[i], Dl, Dl, Dl, Dl, st[0], st[1], st[2], st[3], true));
  }
  return 0;
}

// P[(x_in, y), (o1, o2)] = Ctb[(x_in, o1), (y, o2)]
int pq_regroup(Run& r, const Dims& m, const double* Ctb, double* P) {
  const int x = m.x, Dl = m.Dl;
  const long N = m.N;
  return gather(r, Ctb, P, x, x, Dl, Dl, (long)Dl * N, Dl, N, 1);
}

// Reverse pass from b.Eb: accumulates into Cb, Tb (slots as C, T) and b.xb.
int pq_bwd(Run& r, const Dims& m, EBufs& b, const double* const* C, const double* const* T,
           double* const* Cb, double* const* Tb) {
  const int x = m.x, Dl = m.Dl, n = b.n;
  const long N = m.N, NN = N * N, Dl4 = (long)Dl * Dl * Dl * Dl;
  for (int k = 0; k < 4; ++k) VTRY(fill(r, b.pWb[k], NN, 0.0));
  VTRY(fill(r, b.pCt1b, NN, 0.0));
  VTRY(fill(r, b.pCt3b, NN, 0.0));
  VTRY(fill(r, b.pAb, Dl4, 0.0));
  // Ct0b_i = sum_j Eb[i, j] Zt_j;  G_j = sum_i Eb[i, j] Ct0_i (into the Zt stack)
  VTRY(gemm(r, one(n, (int)NN, n, b.Eb, n, 0, b.pZt, NN, b.pCt0b, NN)));
  VTRY(gemm(r, one(n, (int)NN, n, b.Eb, n, 1, b.pCt0, NN, b.pZt, NN)));
  int ks[kMaxDots];
  for (int i = 0; i < n; ++i) {                 // the Ct0 stack is free from here on
    VTRY(pq_regroup(r, m, b.pCt0b + i * NN, b.pCt0 + i * NN));
    ks[i] = 0;
  }
  VTRY(pq_absorb_bwd(r, m, b, ks, b.xs.data(), b.xb.data(), n));
  for (int j = 0; j < n; ++j) {
    const double* G = b.pZt + j * NN;       // cotangent of Zt_j = (Y_j Ct3)^T
    const double* c2 = b.pCt2 + j * NN;
    const double* y = b.pY + j * NN;
    // H = Y_j_bar^T = Ct3 G
    VTRY(gemm(r, one((int)N, (int)N, (int)N, b.pCt3, N, 0, G, N, b.pH, N)));
    GemmBatch g = one((int)N, (int)N, (int)N, G, N, 0, y, N, b.pCt3b, 0, true);   // (G Y)^T
    transposed_out(g, N);
    VTRY(gemm(r, g));
    g = one((int)N, (int)N, (int)N, c2, N, 0, b.pH, N, b.pCt1b, 0, true);          // (Ct2 H)^T
    transposed_out(g, N);
    VTRY(gemm(r, g));
    g = one((int)N, (int)N, (int)N, b.pH, N, 0, b.pCt1, N, b.pCt2b, 0);            // (H Ct1)^T
    transposed_out(g, N);
    VTRY(gemm(r, g));
    VTRY(pq_regroup(r, m, b.pCt2b, b.pCt0 + j * NN));
  }
  for (int j = 0; j < n; ++j) ks[j] = 2;
  VTRY(pq_absorb_bwd(r, m, b, ks, b.xs.data(), b.xb.data(), n));
  {
    VTRY(pq_regroup(r, m, b.pCt1b, b.pCt0));
    VTRY(pq_regroup(r, m, b.pCt3b, b.pCt0 + NN));
    const int kc[2] = {1, 3};
    const double* xa[2] = {b.pA, b.pA};
    double* xab[2] = {b.pAb, b.pAb};
    VTRY(pq_absorb_bwd(r, m, b, kc, xa, xab, 2));
  }
  for (int s = 0; s < m.d; ++s)
    VTRY(gather(r, b.pAb, b.xb[s * m.d + s], Dl, Dl, Dl, Dl, (long)Dl * Dl * Dl, (long)Dl * Dl, Dl, 1,
                true));
  // W_k = R_k regrouped, R_k = T_(k-1) CT_k, CT_k = C_k T_k
  for (int k = 0; k < 4; ++k) {
    const int km = (k + 3) % 4;
    VTRY(gather(r, b.pWb[k], b.pRb, x, Dl, Dl, x, (long)x * Dl * Dl, Dl, 1, (long)Dl * Dl));
    VTRY(transpose(r, b.pCT[k], b.pCTt, x, (long)Dl * x));
    VTRY(gemm(r, one(x * Dl, x, Dl * x, b.pRb, (long)Dl * x, 0, b.pCTt, x, Tb[km], x, true)));
    VTRY(gemm(r, one(x, Dl * x, x * Dl, T[km], x, 1, b.pRb, (long)Dl * x, b.pCTb, (long)Dl * x)));
    VTRY(transpose(r, T[k], b.pTt, x, (long)Dl * x));
    VTRY(gemm(r, one(x, x, Dl * x, b.pCTb, (long)Dl * x, 0, b.pTt, x, Cb[k], x, true)));
    VTRY(gemm(r, one(x, Dl * x, x, C[k], x, 1, b.pCTb, (long)Dl * x, Tb[k], (long)Dl * x, true)));
  }
  return 0;
}

// ops[dir] is the d^2 x d^2 operator of bond dir (0 H, 1 V, 2 D, 3 AD) for
// every dir in the mask `bonds`.
int energy_vjp_impl(ctm_ctx* ctx, const double* state, const double* const* ops, int bonds,
                    double* e_out, double* state_bar, double* site_bar, void* ws, size_t ws_bytes) {
  VjpView v;
  int rc = vjp_view(ctx, &v);
  if (rc) return rc;
  if (check_cfg(&v.cfg))
    return (ctm_status)vjp_fail(ctx, CTM_E_ARG,
                                "the energy gradient needs an iPEPS site (d >= 1), SI projectors, "
                                "float64 contractions, the stabilised update and no lattice symmetry");
  const Dims m = dims_of(v.cfg);
  EBufs b;
  const size_t need = ecarve(m, &b, nullptr, nullptr);
  if (ws_bytes < need)
    return (ctm_status)vjp_fail(ctx, CTM_E_ARG, "adjoint workspace too small (need " +
                                                    std::to_string(need) + " bytes)");
  Run r;
  r.c = ctx;
  r.st = v.st;
  r.sk_part = v.sk_part;
  r.sk_cus = v.sk_cus;
  const size_t x = m.x, Dl = m.Dl, N = m.N, k = m.k, D4 = (size_t)m.D * m.D * m.D * m.D;
  const size_t nstate = 4 * x * x + 4 * x * Dl * x + 8 * N * k + 4;
  double chi_env = 0.0;
  if (hipMemcpyAsync(&chi_env, state + (nstate - 4), sizeof(double), hipMemcpyDeviceToHost, v.st) !=
          hipSuccess ||
      hipStreamSynchronize(v.st) != hipSuccess)
    return (ctm_status)vjp_fail(ctx, CTM_E_DEVICE, "reading chi_env of the state failed");
  if ((int)chi_env != m.x)
    return (ctm_status)vjp_fail(ctx, CTM_E_STATE, "the energy gradient needs chi_env == chi");
  ecarve(m, &b, (char*)ws, &r.reg);
  r.reg.push_back({(uintptr_t)state, (uintptr_t)(state + nstate)});
  r.reg.push_back({(uintptr_t)state_bar, (uintptr_t)(state_bar + nstate)});
  r.reg.push_back({(uintptr_t)site_bar, (uintptr_t)(site_bar + m.d * D4)});
  r.reg.push_back({(uintptr_t)v.A_site, (uintptr_t)(v.A_site + m.d * D4)});
  const double *C[4], *T[4];
  double *Cb[4], *Tb[4];
  {
    const double* p = state;
    double* q = state_bar;
    for (int i = 0; i < 4; ++i, p += x * x, q += x * x) {
      C[i] = p;
      Cb[i] = q;
    }
    for (int i = 0; i < 4; ++i, p += x * Dl * x, q += x * Dl * x) {
      T[i] = p;
      Tb[i] = q;
    }
  }
  VTRY(fill(r, state_bar, (long)nstate, 0.0));
  const int n = b.n;
  std::vector<double> E(n * n), Eb;
  double total = 0.0;
  for (int dir = 0; dir < 4; ++dir) {
    // dir 0: horizontal pair; dir 1: vertical pair = horizontal pair of the
    // turned network (slot i holds corner / edge i+1, site legs rotated);
    // dir 2: diagonal pair; dir 3: anti-diagonal = diagonal of the turned one
    if (!(bonds & (1 << dir))) continue;
    const bool turned = dir & 1;
    const double* Cs[4];
    const double* Ts[4];
    double* Cbs[4];
    double* Tbs[4];
    for (int i = 0; i < 4; ++i) {
      const int j = turned ? md(i + 1) : i;
      Cs[i] = C[j];
      Ts[i] = T[j];
      Cbs[i] = Cb[j];
      Tbs[i] = Tb[j];
    }
    const double* site = v.A_site;
    if (turned) {
      // Ar[s, i1, i2, i3, i4] = A[s, u = i2, l = i3, d = i4, r = i1]
      const long D = m.D;
      for (int s = 0; s < m.d; ++s)
        VTRY(gather(r, v.A_site + s * D4, b.Ar + s * D4, (int)D, (int)D, (int)D, (int)D, 1, D * D * D,
                    D * D, D));
      site = b.Ar;
    }
    VTRY(open_layers(r, m, b, site));
    if (dir < 2)
      VTRY(echain_fwd(r, m, b, Cs, Ts));
    else
      VTRY(pq_fwd(r, m, b, Cs, Ts));
    CTM_HIP_TRY(hipMemcpyAsync(E.data(), b.E, n * n * sizeof(double), hipMemcpyDeviceToHost, r.st));
    CTM_HIP_TRY(hipStreamSynchronize(r.st));
    const std::vector<double> op(ops[dir], ops[dir] + n * n);
    total += bond_value_and_bar(E, op.data(), m.d, Eb);
    CTM_HIP_TRY(hipMemcpyAsync(b.Eb, Eb.data(), n * n * sizeof(double), hipMemcpyHostToDevice, r.st));
    for (int st = 0; st < n; ++st) VTRY(fill(r, b.xb[st], (long)Dl * Dl * Dl * Dl, 0.0));
    if (dir < 2)
      VTRY(echain_bwd(r, m, b, Cs, Ts, Cbs, Tbs));
    else
      VTRY(pq_bwd(r, m, b, Cs, Ts, Cbs, Tbs));
    if (!turned) {
      VTRY(open_vjp(r, m, b, v.A_site, site_bar));
    } else {
      VTRY(fill(r, b.Abr, (long)(m.d * D4), 0.0));
      VTRY(open_vjp(r, m, b, b.Ar, b.Abr));
      // A_bar[s,u,l,d,r] += Ar_bar[s, r, u, l, d]
      const long D = m.D;
      for (int s = 0; s < m.d; ++s)
        VTRY(gather(r, b.Abr + s * D4, site_bar + s * D4, (int)D, (int)D, (int)D, (int)D, D * D, D, 1,
                    D * D * D, true));
    }
  }
  if (hipStreamSynchronize(v.st) != hipSuccess)
    return vjp_fail(ctx, CTM_E_DEVICE, "synchronisation failed");
  if (e_out) *e_out = total;
  return CTM_OK;
}

}  // namespace

extern "C" {

ctm_status ctm_energy_vjp(ctm_ctx* ctx, const double* state, const double* op_host, double* e_out,
                          double* state_bar, double* site_bar, void* ws, size_t ws_bytes) {
  if (!ctx || !state || !op_host || !state_bar || !site_bar || !ws) {
    set_thread_error("null argument");
    return CTM_E_ARG;
  }
  const double* ops[4] = {op_host, op_host, nullptr, nullptr};
  return (ctm_status)energy_vjp_impl(ctx, state, ops, 3, e_out, state_bar, site_bar, ws, ws_bytes);
}

ctm_status ctm_bond_energy_vjp(ctm_ctx* ctx, const double* state, const double* ops_host, int bonds,
                               double* e_out, double* state_bar, double* site_bar, void* ws,
                               size_t ws_bytes) {
  if (!ctx || !state || !ops_host || !state_bar || !site_bar || !ws) {
    set_thread_error("null argument");
    return CTM_E_ARG;
  }
  if (bonds <= 0 || bonds > 15) {
    set_thread_error("bonds must be a non-empty mask of H = 1, V = 2, D = 4, AD = 8");
    return CTM_E_ARG;
  }
  // one d^2 x d^2 operator per bond of the mask, in the order H, V, D, AD
  const long n2 = (long)ctx_phys_dim(ctx) * ctx_phys_dim(ctx);
  const double* ops[4] = {nullptr, nullptr, nullptr, nullptr};
  long o = 0;
  for (int dir = 0; dir < 4; ++dir)
    if (bonds & (1 << dir)) {
      ops[dir] = ops_host + o;
      o += n2 * n2;
    }
  return (ctm_status)energy_vjp_impl(ctx, state, ops, bonds, e_out, state_bar, site_bar, ws,
                                     ws_bytes);
}

}  // extern "C"
