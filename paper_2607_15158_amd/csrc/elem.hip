// Element-wise and reduction kernels of a CTMRG move: double layer, leg
// permutations, initial boundary, normalisation, the sign rule, projector
// scaling with the pseudo-inverse cutoff, spectra and the convergence
// measure.  None of these is on the FLOP-critical path; they are written for
// clarity and coalesced access.

#include "elem.h"

namespace sictm {
namespace {

template <typename T> __device__ __forceinline__ T from_f64(double x) { return (T)x; }
template <> __device__ __forceinline__ __bf16 from_f64<__bf16>(double x) { return (__bf16)(float)x; }

__device__ __forceinline__ double block_sum(double x, double* sh) {
  // 256-thread block reduction
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// a[(uU),(lL),(dD),(rR)] = sum_{s,t} A[s,u,l,d,r] O[t,s] A[t,U,L,D,R]   (O = identity if null)
__global__ void k_double_layer(const double* A, const double* O, double* a, int d, int D,
                               int s_fix, int t_fix) {
  const long D4 = (long)D * D * D * D;
  const long total = D4 * D4;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    // a index: ((((u U) l L) d D) r R) with each pair ket-major
    long rem = i;
    const int R = rem % D; rem /= D;
    const int r = rem % D; rem /= D;
    const int Dd = rem % D; rem /= D;
    const int dd = rem % D; rem /= D;
    const int L = rem % D; rem /= D;
    const int l = rem % D; rem /= D;
    const int U = rem % D; rem /= D;
    const int u = (int)rem;
    const long ket = (((long)u * D + l) * D + dd) * D + r;
    const long bra = (((long)U * D + L) * D + Dd) * D + R;
    double acc = 0.0;
    if (s_fix >= 0) {
      acc = A[s_fix * D4 + ket] * A[t_fix * D4 + bra];
    } else if (O == nullptr) {
      for (int s = 0; s < d; ++s) acc += A[s * D4 + ket] * A[s * D4 + bra];
    } else {
      for (int s = 0; s < d; ++s)
        for (int t = 0; t < d; ++t) acc += A[s * D4 + ket] * O[t * d + s] * A[t * D4 + bra];
    }
    a[i] = acc;
  }
}

template <typename T>
__global__ void k_permute4(const double* src, T* dst, int n, long s0, long s1, long s2, long s3) {
  const long total = (long)n * n * n * n;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    long rem = i;
    const int i3 = rem % n; rem /= n;
    const int i2 = rem % n; rem /= n;
    const int i1 = rem % n; rem /= n;
    const int i0 = (int)rem;
    dst[i] = from_f64<T>(src[i0 * s0 + i1 * s1 + i2 * s2 + i3 * s3]);
  }
}

// Initial environment: close outer legs with e (see ctm.h / oracle docs).
// C1[d,r] = a[u,l,d,r] e_u e_l        T1[l,d,r] = a[u,l,d,r] e_u
// C2[l,d] = a e_u e_r                 T2[u,l,d] = a e_r
// C3[u,l] = a e_d e_r                 T3[r,u,l] = a e_d
// C4[r,u] = a e_l e_d                 T4[d,r,u] = a e_l
__global__ void k_init_env(const double* a, const double* e, int n, double* C1, double* C2,
                           double* C3, double* C4, double* T1, double* T2, double* T3,
                           double* T4) {
  const long n2 = (long)n * n, n3 = n2 * n;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  auto A = [&](int u, int l, int d, int r) { return a[u * n3 + l * n2 + d * n + r]; };
  if (tid < n2) {
    const int x = tid / n, y = tid % n;
    double c1 = 0, c2 = 0, c3 = 0, c4 = 0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        const double w = e[p] * e[q];
        c1 += A(p, q, x, y) * w;   // C1[d=x, r=y], u=p, l=q
        c2 += A(p, x, y, q) * w;   // C2[l=x, d=y], u=p, r=q
        c3 += A(x, y, p, q) * w;   // C3[u=x, l=y], d=p, r=q
        c4 += A(y, p, q, x) * w;   // C4[r=x, u=y], l=p, d=q
      }
    C1[tid] = c1; C2[tid] = c2; C3[tid] = c3; C4[tid] = c4;
  }
  if (tid < n3) {
    const int x = tid / (int)n2, y = (tid / n) % n, z = tid % n;
    double t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    for (int p = 0; p < n; ++p) {
      t1 += A(p, x, y, z) * e[p];  // T1[l=x, d=y, r=z]
      t2 += A(x, y, z, p) * e[p];  // T2[u=x, l=y, d=z]
      t3 += A(y, z, p, x) * e[p];  // T3[r=x, u=y, l=z]
      t4 += A(z, p, x, y) * e[p];  // T4[d=x, r=y, u=z]
    }
    T1[tid] = t1; T2[tid] = t2; T3[tid] = t3; T4[tid] = t4;
  }
}

// Frobenius norms of up to 8 tensors -> out[i]; sets *bad when a norm is
// zero or not finite.  Block (b, t) sums the squares of the elements
// b * 256 + j + m * kNormBlocks * 256 of tensor t; k_norms_final adds the
// kNormBlocks partial sums of a tensor in block order.
__global__ __launch_bounds__(256) void k_norms_part(NormArgs na) {
  __shared__ double sh[4];
  const int t = blockIdx.y;
  const double* x = na.x[t];
  const long n = na.n[t];
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)kNormBlocks * 256)
    acc += x[i] * x[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) na.part[(long)t * kNormBlocks + blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_norms_final(NormArgs na) {
  __shared__ double sh[4];
  const int t = blockIdx.x;
  double acc = threadIdx.x < kNormBlocks ? na.part[(long)t * kNormBlocks + threadIdx.x] : 0.0;
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    const double nr = sqrt(acc);
    na.out[t] = nr;
    if (!(nr > 0.0) || !isfinite(nr)) atomicOr(na.bad, 1);
  }
}

__global__ void k_scale(NormArgs na) {
  const int t = blockIdx.y;
  double* x = na.x[t];
  const long n = na.n[t];
  const double inv = 1.0 / na.out[t];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    x[i] *= inv;
}

// Mean sin^2 of the principal angles between the spans of two orthonormal
// chi-column blocks: the cosines are the singular values of G = Q_old^T Q_new,
// so the mean is 1 - |G|_F^2 / chi.  One block of 256 threads; out[0] is the
// largest value over the count products.
__global__ __launch_bounds__(256) void k_sin2(OverlapArgs oa) {
  __shared__ double sh[4];
  const long n = (long)oa.chi * oa.chi;
  double worst = -1.0;
  for (int b = 0; b < oa.count; ++b) {
    const double* G = oa.G[b];
    double acc = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) acc += G[i] * G[i];
    acc = block_sum(acc, sh);
    worst = fmax(worst, 1.0 - acc / oa.chi);
  }
  if (threadIdx.x == 0) oa.out[0] = worst;
}

// Sign rule: for every column j of the N x k block Y (ld = ld), the dominant
// entry -- the lowest-index entry whose magnitude is within a relative 1e-8
// of the column's largest magnitude -- is made positive; sg[j] = +-1.
// Roundoff-level ties (the ket/bra exchange symmetry of the double layer
// pairs entries of equal magnitude) are thereby resolved by index.
__global__ void k_col_sign(SignArgs sa) {
  const int b = blockIdx.y;
  const double* Y = sa.Y[b];
  double* sg = sa.sg[b];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = blockIdx.x * 4 + wave; j < sa.k; j += gridDim.x * 4) {
    double best = 0.0;
    for (int r = lane; r < sa.N; r += 64) best = fmax(best, fabs(Y[(long)r * sa.ld + j]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) best = fmax(best, __shfl_xor(best, off, 64));
    const double thr = (1.0 - 1e-8) * best;
    int bi = 1 << 30;
    double val = 0.0;
    for (int r = lane; r < sa.N; r += 64) {
      const double v = Y[(long)r * sa.ld + j];
      if (fabs(v) >= thr) { bi = r; val = v; break; }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int oi = __shfl_xor(bi, off, 64);
      const double ov = __shfl_xor(val, off, 64);
      if (oi < bi) { bi = oi; val = ov; }
    }
    if (lane == 0) sg[j] = val < 0.0 ? -1.0 : 1.0;
  }
}

// Projector factors for one bond (blockIdx.y; the k x k elements spread
// over the blocks of x):
//   sinv_i = s_i^-1/2 if s_i > rtol * s_0 else 0    (i < keep)
//   vs  = v diag(sg)            (k x k)   -> recycled X = X vs
//   vsc = v[:, :keep] diag(sg * sinv)     -> P_l = A vsc
//   usc = u[:, :keep] diag(sg * sinv)     -> P_r^T = B^T usc
//   gap = s_keep / s_(keep+1) - 1 (or -1)
__global__ void k_proj_prep(ProjPrepArgs pa) {
  const int b = blockIdx.y;
  const int k = pa.k, keep = pa.keep;
  const double* s = pa.s[b];
  const double* sg = pa.sg[b];
  const double s0 = s[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k * k; i += gridDim.x * blockDim.x) {
    const int r = i / k, c = i % k;
    const double sgc = sg[c];
    if (pa.vs[b]) pa.vs[b][i] = pa.v[b][i] * sgc;
    if (c < keep) {
      const double sc = s[c];
      const double si = (s0 > 0.0 && sc > pa.rtol * s0) ? 1.0 / sqrt(sc) : 0.0;
      pa.vsc[b][r * keep + c] = pa.v[b][i] * sgc * si;
      pa.usc[b][r * keep + c] = pa.u[b][i] * sgc * si;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && pa.gap) {
    double g = -1.0;
    if (keep < k && s[keep] > 0.0) g = s[keep - 1] / s[keep] - 1.0;
    pa.gap[b] = g;
  }
}

// Full-SVD variant: U (N x N row-major), Vt (N x N row-major) from the
// dense SVD, column signs sg of U.  Writes Vs[r][c] = Vt[c][r] sg_c sinv_c
// and Us[r][c] = U[r][c] sg_c sinv_c for c < keep (both N x keep).
__global__ void k_proj_prep_full(const double* U, const double* Vt, const double* s,
                                 const double* sg, int N, int keep, double rtol, double* Us,
                                 double* Vs, double* gap) {
  const double s0 = s[0];
  const long total = (long)N * keep;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int r = (int)(i / keep), c = (int)(i % keep);
    const double sc = s[c];
    const double si = (s0 > 0.0 && sc > rtol * s0) ? 1.0 / sqrt(sc) : 0.0;
    const double f = sg[c] * si;
    Us[i] = U[(long)r * N + c] * f;
    Vs[i] = Vt[(long)c * N + r] * f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && gap) {
    double g = -1.0;
    if (keep < N && s[keep] > 0.0) g = s[keep - 1] / s[keep] - 1.0;
    *gap = g;
  }
}

// Descending order of n singular values: perm[rank] = i, rank = number of
// values larger than s[i] (ties by index), so the order is stable.
__global__ __launch_bounds__(256) void k_rank_desc(const double* __restrict__ s, int n,
                                                   int* __restrict__ perm) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double v = s[i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double w = s[j];
      r += (w > v || (w == v && j < i)) ? 1 : 0;
    }
    perm[r] = i;
  }
}

// Sorted copies of the first m singular triples: s_out[j] = s[perm[j]],
// U_out[:, j] = U[:, perm[j]] (row-major, ld n), Vt_out[j, :] = Vt[perm[j], :].
__global__ __launch_bounds__(256) void k_gather_triples(const double* __restrict__ s,
                                                        const double* __restrict__ U,
                                                        const double* __restrict__ Vt,
                                                        const int* __restrict__ perm, int n, int m,
                                                        double* __restrict__ s_out,
                                                        double* __restrict__ U_out,
                                                        double* __restrict__ Vt_out) {
  const long total = (long)n * m;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const int r = (int)(i / m), j = (int)(i % m);
    const int pj = perm[j];
    U_out[(long)r * n + j] = U[(long)r * n + pj];
    Vt_out[(long)j * n + r] = Vt[(long)pj * n + r];
    if (r == 0) s_out[j] = s[pj];
  }
}

__global__ void k_scale_cols(SignArgs sa) {
  const int b = blockIdx.y;
  double* Y = sa.Y[b];
  const double* sg = sa.sg[b];
  const long total = (long)sa.N * sa.k;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int r = (int)(i / sa.k), c = (int)(i % sa.k);
    Y[(long)r * sa.ld + c] *= sg[c];
  }
}

__global__ void k_identity(double* P, int n, int m) {
  const long total = (long)n * m;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x)
    P[i] = ((i / m) == (i % m)) ? 1.0 : 0.0;
}

// Unit-2-norm spectra of the four corners (values of length x, descending),
// zero-padded to chi; delta = max_i |s_new - s_old|_2.  One block.
__global__ void k_spectra_delta(SpecArgs sp) {
  __shared__ double sh[4];
  __shared__ double dmax;
  if (threadIdx.x == 0) dmax = 0.0;
  __syncthreads();
  for (int c = 0; c < 4; ++c) {
    const double* s = sp.s[c];
    double acc = 0.0;
    for (int i = threadIdx.x; i < sp.x; i += blockDim.x) acc += s[i] * s[i];
    const double nrm = sqrt(block_sum(acc, sh));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    double dd = 0.0;
    for (int i = threadIdx.x; i < sp.chi; i += blockDim.x) {
      const double v = i < sp.x ? s[i] * inv : 0.0;
      const double o = sp.old_spec[c * sp.chi + i];
      dd += (v - o) * (v - o);
      sp.new_spec[c * sp.chi + i] = v;
    }
    dd = block_sum(dd, sh);
    if (threadIdx.x == 0) dmax = fmax(dmax, sqrt(dd));
    __syncthreads();
  }
  if (threadIdx.x == 0) *sp.delta = dmax;
}

// Standard normals from a counter-based generator (SplitMix64 finaliser of
// (seed, index), Box-Muller): used only when the caller gives no start block.
__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_gauss(double* x, long n, uint64_t seed) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const uint64_t h1 = splitmix(seed * 0x100000001B3ull + 2 * (uint64_t)i);
    const uint64_t h2 = splitmix(seed * 0x100000001B3ull + 2 * (uint64_t)i + 1);
    const double u1 = ((h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

// sum_{t,d,e} X[t,d,e] Y[e,d,t] (X, Y of shape x, m, x) into *out.  One block.
__global__ void k_dot_rev(const double* X, const double* Y, int x, int m, double* out) {
  __shared__ double sh[4];
  const long total = (long)x * m * x;
  double acc = 0.0;
  for (long i = threadIdx.x; i < total; i += blockDim.x) {
    const int t = (int)(i / ((long)m * x));
    const int d = (int)((i / x) % m);
    const int e = (int)(i % x);
    acc += X[i] * Y[((long)e * m + d) * x + t];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = acc;
}

// Batched variant over nb leading blocks: out[b] = sum X_b[t,d,e] Y_b'[e,d,t].
__global__ void k_dot_rev_batched(const double* X, long xs, const double* Y, long ys, int x,
                                  int m, double* out) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  const double* Xb = X + b * xs;
  const double* Yb = Y + b * ys;
  const long total = (long)x * m * x;
  double acc = 0.0;
  for (long i = threadIdx.x; i < total; i += blockDim.x) {
    const int t = (int)(i / ((long)m * x));
    const int d = (int)((i / x) % m);
    const int e = (int)(i % x);
    acc += Xb[i] * Yb[((long)e * m + d) * x + t];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[b] = acc;
}

__global__ void k_trace(const double* A, int n, double* out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += A[(long)i * n + i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = acc;
}

// sum_i X[i] * Y[perm(i)] for X of shape (x, m, x) and Y[t,m?]: general
// elementwise dot of equal-layout arrays.
__global__ void k_dot(const double* X, const double* Y, long n, double* out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) acc += X[i] * Y[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = acc;
}

// out[i * nj + j] = sum_idx X_i[idx] Y_j[idx'] over arrays of shape (x, m, x);
// idx' = idx (rev == 0) or the reversed index (t,d,e) -> (e,d,t) (rev == 1).
__global__ void k_pair_dot(const double* X, const double* Y, long stride, int nj, int x, int m,
                           int rev, double* out) {
  __shared__ double sh[4];
  const int i = blockIdx.x / nj, j = blockIdx.x % nj;
  const double* Xi = X + i * stride;
  const double* Yj = Y + j * stride;
  const long total = (long)x * m * x;
  double acc = 0.0;
  for (long q = threadIdx.x; q < total; q += blockDim.x) {
    long r = q;
    if (rev) {
      const int t = (int)(q / ((long)m * x));
      const int d = (int)((q / x) % m);
      const int e = (int)(q % x);
      r = ((long)e * m + d) * x + t;
    }
    acc += Xi[q] * Yj[r];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// Partial sums of <X, Y_j> for up to kMaxDots vectors Y_j of n doubles: each
// block writes one partial per j; k_dots_final adds them in block order.
struct DotPtrs {
  const double* y[kMaxDots];
};

__global__ __launch_bounds__(256) void k_dots_part(const double* X, DotPtrs Y, int ny, long n,
                                                   double* part) {
  __shared__ double sh[4];
  double acc[kMaxDots];
#pragma unroll
  for (int j = 0; j < kMaxDots; ++j) acc[j] = 0.0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const double xv = X[e];
#pragma unroll
    for (int j = 0; j < kMaxDots; ++j)
      if (j < ny) acc[j] += xv * Y.y[j][e];
  }
  for (int j = 0; j < ny; ++j) {
    const double t = block_sum(acc[j], sh);
    if (threadIdx.x == 0) part[(long)j * gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void k_dots_final(const double* part, int nb, double* out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[(long)blockIdx.x * nb + b];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// dst (cols x rows) = src (rows x cols)^T
__global__ void k_transpose(const double* src, double* dst, long rows, long cols) {
  const long total = rows * cols;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const long r = i / cols, c = i % cols;
    dst[c * rows + r] = src[i];
  }
}

// Correlation length from the m x m Rayleigh-Ritz matrix H of a transfer
// matrix (m <= kMaxSmallEig, row-major): out[0] = -1 / ln(|l2| / |l1|),
// out[1] = |l2| / |l1|, out[2] = l1 (0, 0, l1 when l2 = 0).  One thread.
// Normalised repeated squaring of H converges to a multiple of the spectral
// projector r l^T of the dominant eigenvalue l1 (simple and alone on its
// circle for a gapped transfer matrix); l1 = l^T H r / l^T r.  |l2| is the
// spectral radius of H - l1 r l^T / (l^T r), from the norms of its powers
// 2^j (the logarithms of the normalisations, weighted 2^-j): this needs no
// separation between |l2| and |l3| and covers complex pairs.
__device__ void sq_norm(double (*B)[kMaxSmallEig], double (*T)[kMaxSmallEig], int m, double* nb) {
  double mx = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double acc = 0.0;
      for (int q = 0; q < m; ++q) acc += B[i][q] * B[q][j];
      T[i][j] = acc;
      mx = fmax(mx, fabs(acc));
    }
  *nb = mx;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) B[i][j] = mx > 0.0 ? T[i][j] / mx : 0.0;
}

__global__ void k_xi_from_ritz(const double* Hin, int m, int squarings, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double H[kMaxSmallEig][kMaxSmallEig], B[kMaxSmallEig][kMaxSmallEig], T[kMaxSmallEig][kMaxSmallEig];
  double mx = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      H[i][j] = Hin[i * m + j];
      mx = fmax(mx, fabs(H[i][j]));
    }
  out[0] = out[1] = out[2] = 0.0;
  if (mx == 0.0) return;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) B[i][j] = H[i][j] / mx;
  double nb = 1.0;
  for (int it = 0; it < squarings && nb > 0.0; ++it) sq_norm(B, T, m, &nb);
  if (nb == 0.0) return;
  // r: the column of largest norm, l: the row of largest norm
  int ci = 0, ri = 0;
  double bc = -1.0, br = -1.0;
  for (int q = 0; q < m; ++q) {
    double c2 = 0.0, r2 = 0.0;
    for (int p = 0; p < m; ++p) {
      c2 += B[p][q] * B[p][q];
      r2 += B[q][p] * B[q][p];
    }
    if (c2 > bc) { bc = c2; ci = q; }
    if (r2 > br) { br = r2; ri = q; }
  }
  double r[kMaxSmallEig], l[kMaxSmallEig];
  for (int p = 0; p < m; ++p) {
    r[p] = B[p][ci];
    l[p] = B[ri][p];
  }
  double lr = 0.0, lhr = 0.0;
  for (int p = 0; p < m; ++p) {
    lr += l[p] * r[p];
    double hr = 0.0;
    for (int q = 0; q < m; ++q) hr += H[p][q] * r[q];
    lhr += l[p] * hr;
  }
  if (lr == 0.0) return;
  const double l1 = lhr / lr;
  out[2] = l1;
  double c0 = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      B[i][j] = H[i][j] - l1 * r[i] * l[j] / lr;
      c0 = fmax(c0, fabs(B[i][j]));
    }
  if (c0 == 0.0 || l1 == 0.0) return;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) B[i][j] /= c0;
  double logr = log(c0), w = 1.0;
  for (int it = 0; it < squarings; ++it) {
    sq_norm(B, T, m, &nb);
    if (nb == 0.0) return;                 // nilpotent remainder: l2 = 0
    w *= 0.5;
    logr += w * log(nb);
  }
  const double rat = exp(logr) / fabs(l1);
  out[1] = rat;
  out[0] = (rat > 0.0 && rat < 1.0) ? -1.0 / log(rat) : 0.0;
}

// vals = [Z11, Z00, Z10, Z01] -> out = Z11 Z00 / (Z10 Z01)
__global__ void k_kappa(const double* z, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = z[0] * z[1] / (z[2] * z[3]);
}

// <op> = sum_{s1 t1 s2 t2} op[(t1 t2),(s1 s2)] E[(s1 t1),(s2 t2)] / sum_{s1 s2} E[(s1 s1),(s2 s2)]
__global__ void k_bond_value(const double* E, const double* op, int d, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int d2 = d * d;
  double num = 0.0, den = 0.0;
  for (int s1 = 0; s1 < d; ++s1)
    for (int t1 = 0; t1 < d; ++t1)
      for (int s2 = 0; s2 < d; ++s2)
        for (int t2 = 0; t2 < d; ++t2) {
          const double e = E[(s1 * d + t1) * d2 + (s2 * d + t2)];
          num += op[(t1 * d + t2) * d2 + (s1 * d + s2)] * e;
          if (s1 == t1 && s2 == t2) den += e;
        }
  out[0] = num / den;
}

__global__ void k_ratio(const double* a, const double* b, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = a[0] / b[0];
}

// x[0] = 0 (a kernel, so that it can be captured into a graph)
__global__ void k_zero_int(int* x) {
  if (threadIdx.x == 0) x[0] = 0;
}

// ---------------------------------------------------------------------------
// C4v helpers
// ---------------------------------------------------------------------------
// A <- (A + A^T) / 2 for a square row-major n x n matrix, one thread per pair.
__global__ void k_symmetrize(double* A, int n) {
  const long total = (long)n * n;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int r = (int)(i / n), c = (int)(i % n);
    if (c < r) continue;
    const double v = 0.5 * (A[(long)r * n + c] + A[(long)c * n + r]);
    A[(long)r * n + c] = v;
    A[(long)c * n + r] = v;
  }
}

// T[a, m, b] <- (T[a, m, b] + T[b, m, a]) / 2 for an x x Dl x x edge tensor.
__global__ void k_symmetrize_edge(double* T, int x, int Dl) {
  const long total = (long)x * Dl * x;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int a = (int)(i / ((long)Dl * x)), m = (int)((i / x) % Dl), b = (int)(i % x);
    if (b < a) continue;
    const long p = ((long)a * Dl + m) * x + b, q = ((long)b * Dl + m) * x + a;
    const double v = 0.5 * (T[p] + T[q]);
    T[p] = v;
    T[q] = v;
  }
}

// P (n x keep, row-major) = eigenvectors of the keep eigenvalues of largest
// |w|, in descending |w| with ties by index; V holds the eigenvectors as
// columns of a column-major n x n matrix (rocSOLVER's layout).  One block.
__global__ void k_c4v_order(const double* w, const double* V, int n, int keep, double* P) {
  extern __shared__ int order[];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double aj = fabs(w[j]);
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      const double ao = fabs(w[o]);
      rank += (ao > aj) || (ao == aj && o < j);
    }
    order[rank] = j;
  }
  __syncthreads();
  for (long i = threadIdx.x; i < (long)n * keep; i += blockDim.x) {
    const int r = (int)(i / keep), c = (int)(i % keep);
    P[i] = V[(long)order[c] * n + r];
  }
}

// P[r, c] = X[r, c] for c < keep (X has leading dimension ld).
__global__ void k_copy_cols(const double* X, int n, long ld, int keep, double* P) {
  const long total = (long)n * keep;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int r = (int)(i / keep), c = (int)(i % keep);
    P[i] = X[(long)r * ld + c];
  }
}

}  // namespace

int elem_pair_dot(const double* X, const double* Y, long stride, int ni, int nj, int x, int m,
                  int rev, double* out, hipStream_t s) {
  k_pair_dot<<<ni * nj, 256, 0, s>>>(X, Y, stride, nj, x, m, rev, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_dots(const double* X, const double* const* Y, int ny, long n, double* part,
              double* out, hipStream_t s) {
  if (ny < 1 || ny > kMaxDots || n < 0) return 1;
  DotPtrs p{};
  for (int j = 0; j < ny; ++j) p.y[j] = Y[j];
  k_dots_part<<<kDotBlocks, 256, 0, s>>>(X, p, ny, n, part);
  CTM_HIP_TRY(hipGetLastError());
  k_dots_final<<<ny, 256, 0, s>>>(part, kDotBlocks, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_transpose(const double* src, double* dst, long rows, long cols, hipStream_t s) {
  const long total = rows * cols;
  if (total <= 0) return 0;
  k_transpose<<<(int)std::min<long>(4096, (total + 255) / 256), 256, 0, s>>>(src, dst, rows, cols);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_xi_from_ritz(const double* H, int m, int squarings, double* out, hipStream_t s) {
  if (m < 1 || m > kMaxSmallEig || squarings < 1) return 1;
  k_xi_from_ritz<<<1, 64, 0, s>>>(H, m, squarings, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_kappa(const double* z, double* out, hipStream_t s) {
  k_kappa<<<1, 64, 0, s>>>(z, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_bond_value(const double* E, const double* op, int d, double* out, hipStream_t s) {
  k_bond_value<<<1, 64, 0, s>>>(E, op, d, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_ratio(const double* a, const double* b, double* out, hipStream_t s) {
  k_ratio<<<1, 64, 0, s>>>(a, b, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_double_layer(const double* A, const double* O, double* a, int d, int D, hipStream_t s,
                      int s_fix, int t_fix) {
  const long total = (long)D * D * D * D * D * D * D * D;
  const int blocks = (int)std::min<long>(4096, (total + 255) / 256);
  k_double_layer<<<blocks, 256, 0, s>>>(A, O, a, d, D, s_fix, t_fix);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_permute4(const double* src, void* dst, DT t, int n, long s0, long s1, long s2, long s3,
                  hipStream_t s) {
  const long total = (long)n * n * n * n;
  const int blocks = (int)std::min<long>(4096, (total + 255) / 256);
  if (t == DT::F64) k_permute4<double><<<blocks, 256, 0, s>>>(src, (double*)dst, n, s0, s1, s2, s3);
  else if (t == DT::F32) k_permute4<float><<<blocks, 256, 0, s>>>(src, (float*)dst, n, s0, s1, s2, s3);
  else k_permute4<__bf16><<<blocks, 256, 0, s>>>(src, (__bf16*)dst, n, s0, s1, s2, s3);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_init_env(const double* a, const double* e, int n, double* const* C, double* const* T,
                  hipStream_t s) {
  const long n3 = (long)n * n * n;
  const int blocks = (int)((n3 + 255) / 256);
  k_init_env<<<blocks, 256, 0, s>>>(a, e, n, C[0], C[1], C[2], C[3], T[0], T[1], T[2], T[3]);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

static int launch_norms(const NormArgs& na, int count, hipStream_t s) {
  if (count < 1 || count > 8 || na.part == nullptr) {
    set_thread_error("norms: need 1 to 8 tensors and a partial-sum workspace");
    return 1;
  }
  k_norms_part<<<dim3(kNormBlocks, count), 256, 0, s>>>(na);
  CTM_HIP_TRY(hipGetLastError());
  k_norms_final<<<count, 256, 0, s>>>(na);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_normalize(const NormArgs& na, int count, hipStream_t s) {
  if (launch_norms(na, count, s)) return 1;
  long mx = 0;
  for (int i = 0; i < count; ++i) mx = std::max(mx, na.n[i]);
  const int blocks = (int)std::min<long>(1024, (mx + 255) / 256);
  k_scale<<<dim3(blocks, count), 256, 0, s>>>(na);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_norms(const NormArgs& na, int count, hipStream_t s) { return launch_norms(na, count, s); }

int elem_sin2(const OverlapArgs& oa, hipStream_t s) {
  if (oa.count < 1 || oa.count > 8 || oa.chi < 1) return 1;
  k_sin2<<<1, 256, 0, s>>>(oa);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_col_sign(const SignArgs& sa, int count, hipStream_t s) {
  const int blocks = std::max(1, std::min(64, (sa.k + 3) / 4));
  k_col_sign<<<dim3(blocks, count), 256, 0, s>>>(sa);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_scale_cols(const SignArgs& sa, int count, hipStream_t s) {
  const long total = (long)sa.N * sa.k;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  k_scale_cols<<<dim3(blocks, count), 256, 0, s>>>(sa);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_proj_prep(const ProjPrepArgs& pa, int count, hipStream_t s) {
  const int blocks = std::max(1, std::min(64, (pa.k * pa.k + 255) / 256));
  k_proj_prep<<<dim3(blocks, count), 256, 0, s>>>(pa);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_proj_prep_full(const double* U, const double* Vt, const double* sv, const double* sg,
                        int N, int keep, double rtol, double* Us, double* Vs, double* gap,
                        hipStream_t s) {
  const long total = (long)N * keep;
  const int blocks = (int)std::min<long>(2048, (total + 255) / 256);
  k_proj_prep_full<<<blocks, 256, 0, s>>>(U, Vt, sv, sg, N, keep, rtol, Us, Vs, gap);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_sort_triples(const double* s, const double* U, const double* Vt, int n, int m, int* perm,
                      double* s_out, double* U_out, double* Vt_out, hipStream_t st) {
  if (n < 1 || m < 1 || m > n) return 1;
  k_rank_desc<<<(n + 255) / 256, 256, 0, st>>>(s, n, perm);
  CTM_HIP_TRY(hipGetLastError());
  const long total = (long)n * m;
  k_gather_triples<<<(int)std::min<long>(4096, (total + 255) / 256), 256, 0, st>>>(
      s, U, Vt, perm, n, m, s_out, U_out, Vt_out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_zero_int(int* x, hipStream_t s) {
  k_zero_int<<<1, 64, 0, s>>>(x);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_symmetrize(double* A, int n, hipStream_t s) {
  const long total = (long)n * n;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  k_symmetrize<<<blocks, 256, 0, s>>>(A, n);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_symmetrize_edge(double* T, int x, int Dl, hipStream_t s) {
  const long total = (long)x * Dl * x;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  k_symmetrize_edge<<<blocks, 256, 0, s>>>(T, x, Dl);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_c4v_order(const double* w, const double* V, int n, int keep, double* P, hipStream_t s) {
  k_c4v_order<<<1, 256, n * sizeof(int), s>>>(w, V, n, keep, P);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_copy_cols(const double* X, int n, long ld, int keep, double* P, hipStream_t s) {
  const long total = (long)n * keep;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  k_copy_cols<<<blocks, 256, 0, s>>>(X, n, ld, keep, P);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_identity(double* P, int n, int m, hipStream_t s) {
  const long total = (long)n * m;
  const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
  k_identity<<<blocks, 256, 0, s>>>(P, n, m);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_spectra_delta(const SpecArgs& sp, hipStream_t s) {
  k_spectra_delta<<<1, 256, 0, s>>>(sp);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_gauss(double* x, long n, uint64_t seed, hipStream_t s) {
  const int blocks = (int)std::min<long>(2048, (n + 255) / 256);
  k_gauss<<<blocks, 256, 0, s>>>(x, n, seed);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_dot_rev(const double* X, const double* Y, int x, int m, double* out, hipStream_t s) {
  k_dot_rev<<<1, 256, 0, s>>>(X, Y, x, m, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_dot_rev_batched(const double* X, long xs, const double* Y, long ys, int nb, int x, int m,
                         double* out, hipStream_t s) {
  k_dot_rev_batched<<<nb, 256, 0, s>>>(X, xs, Y, ys, x, m, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_trace(const double* A, int n, double* out, hipStream_t s) {
  k_trace<<<1, 256, 0, s>>>(A, n, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int elem_dot(const double* X, const double* Y, long n, double* out, hipStream_t s) {
  k_dot<<<1, 256, 0, s>>>(X, Y, n, out);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace sictm
