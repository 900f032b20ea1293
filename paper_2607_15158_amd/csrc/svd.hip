// SVD of the small (chi+p) x (chi+p) reduced matrix rho = Y M X (QR-based
// projector section, step 2), and of the chi x chi corners for the
// convergence measure.
//
// One-sided (Hestenes) Jacobi: U <- X V with V accumulating plane rotations
// until all column pairs of U are orthogonal to working precision; then
// s_j = |u_j|, u_j <- u_j / s_j.  One-sided Jacobi computes small singular
// values to high relative accuracy, which matters here because the
// pseudo-inverse s^-1/2 keeps directions down to a relative 1e-12.
// Preconditioning (Drmac & Veselic): the columns of A are sorted by norm
// (permutation P), A P = Q R by the Householder QR of this library, and the
// Jacobi iteration runs on X = R^T, which converges in a few sweeps where A
// itself needs dozens: R^T = Ut S V'^T gives A = (Q V') S (P Ut)^T.
//
// Block-pair parallel ordering: the columns are cut into blocks of kBlk; an
// outer sweep pairs the blocks in a round-robin tournament, one launch per
// round, one workgroup per block pair and matrix.  The workgroup loads the
// 2 kBlk columns of U into LDS and rotates the pairs across the two blocks
// in kBlk inner steps of kBlk disjoint pairs (in the sweep's first round,
// where every block is visited once, the pairs within each block first, in
// kBlk - 1 more steps), so that every column pair meets once per sweep;
// 16 lanes per pair (rows spread over the lanes, dot products reduced by
// DPP row sums); the
// rotations of the visit are accumulated in a 2 kBlk x 2 kBlk matrix W and
// applied to the right vectors once at the end (V_cols <- V_cols W).
// A per-matrix flag records
// whether a sweep rotated anything, and later launches return at once after
// a sweep without rotations.  Columns that end numerically zero
// (rank-deficient input) are replaced by an orthonormal completion so that
// u stays orthogonal.  Singular values are returned in descending order (ties by
// index).

#include "common.h"

#include <hip/hip_cooperative_groups.h>

namespace sictm {
namespace {

constexpr int kSvdMaxN = 192;   // the preconditioning QR holds n <= 192 rows per leaf
constexpr int kRPL = kSvdMaxN / 64;   // rows per lane in the finalisation
constexpr int kCompChunk = 32;       // non-zero columns staged per LDS pass of the completion
constexpr int kBlk = 16;              // columns per block
constexpr int kMaxSweeps = 24;
constexpr int kInner = 1;            // inner sweeps per block-pair visit
constexpr int kLanesPerPair = 16;

__device__ __forceinline__ double wsum(double x) { return wave_sum64(x); }

__device__ __forceinline__ double gsum16(double x) { return row_sum16(x); }

struct SvdArgs {
  const double* A[kMaxProb];   // matrices the Jacobi kernels act on (R^T)
  double* U[kMaxProb];         // Jacobi outputs: left vectors of R^T (Ut) ...
  double* S[kMaxProb];
  double* V[kMaxProb];         // ... and right vectors (V')
  double* work;       // [count][2][n][n] column-major working columns
  int* flags;         // [count][kMaxSweeps] "a rotation happened in sweep s"
  int n, nblk, want_v;
  // preconditioning
  const double* Ain[kMaxProb]; // the caller's matrices
  double* Wp[kMaxProb];        // A P, then Q
  double* Wc[kMaxProb];        // A P
  double* Ut[kMaxProb];        // left vectors of R^T
  int* perm;                   // [count][n]
  double* fro2;                // [count] squared Frobenius norm of each input
};

// Tournament position -> block / column index (position 0 fixed).
__device__ __forceinline__ int tour(int pos, int round, int m) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (m - 1)) + 1;
}

__global__ void svd_init(SvdArgs a) {
  const int mat = blockIdx.y;
  const int n = a.n;
  double* Uc = a.work + (size_t)mat * 2 * n * n;
  double* Vc = Uc + (size_t)n * n;
  const double* A = a.A[mat];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += gridDim.x * blockDim.x) {
    const int r = i / n, c = i % n;
    Uc[(size_t)c * n + r] = A[i];
    if (a.want_v) Vc[(size_t)c * n + r] = (r == c) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kMaxSweeps; i += blockDim.x) a.flags[mat * kMaxSweeps + i] = 0;
}

// Column norms, stable descending sort -> perm (the copy Wp = Wc = A[:, perm]
// follows in svd_prep_copy).  Thread c sums column c down the rows, so
// that each row is read by consecutive threads.
__global__ __launch_bounds__(256) void svd_prep(SvdArgs a) {
  __shared__ double nrm[kSvdMaxN];
  __shared__ int perm[kSvdMaxN];
  const int mat = blockIdx.x, n = a.n, tid = threadIdx.x;
  const double* A = a.Ain[mat];
  for (int c = tid; c < n; c += 256) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int r = 0;
    for (; r + 3 < n; r += 4) {
      const double x0 = A[(size_t)r * n + c], x1 = A[(size_t)(r + 1) * n + c];
      const double x2 = A[(size_t)(r + 2) * n + c], x3 = A[(size_t)(r + 3) * n + c];
      s0 += x0 * x0;
      s1 += x1 * x1;
      s2 += x2 * x2;
      s3 += x3 * x3;
    }
    for (; r < n; ++r) s0 += A[(size_t)r * n + c] * A[(size_t)r * n + c];
    nrm[c] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    for (int c = 0; c < n; ++c) f += nrm[c];
    a.fro2[mat] = f;
  }
  for (int c = tid; c < n; c += 256) {
    int rank = 0;
    for (int o = 0; o < n; ++o) rank += (nrm[o] > nrm[c]) || (nrm[o] == nrm[c] && o < c);
    perm[rank] = c;
  }
  __syncthreads();
  int* pg = a.perm + (size_t)mat * n;
  for (int c = tid; c < n; c += 256) pg[c] = perm[c];
}

// Wp = Wc = A[:, perm], over the blocks of x (matrix blockIdx.y).
__global__ __launch_bounds__(256) void svd_prep_copy(SvdArgs a) {
  const int mat = blockIdx.y, n = a.n;
  const double* A = a.Ain[mat];
  const int* pg = a.perm + (size_t)mat * n;
  double* Wp = a.Wp[mat];
  double* Wc = a.Wc[mat];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n * n; i += gridDim.x * 256) {
    const int r = i / n, j = i % n;
    const double v = A[(size_t)r * n + pg[j]];
    Wp[i] = v;
    Wc[i] = v;
  }
}

// v[perm[i], :] = Ut[i, :]
__global__ void svd_unpermute_rows(SvdArgs a) {
  const int mat = blockIdx.y, n = a.n;
  const int* pg = a.perm + (size_t)mat * n;
  const double* Ut = a.Ut[mat];
  double* V = a.V[mat];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += gridDim.x * blockDim.x) {
    const int r = i / n, c = i % n;
    V[(size_t)pg[r] * n + c] = Ut[i];
  }
}

// 1/sqrt(x) and 1/x to full double precision from the hardware estimates
// (Newton steps); used for the rotation angles, where x > 0.
__device__ __forceinline__ double fast_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x * y;
  y = fma(y, fma(-h, y, 0.5), y);
  h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// One round of an outer sweep: block pair (tournament positions bp,
// nblk-1-bp).  The 2 kBlk columns of U live in LDS; the rotations of the
// visit are accumulated in a 2 kBlk x 2 kBlk matrix W (also in LDS) and the
// right vectors are updated once at the end, V_cols <- V_cols W.  RPL is the
// number of rows per lane (n <= 16 RPL).
template <int RPL>
struct RoundLds {
  static constexpr int kC = 2 * kBlk;
  static constexpr int LD = 16 * RPL + 1;   // odd row length: no bank conflicts
  double Ul[kC][LD];
  double Vl[kC][LD];
  double Wl[kC][kC + 1];
  int rot;
};

template <int RPL>
__device__ __forceinline__ void block_round(const SvdArgs& a, int sweep, int round, int inner,
                                            int mat, int bp, RoundLds<RPL>& sh) {
  constexpr int kC = RoundLds<RPL>::kC;
  auto& Ul = sh.Ul;
  auto& Vl = sh.Vl;
  auto& Wl = sh.Wl;
  int& rot = sh.rot;
  const int n = a.n, nblk = a.nblk;
  const int b0 = tour(bp, round, nblk), b1 = tour(nblk - 1 - bp, round, nblk);
  const int tid = threadIdx.x;
  double* Uc = a.work + (size_t)mat * 2 * n * n;
  double* Vc = Uc + (size_t)n * n;
  // local column j -> global column: j < kBlk from b0, else from b1
  auto gcol = [&](int j) { return (j < kBlk ? b0 : b1) * kBlk + (j % kBlk); };
  // the 2 kBlk columns of U (and of V) into LDS, one column per wave at a
  // time, rows lane + 64 t: coalesced, with no index division; four columns
  // per wave in flight
  const int nv = a.want_v ? 2 : 1;
  const int wv = tid / 64, ln = tid % 64;
  constexpr int kRW = (16 * RPL + 63) / 64;   // row chunks per lane (n <= 16 RPL)
  const int ncol = nv * kC;
  for (int c0 = wv; c0 < ncol; c0 += 16) {
    double t[4][kRW];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = c0 + 4 * u, g = gcol(cc % kC);
      const double* src = (cc < kC ? Uc : Vc) + (size_t)g * n;
#pragma unroll
      for (int r = 0; r < kRW; ++r) {
        const int row = ln + 64 * r;
        t[u][r] = (cc < ncol && g < n && row < n) ? src[row] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = c0 + 4 * u;
      if (cc < ncol) {
        double* dst = cc < kC ? Ul[cc] : Vl[cc - kC];
#pragma unroll
        for (int r = 0; r < kRW; ++r) {
          const int row = ln + 64 * r;
          if (row < n)
            dst[row] = t[u][r];
          else if (row < 16 * RPL)
            dst[row] = 0.0;   // rows n .. 16 RPL - 1 hold exact zeros
        }
      }
    }
  }
  for (int idx = tid; idx < kC * kC; idx += 256) Wl[idx / kC][idx % kC] = (idx / kC == idx % kC);
  if (tid == 0) rot = 0;
  __syncthreads();
  const int grp = tid / kLanesPerPair, li = tid % kLanesPerPair;   // 16 pair groups
  const double tol = 1e-15 * sqrt((double)n);
  // columns below 1e-15 of the matrix norm are numerically zero: rotating
  // them against the others cannot converge in the relative sense and does
  // not change the result above roundoff; they are completed at the end
  const double negl = 1e-30 * a.fro2[mat];
  int my_rot = 0;
  // each step's rotation of W is applied at the start of the next step,
  // beside that step's loads (every W column is still rotated in step
  // order: a column belongs to one pair per step, and only that pair's
  // group touches it until the next barrier)
  int wpp = -1, wqq = 0;
  double wc = 1.0, ws = 0.0;
  auto rotate_w = [&]() {
#pragma unroll
    for (int tt = 0; tt < kC / kLanesPerPair; ++tt) {
      const int row = li + kLanesPerPair * tt;
      const double wp = Wl[row][wpp], wq = Wl[row][wqq];
      Wl[row][wpp] = wc * wp - ws * wq;
      Wl[row][wqq] = ws * wp + wc * wq;
    }
  };
  // the sweep's first round (every block in exactly one pair) also pairs
  // the columns within each block: kBlk - 1 steps of a round-robin per
  // block, kBlk / 2 pairs of each block per step; then kBlk steps pair
  // column i of the first block with column (i + step) mod kBlk of the
  // second, so that a sweep meets every column pair exactly once
  const int nintra = round == 0 ? kBlk - 1 : 0, nstep = nintra + kBlk;
  for (int rr = 0; rr < inner * nstep; ++rr) {
    if (wpp >= 0) {
      rotate_w();
      wpp = -1;
    }
    const int r = rr % nstep;
    int p, q;
    if (r < nintra) {
      const int blk = grp / (kBlk / 2), k = grp % (kBlk / 2);
      const int ca = tour(k, r, kBlk), cb = tour(kBlk - 1 - k, r, kBlk);
      p = blk * kBlk + min(ca, cb);
      q = blk * kBlk + max(ca, cb);
    } else {
      p = grp;
      q = kBlk + (grp + r - nintra) % kBlk;
    }
    const bool live = gcol(p) < n && gcol(q) < n;
    if (live) {
      double up[RPL], uq[RPL];
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        // rows n .. 16 RPL - 1 are zero: no guard
        const int row = li + kLanesPerPair * t;
        up[t] = Ul[p][row];
        uq[t] = Ul[q][row];
        al += up[t] * up[t];
        be += uq[t] * uq[t];
        ga += up[t] * uq[t];
      }
      al = gsum16(al);
      be = gsum16(be);
      ga = gsum16(ga);
      const double thr = tol * sqrt(al) * sqrt(be);
      if (ga != 0.0 && fabs(ga) > thr && al > negl && be > negl) {
        // tan of the rotation angle, the smaller root of t^2 + 2 zeta t = 1
        const double zeta = (be - al) * fast_rcp(2.0 * ga);
        const double z2 = 1.0 + zeta * zeta;
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) * fast_rcp(fabs(zeta) + z2 * fast_rsqrt(z2));
        const double c = fast_rsqrt(1.0 + t * t), s = c * t;
        // convergence counts only rotations clearly above roundoff: a pair
        // left at |gamma| ~ tol sqrt(alpha beta) keeps being rotated but does
        // not prevent the sweep loop from stopping
        if (fabs(ga) > 16.0 * thr) ++my_rot;
#pragma unroll
        for (int tt = 0; tt < RPL; ++tt) {
          const int row = li + kLanesPerPair * tt;
          Ul[p][row] = c * up[tt] - s * uq[tt];
          Ul[q][row] = s * up[tt] + c * uq[tt];
        }
        if (a.want_v) {   // W's rotation waits for the next step
          wpp = p;
          wqq = q;
          wc = c;
          ws = s;
        }
      }
    }
    __syncthreads();
  }
  if (wpp >= 0) rotate_w();
  if (a.want_v) __syncthreads();   // W is complete before V_cols <- V_cols W
  if (li == 0 && my_rot) atomicAdd(&rot, my_rot);
  for (int j = wv; j < kC; j += 4) {
    const int g = gcol(j);
    if (g < n) {
#pragma unroll
      for (int r = 0; r < kRW; ++r) {
        const int row = ln + 64 * r;
        if (row < n) Uc[(size_t)g * n + row] = Ul[j][row];
      }
    }
  }
  if (a.want_v) {
    // V_cols <- V_cols W, register-blocked over the whole workgroup: thread
    // (rg, cg) computes rows rg + 32 i of columns kVc cg .. kVc cg + kVc - 1
    // (each sum over l in ascending order from zero, 20 independent chains
    // per thread in place of one 32-long chain per row)
    constexpr int kVr = (16 * RPL + 31) / 32, kVc = kC / 8;
    const int rg = tid % 32, cg = tid / 32;
    double acc[kVr][kVc];
#pragma unroll
    for (int i = 0; i < kVr; ++i)
#pragma unroll
      for (int c = 0; c < kVc; ++c) acc[i][c] = 0.0;
#pragma unroll 4
    for (int l = 0; l < kC; ++l) {
      double w[kVc];
#pragma unroll
      for (int c = 0; c < kVc; ++c) w[c] = Wl[l][kVc * cg + c];
#pragma unroll
      for (int i = 0; i < kVr; ++i) {
        const int r = rg + 32 * i;
        const double v = r < n ? Vl[l][r] : 0.0;
#pragma unroll
        for (int c = 0; c < kVc; ++c) acc[i][c] += v * w[c];
      }
    }
#pragma unroll
    for (int c = 0; c < kVc; ++c) {
      const int g = gcol(kVc * cg + c);
      if (g < n) {
#pragma unroll
        for (int i = 0; i < kVr; ++i) {
          const int r = rg + 32 * i;
          if (r < n) Vc[(size_t)g * n + r] = acc[i][c];
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0 && rot) atomicOr(&a.flags[mat * kMaxSweeps + sweep], 1);
}

// One round per launch; later launches return at once after a sweep
// without rotations.
template <int RPL>
__global__ __launch_bounds__(256) void svd_block_round(SvdArgs a, int sweep, int round, int inner) {
  __shared__ RoundLds<RPL> sh;
  const int mat = blockIdx.y;
  if (sweep > 0 && a.flags[mat * kMaxSweeps + sweep - 1] == 0) return;   // converged
  block_round<RPL>(a, sweep, round, inner, mat, blockIdx.x, sh);
}

// All sweeps in one cooperative launch: a grid-wide barrier separates the
// rounds, matrices whose last sweep rotated nothing stop working, and the
// launch ends when every matrix has converged (a decision every workgroup
// takes from the same flags after the barrier).
template <int RPL>
__global__ __launch_bounds__(256) void svd_sweeps(SvdArgs a, int inner, int count) {
  __shared__ RoundLds<RPL> sh;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int mat = blockIdx.y;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    const bool active = sweep == 0 || a.flags[mat * kMaxSweeps + sweep - 1] != 0;
    for (int round = 0; round < a.nblk - 1; ++round) {
      if (active) block_round<RPL>(a, sweep, round, inner, mat, blockIdx.x, sh);
      grid.sync();
    }
    bool any = false;
    for (int m = 0; m < count; ++m) any |= a.flags[m * kMaxSweeps + sweep] != 0;
    if (!any) break;
  }
}

// Singular values, normalisation, completion of zero columns, ordering.
__global__ __launch_bounds__(1024) void svd_finalize(SvdArgs a) {
  const int mat = blockIdx.x;
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nwaves = 1024 / 64;
  double* Uc = a.work + (size_t)mat * 2 * n * n;
  double* Vc = Uc + (size_t)n * n;
  __shared__ double snorm[kSvdMaxN];
  __shared__ int order[kSvdMaxN];
  // singular values = column norms
  for (int c = wave; c < n; c += nwaves) {
    double ss = 0.0;
    for (int r = lane; r < n; r += 64) ss += Uc[(size_t)c * n + r] * Uc[(size_t)c * n + r];
    ss = wsum(ss);
    if (lane == 0) snorm[c] = sqrt(ss);
  }
  __syncthreads();
  // normalise non-zero columns
  for (int c = wave; c < n; c += nwaves) {
    const double sn = snorm[c];
    if (sn > 0.0)
      for (int r = lane; r < n; r += 64) Uc[(size_t)c * n + r] /= sn;
  }
  __syncthreads();
  // orthonormal completion of numerically zero columns; the cut is the one
  // below which the rotations left a column alone.  The unit vectors are
  // projected on the complement of the non-zero columns at once
  // (X = I - U U^T), and the complement's basis is drawn from X's columns
  // in index order by Gram-Schmidt: the zero columns, in index order, take
  // the unit vectors e_0, e_1, ... that keep enough of their length after
  // the projection on the complement of the non-zero columns and of the
  // zero columns completed before.  Wavefront w keeps columns w, w + 16, ...
  // of X in registers, rows lane, lane + 64, lane + 128.
  const double zero_cut = 1e-15 * sqrt(a.fro2[mat]);
  if (a.U[mat] != nullptr) {
    __shared__ int nzl[kSvdMaxN], zl[kSvdMaxN];
    __shared__ int cnt[2];
    __shared__ double qs[kSvdMaxN];
    __shared__ int took[2];
    __shared__ double ust[kCompChunk][kSvdMaxN];
    if (wave == 0) {
      int nr = 0, nz = 0;
      for (int base = 0; base < n; base += 64) {
        const int c = base + lane;
        const bool in = c < n;
        const bool live = in && snorm[c] > zero_cut;
        const unsigned long long ml = __ballot(live), mz = __ballot(in && !live);
        const unsigned long long below = (1ull << lane) - 1ull;
        if (live) nzl[nr + __popcll(ml & below)] = c;
        else if (in) zl[nz + __popcll(mz & below)] = c;
        nr += __popcll(ml);
        nz += __popcll(mz);
      }
      if (lane == 0) {
        cnt[0] = nr;
        cnt[1] = nz;
      }
    }
    __syncthreads();
    const int nr = cnt[0], nz = cnt[1];
    if (nz > 0) {
      constexpr int CPW = kSvdMaxN / nwaves;   // columns per wavefront
      double x[CPW][kRPL];
#pragma unroll
      for (int q = 0; q < CPW; ++q)
#pragma unroll
        for (int e = 0; e < kRPL; ++e) {
          const int j = wave + nwaves * q, i = lane + 64 * e;
          x[q][e] = (i == j && j < n) ? 1.0 : 0.0;
        }
      // X -= U_nz U_nz^T, kCompChunk non-zero columns staged in LDS at a time
      for (int o0 = 0; o0 < nr; o0 += kCompChunk) {
        const int m = min(kCompChunk, nr - o0);
        for (int t = tid; t < m * n; t += 1024) {
          const int oo = t / n, i = t % n;
          ust[oo][i] = Uc[(size_t)nzl[o0 + oo] * n + i];
        }
        __syncthreads();
        for (int oo = 0; oo < m; ++oo) {
          double ui[kRPL];
#pragma unroll
          for (int e = 0; e < kRPL; ++e) {
            const int i = lane + 64 * e;
            ui[e] = i < n ? ust[oo][i] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < CPW; ++q) {
            const int j = wave + nwaves * q;
            const double uj = j < n ? ust[oo][j] : 0.0;
#pragma unroll
            for (int e = 0; e < kRPL; ++e) x[q][e] -= uj * ui[e];
          }
        }
        __syncthreads();
      }
      // candidates in index order: a column of X that keeps more than
      // 1/(2 sqrt(n)) of its length (some column of the complement's
      // projector always does) becomes the next zero column and is removed
      // from the later candidates
      const double keep_min = 0.5 / sqrt((double)n);
      int t = 0;
      for (int cand = 0; cand < n && t < nz; ++cand) {
        if (wave == cand % nwaves) {
          const int qc = cand / nwaves;
          double xc[kRPL] = {};
#pragma unroll
          for (int q = 0; q < CPW; ++q)
            if (q == qc)
#pragma unroll
              for (int e = 0; e < kRPL; ++e) xc[e] = x[q][e];
          double ss = 0.0;
#pragma unroll
          for (int e = 0; e < kRPL; ++e) ss += xc[e] * xc[e];
          const double nn = sqrt(wsum(ss));
          const bool take = nn > keep_min;
          if (take) {
            const double inv = 1.0 / nn;
            const int c = zl[t];
#pragma unroll
            for (int e = 0; e < kRPL; ++e) {
              const int i = lane + 64 * e;
              if (i < n) {
                qs[i] = xc[e] * inv;
                Uc[(size_t)c * n + i] = xc[e] * inv;
              }
            }
          }
          if (lane == 0) took[cand & 1] = take ? 1 : 0;
        }
        __syncthreads();
        if (!took[cand & 1]) continue;
        ++t;
        if (t == nz) break;
        double qv[kRPL];
#pragma unroll
        for (int e = 0; e < kRPL; ++e) {
          const int i = lane + 64 * e;
          qv[e] = i < n ? qs[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
          const int j = wave + nwaves * q;
          if (j <= cand || j >= n) continue;
          double d = 0.0;
#pragma unroll
          for (int e = 0; e < kRPL; ++e) d += qv[e] * x[q][e];
          d = wsum(d);
#pragma unroll
          for (int e = 0; e < kRPL; ++e) x[q][e] -= d * qv[e];
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // descending order, ties by index
  for (int c = tid; c < n; c += 1024) {
    const double sc = snorm[c];
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      const double so = snorm[o];
      rank += (so > sc) || (so == sc && o < c);
    }
    order[rank] = c;
  }
  __syncthreads();
  double* S = a.S[mat];
  double* U = a.U[mat];
  double* V = a.V[mat];
  for (int i = tid; i < n; i += 1024) S[i] = snorm[order[i]];
  for (int i = tid; i < n * n; i += 1024) {
    const int r = i / n, j = i % n;
    const int c = order[j];
    if (U) U[i] = Uc[(size_t)c * n + r];
    if (V) V[i] = Vc[(size_t)c * n + r];
  }
}

}  // namespace

size_t svd_workspace_bytes(int count, int n) {
  const size_t nn = (size_t)n * n;
  return (size_t)count * (2 * nn + 5 * nn) * sizeof(double) +
         (size_t)count * (kMaxSweeps + n) * sizeof(int) + (size_t)count * sizeof(double) +
         qr_workspace_bytes(count, n, n) + 4096;
}

int launch_svd(int count, const double* const* A, double* const* U, double* const* S,
               double* const* V, int n, void* ws, hipStream_t s) {
  if (count <= 0 || n <= 0) return 0;
  if (count > kMaxProb || n > kSvdMaxN) {
    set_thread_error("launch_svd: n <= 192 and at most 8 matrices per launch");
    return 1;
  }
  const size_t nn = (size_t)n * n;
  double* base = (double*)ws;
  SvdArgs a{};
  a.n = n;
  a.work = base;                                   // 2 nn per matrix
  double* wp = a.work + (size_t)count * 2 * nn;    // A P -> Q
  double* wc = wp + (size_t)count * nn;            // A P
  double* rt = wc + (size_t)count * nn;            // R^T
  double* ut = rt + (size_t)count * nn;            // left vectors of R^T
  double* vp = ut + (size_t)count * nn;            // right vectors of R^T
  a.flags = (int*)(vp + (size_t)count * nn);
  a.perm = a.flags + (size_t)count * kMaxSweeps;
  a.fro2 = (double*)(((uintptr_t)(a.perm + (size_t)count * n) + 7) & ~(uintptr_t)7);
  char* qws = (char*)(a.fro2 + count);
  qws = (char*)(((uintptr_t)qws + 255) & ~(uintptr_t)255);
  int nblk = (n + kBlk - 1) / kBlk;
  nblk += nblk & 1;
  if (nblk < 2) nblk = 2;
  a.nblk = nblk;
  const bool want_u = U != nullptr, want_vout = V != nullptr;
  a.want_v = want_u ? 1 : 0;                       // V' is needed for u = Q V'
  double* qptr[kMaxProb];
  for (int i = 0; i < count; ++i) {
    a.Ain[i] = A[i];
    a.Wp[i] = wp + i * nn;
    a.Wc[i] = wc + i * nn;
    a.A[i] = rt + i * nn;
    a.Ut[i] = ut + i * nn;
    a.U[i] = want_vout ? a.Ut[i] : nullptr;
    a.S[i] = S[i];
    a.V[i] = want_u ? vp + i * nn : nullptr;
    qptr[i] = a.Wp[i];
  }
  svd_prep<<<count, 256, 0, s>>>(a);
  CTM_HIP_TRY(hipGetLastError());
  svd_prep_copy<<<dim3(std::max(1, std::min(64, n * n / 256)), count), 256, 0, s>>>(a);
  CTM_HIP_TRY(hipGetLastError());
  int r = launch_qr(count, qptr, n, n, qws, s);
  if (r) return r;
  // R^T = (A P)^T Q
  GemmBatch g{};
  g.count = count;
  g.M = g.N = g.K = n;
  g.lda = g.ldb = n;
  gemm_set_rowmajor_c(g, n);
  g.nbatch = 1;
  g.alpha = 1.0;
  for (int i = 0; i < count; ++i) {
    g.A[i] = a.Wc[i];
    g.transA[i] = 1;
    g.B[i] = a.Wp[i];
    g.C[i] = rt + i * nn;
  }
  r = launch_gemm(g, DT::F64, DT::F64, DT::F64, s);
  if (r) return r;
  svd_init<<<dim3(std::max(1, std::min(64, n * n / 256)), count), 256, 0, s>>>(a);
  const int rpl = (n + kLanesPerPair - 1) / kLanesPerPair;
  {
    const dim3 grid(nblk / 2, count);
    int inner = kInner, cnt = count;
    void* args[] = {&a, &inner, &cnt};
    const void* fn = rpl <= 4    ? (const void*)svd_sweeps<4>
                     : rpl <= 8  ? (const void*)svd_sweeps<8>
                     : rpl <= 10 ? (const void*)svd_sweeps<10>
                                 : (const void*)svd_sweeps<12>;
    // inside a stream capture (graph) the per-round launches are used
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    if (cs == hipStreamCaptureStatusNone &&
        hipLaunchCooperativeKernel(fn, grid, dim3(256), args, 0, s) == hipSuccess)
      goto sweeps_done;
    (void)hipGetLastError();
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep)
      for (int round = 0; round < nblk - 1; ++round) {
        if (rpl <= 4)
          svd_block_round<4><<<grid, 256, 0, s>>>(a, sweep, round, kInner);
        else if (rpl <= 8)
          svd_block_round<8><<<grid, 256, 0, s>>>(a, sweep, round, kInner);
        else if (rpl <= 10)
          svd_block_round<10><<<grid, 256, 0, s>>>(a, sweep, round, kInner);
        else
          svd_block_round<12><<<grid, 256, 0, s>>>(a, sweep, round, kInner);
      }
  }
sweeps_done:
  svd_finalize<<<count, 1024, 0, s>>>(a);
  CTM_HIP_TRY(hipGetLastError());
  if (want_u) {   // u = Q V'
    for (int i = 0; i < count; ++i) {
      g.A[i] = a.Wp[i];
      g.transA[i] = 0;
      g.B[i] = vp + i * nn;
      g.C[i] = U[i];
    }
    r = launch_gemm(g, DT::F64, DT::F64, DT::F64, s);
    if (r) return r;
  }
  if (want_vout) {   // v = P Ut
    for (int i = 0; i < count; ++i) a.V[i] = V[i];
    svd_unpermute_rows<<<dim3(std::max(1, std::min(64, n * n / 256)), count), 256, 0, s>>>(a);
    CTM_HIP_TRY(hipGetLastError());
  }
  return 0;
}

}  // namespace sictm
