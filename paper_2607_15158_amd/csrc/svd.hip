// SVD of the small (chi+p) x (chi+p) reduced matrix rho = Y M X (QR-based
// projector section, step 2), and of the chi x chi corners for the
// convergence measure.
//
// One-sided (Hestenes) Jacobi: U <- A V with V accumulating plane rotations
// until all column pairs of U are orthogonal to working precision; then
// s_j = |u_j|, u_j <- u_j / s_j.  One-sided Jacobi computes small singular
// values to high relative accuracy, which matters here because the
// pseudo-inverse s^-1/2 keeps directions down to a relative 1e-12.
//
// One workgroup of 1024 threads (16 wavefronts) per matrix.  A sweep visits
// all n(n-1)/2 pairs in n-1 rounds of n/2 disjoint pairs (round-robin
// tournament order); each wavefront rotates its pairs with the column data in
// registers (rows spread over the 64 lanes, reductions by cross-lane
// shuffles), and rounds are separated by workgroup barriers.  The working
// columns live in the workspace (L2-resident).  Sweeps stop when a full sweep
// performs no rotation.  Columns that end exactly zero (rank-deficient input)
// are replaced by an orthonormal completion so that u stays orthogonal.
// Singular values are returned in descending order (ties by index).

#include "common.h"

namespace sictm {
namespace {

constexpr int kSvdThreads = 1024;
constexpr int kSvdMaxN = 256;
constexpr int kRPL = kSvdMaxN / 64;   // rows per lane
constexpr int kMaxSweeps = 40;

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

struct SvdArgs {
  const double* A[kMaxProb];
  double* U[kMaxProb];
  double* S[kMaxProb];
  double* V[kMaxProb];
  double* work;       // [count][2][n][n] column-major U, V
  int n;
};

__global__ __launch_bounds__(kSvdThreads) void jacobi_svd(SvdArgs a) {
  const int mat = blockIdx.x;
  const int n = a.n;
  const int ne = n + (n & 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nwaves = kSvdThreads / 64;
  double* Uc = a.work + (size_t)mat * 2 * n * n;   // column c at Uc + c*n
  double* Vc = Uc + (size_t)n * n;
  const bool want_v = a.V[mat] != nullptr;
  const double* A = a.A[mat];

  __shared__ int rotated;
  __shared__ double snorm[kSvdMaxN];
  __shared__ int order[kSvdMaxN];

  for (int i = tid; i < n * n; i += kSvdThreads) {
    const int r = i / n, c = i % n;
    Uc[(size_t)c * n + r] = A[i];
    Vc[(size_t)c * n + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  const double tol = 1e-15 * sqrt((double)n);
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    int my_rot = 0;
    for (int round = 0; round < ne - 1; ++round) {
      for (int pi = wave; pi < ne / 2; pi += nwaves) {
        // tournament positions pi and ne-1-pi
        const int pos_a = pi, pos_b = ne - 1 - pi;
        int ca = pos_a == 0 ? 0 : ((pos_a - 1 + round) % (ne - 1)) + 1;
        int cb = ((pos_b - 1 + round) % (ne - 1)) + 1;
        if (ca >= n || cb >= n) continue;
        const int p = min(ca, cb), q = max(ca, cb);
        double up[kRPL], uq[kRPL];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < kRPL; ++t) {
          const int r = lane + 64 * t;
          up[t] = r < n ? Uc[(size_t)p * n + r] : 0.0;
          uq[t] = r < n ? Uc[(size_t)q * n + r] : 0.0;
          al += up[t] * up[t];
          be += uq[t] * uq[t];
          ga += up[t] * uq[t];
        }
        al = wsum(al);
        be = wsum(be);
        ga = wsum(ga);
        if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        ++my_rot;
#pragma unroll
        for (int tt = 0; tt < kRPL; ++tt) {
          const int r = lane + 64 * tt;
          if (r < n) {
            Uc[(size_t)p * n + r] = c * up[tt] - s * uq[tt];
            Uc[(size_t)q * n + r] = s * up[tt] + c * uq[tt];
          }
        }
        if (want_v) {
#pragma unroll
          for (int tt = 0; tt < kRPL; ++tt) {
            const int r = lane + 64 * tt;
            if (r < n) {
              const double vp = Vc[(size_t)p * n + r], vq = Vc[(size_t)q * n + r];
              Vc[(size_t)p * n + r] = c * vp - s * vq;
              Vc[(size_t)q * n + r] = s * vp + c * vq;
            }
          }
        }
      }
      __syncthreads();
    }
    if (lane == 0 && my_rot) atomicAdd(&rotated, my_rot);
    __syncthreads();
    if (rotated == 0) break;
  }

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
  // orthonormal completion of exactly-zero columns (sequential, wavefront 0)
  if (a.U[mat] != nullptr && wave == 0) {
    int cand = 0;
    for (int c = 0; c < n; ++c) {
      if (snorm[c] > 0.0) continue;
      for (; cand < n; ++cand) {
        double x[kRPL];
#pragma unroll
        for (int t = 0; t < kRPL; ++t) x[t] = (lane + 64 * t == cand) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass) {
          for (int o = 0; o < n; ++o) {
            if (o == c || (snorm[o] <= 0.0 && o > c)) continue;
            double d = 0.0;
#pragma unroll
            for (int t = 0; t < kRPL; ++t) {
              const int r = lane + 64 * t;
              if (r < n) d += Uc[(size_t)o * n + r] * x[t];
            }
            d = wsum(d);
#pragma unroll
            for (int t = 0; t < kRPL; ++t) {
              const int r = lane + 64 * t;
              if (r < n) x[t] -= d * Uc[(size_t)o * n + r];
            }
          }
        }
        double nn = 0.0;
#pragma unroll
        for (int t = 0; t < kRPL; ++t) nn += x[t] * x[t];
        nn = sqrt(wsum(nn));
        if (nn > 0.5) {
#pragma unroll
          for (int t = 0; t < kRPL; ++t) {
            const int r = lane + 64 * t;
            if (r < n) Uc[(size_t)c * n + r] = x[t] / nn;
          }
          ++cand;
          break;
        }
      }
    }
  }
  __syncthreads();
  // descending order, ties by index
  for (int c = tid; c < n; c += kSvdThreads) {
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
  for (int i = tid; i < n; i += kSvdThreads) S[i] = snorm[order[i]];
  for (int i = tid; i < n * n; i += kSvdThreads) {
    const int r = i / n, j = i % n;
    const int c = order[j];
    if (U) U[i] = Uc[(size_t)c * n + r];
    if (V) V[i] = Vc[(size_t)c * n + r];
  }
}

}  // namespace

size_t svd_workspace_bytes(int count, int n) { return (size_t)count * 2 * n * n * sizeof(double); }

int launch_svd(int count, const double* const* A, double* const* U, double* const* S,
               double* const* V, int n, void* ws, hipStream_t s) {
  if (count <= 0 || n <= 0) return 0;
  if (count > kMaxProb || n > kSvdMaxN) {
    set_thread_error("launch_svd: n <= 256 and at most 8 matrices per launch");
    return 1;
  }
  SvdArgs a{};
  a.n = n;
  a.work = (double*)ws;
  for (int i = 0; i < count; ++i) {
    a.A[i] = A[i];
    a.U[i] = U ? U[i] : nullptr;
    a.S[i] = S[i];
    a.V[i] = V ? V[i] : nullptr;
  }
  jacobi_svd<<<count, kSvdThreads, 0, s>>>(a);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace sictm
