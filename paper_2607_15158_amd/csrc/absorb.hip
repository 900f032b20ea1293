// Site absorption of the enlarged corners through the single-layer tensor.
//
// The enlarged corner of the CTMRG move (Fig. 1, the corner C T T a) ends
// with the absorption Ct[(x, o1), (y, o2)] = sum_(p, q) W[(x, y), p, q]
// a[(p, q), (o1, o2)] of the double-layer site tensor a, whose legs pair a
// ket and a bra index (p = pk D + pb, ket-major) with
// a = sum_s A[s, pk, qk, o1k, o2k] A[s, pb, qb, o1b, o2b].  Contracted as one
// D^4 x D^4 matrix that costs 2 chi^2 D^8 flops per corner.  Here the ket
// layer is absorbed first and the bra layer (with the physical index) second:
//   X[(x, y), pb, qb, (s, o1k, o2k)] = sum_(pk, qk) W[(x, y), (pk pb), (qk qb)] A[s, pk, qk, o1k, o2k]
//   Ct[(x, o1k o1b), (y, o2k o2b)]   = sum_(pb, qb, s) X[...] A[s, pb, qb, o1b, o2b]
// the same tensor for 4 d chi^2 D^6 flops (9x less at D = 6, d = 2).
//
// One workgroup takes kAbsG = 2 consecutive (x, y) pairs of one problem:
// their W rows and the problem's leg permutation of A are staged in LDS, the
// first product (rows (g, pb, qb), K = D^2, N = d D^2) writes X to LDS, the
// second (rows (g, o1k, o2k), K = d D^2, N = D^2) stages the output block in
// LDS, from where it is written through the output's index map (for the
// corners, each pair's D^2 columns of a row of Ct contiguously).  The edges'
// absorption Z2 = Z1 a has the same form with rows (b, g').  Both run on v_mfma_f64_16x16x4; the index
// groupings of every operand are additive, so per-dimension offset tables in
// LDS turn each fragment into a per-lane base plus one table entry per
// k-step.

#include "common.h"
#include "elem.h"

namespace sictm {
namespace {

constexpr int kAbsG = 2;          // (x, y) pairs per workgroup
constexpr int kAbsMaxDl = 36;     // D^2 up to D = 6
constexpr int kAbsMaxN = 72;      // d D^2 up to d = 2 at D = 6
constexpr int kAbsRB = ((kAbsG * kAbsMaxDl + 15) / 16 + 3) / 4;   // 16-row blocks per wavefront
constexpr int kAbsNB1 = (kAbsMaxN + 15) / 16;    // column blocks of the first product
constexpr int kAbsNB2 = (kAbsMaxDl + 15) / 16;   // column blocks of the second

constexpr int kAbsMaxProb = 8;

struct AbsArgs {
  const double* W[kAbsMaxProb];    // [nR][Dl][Dl] per problem
  void* Ct[kAbsMaxProb];           // output (TO) per problem, element (R, o1, o2) at
                                   // (R / n2) sR1 + (R % n2) sR2 + o1 so1 + o2 so2
  const double* A[kAbsMaxProb];    // single-layer site tensor [s][u][l][d][r] per problem
  long sA[kAbsMaxProb][4];         // per problem: strides in A of the legs p, q, o1, o2
  long nR, sR1, sR2, so1, so2;
  int n2, D, d, Dl;
};

// DT: the bond dimension D as a compile-time constant (every index division
// by D or D^2 becomes a multiply).
template <int DT, typename TO>
__global__ __launch_bounds__(256) void k_absorb_corner(AbsArgs a) {
  // LDS: one buffer holds in turn the W rows [G][Dl][Dl], X [G * Dl][dDl]
  // and the corner block in Ct's order; A [s][p][q][o1][o2] (62 KB in all:
  // two workgroups share a CU)
  static_assert(kAbsMaxN >= kAbsMaxDl, "X is the largest stage");
  __shared__ double Bx[kAbsG * kAbsMaxDl * kAbsMaxN];
  __shared__ double As[kAbsMaxN * kAbsMaxDl];
  double* const Ws = Bx;
  double* const Xs = Bx;
  const int corner = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int D = DT, Dl = DT * DT;
  const int d = a.d, dDl = d * Dl;
  const long nR = a.nR;
  const long R0 = (long)blockIdx.x * kAbsG;
  const int G = (int)min((long)kAbsG, nR - R0);
  __shared__ long rowoff[kAbsG];   // output offset of pair g
  if (tid < G) {
    const long R = R0 + tid;
    rowoff[tid] = (R / a.n2) * a.sR1 + (R % a.n2) * a.sR2;
  }
  __shared__ int ko1[kAbsMaxDl], mo1[kAbsMaxDl], k1off[kAbsMaxDl], n1off[kAbsMaxN];
  __shared__ int ko2[kAbsMaxN], k2off[kAbsMaxN], n2off[kAbsMaxDl], mo2[kAbsMaxDl];
  const double* W = a.W[corner];
  for (long i = tid; i < (long)G * Dl * Dl; i += 256) Ws[i] = W[R0 * Dl * Dl + i];
  const long* st = a.sA[corner];
  constexpr int D2 = D * D, D3 = D2 * D, D4 = D3 * D;
  for (int i = tid; i < d * D4; i += 256) {
    int rem = i;
    const int o2 = rem % D; rem /= D;
    const int o1 = rem % D; rem /= D;
    const int q = rem % D; rem /= D;
    const int p = rem % D;
    const int s = rem / D;
    As[i] = a.A[corner][(long)s * D4 + p * st[0] + q * st[1] + o1 * st[2] + o2 * st[3]];
  }
  for (int i = tid; i < Dl; i += 256) {
    const int hi = i / D, lo = i % D;
    ko1[i] = hi * D * Dl + lo * D;       // k = (pk, qk) -> W offset
    mo1[i] = hi * Dl + lo;               // m' = (pb, qb) -> W offset
    k1off[i] = hi * D3 + lo * D2;        // k = (pk, qk) -> A offset
    n2off[i] = hi * D + lo;              // n = (o1b, o2b) -> A offset
    mo2[i] = hi * D + lo;                // (o1k, o2k) -> X column offset
  }
  for (int i = tid; i < dDl; i += 256) {
    const int s = i / Dl, r = i % Dl;
    n1off[i] = s * D4 + (r / D) * D + r % D;                  // n = (s, o1k, o2k) -> A
    ko2[i] = (r / D * D + r % D) * dDl + s * Dl;              // k = (pb, qb, s) (pairs first) -> X
    k2off[i] = s * D4 + (r / D) * D3 + (r % D) * D2;          // k = (pb, qb, s) -> A
  }
  __syncthreads();
  // Wavefront w takes the 16-row blocks w and w + 4 of both products and
  // every column block, so each k-step's fragments feed up to 10 (then 6)
  // independent accumulators.
  const int M = G * Dl;
  const int mb = (M + 15) >> 4, nb1 = (dDl + 15) >> 4, nb2 = (Dl + 15) >> 4;
  const int li = lane & 15, lk = lane >> 4;
  int abase[kAbsRB];
  bool arow[kAbsRB];   // this lane's operand row m exists (per lane)
  bool blk[kAbsRB];    // the wavefront's u-th row block exists (uniform)
  // product 1: X[(g, pb, qb), (s, o1k, o2k)], rows m = g Dl + m'
  {
    int bbase[kAbsNB1];
    bool bcol[kAbsNB1];
#pragma unroll
    for (int u = 0; u < kAbsRB; ++u) {
      const int m = ((wave + 4 * u) << 4) + li;
      blk[u] = (wave + 4 * u) < mb;
      arow[u] = blk[u] && m < M;
      abase[u] = arow[u] ? (m / Dl) * Dl * Dl + mo1[m % Dl] : 0;
    }
#pragma unroll
    for (int v = 0; v < kAbsNB1; ++v) {
      const int n = (v << 4) + li;
      bcol[v] = v < nb1 && n < dDl;
      bbase[v] = bcol[v] ? n1off[n] : 0;
    }
    v4d acc[kAbsRB][kAbsNB1];
#pragma unroll
    for (int u = 0; u < kAbsRB; ++u)
#pragma unroll
      for (int v = 0; v < kAbsNB1; ++v) acc[u][v] = v4d{0, 0, 0, 0};
    for (int t = 0; t < Dl; t += 4) {
      const int k = t + lk;
      const bool kin = k < Dl;
      const int kk = kin ? k : 0;
      const int ka = ko1[kk], kb = k1off[kk];
      double av[kAbsRB], bv[kAbsNB1];
#pragma unroll
      for (int u = 0; u < kAbsRB; ++u) av[u] = (arow[u] && kin) ? Ws[abase[u] + ka] : 0.0;
#pragma unroll
      for (int v = 0; v < kAbsNB1; ++v) bv[v] = (bcol[v] && kin) ? As[bbase[v] + kb] : 0.0;
#pragma unroll
      for (int u = 0; u < kAbsRB; ++u)
#pragma unroll
        for (int v = 0; v < kAbsNB1; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
    }
    __syncthreads();   // every wavefront is done with the W rows
#pragma unroll
    for (int u = 0; u < kAbsRB; ++u)
#pragma unroll
      for (int v = 0; v < kAbsNB1; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ((wave + 4 * u) << 4) + lk + 4 * r, col = (v << 4) + li;
          if (blk[u] && row < M && col < dDl) Xs[row * dDl + col] = acc[u][v][r];
        }
  }
  __syncthreads();
  // product 2: rows (g, o1k, o2k), columns (o1b, o2b), K = (s, pb, qb); the
  // results go to LDS (over X) in Ct's order, [g][(o1k, o1b)][(o2k, o2b)]
  {
    int bbase[kAbsNB2];
    bool bcol[kAbsNB2];
#pragma unroll
    for (int u = 0; u < kAbsRB; ++u) {
      const int m = ((wave + 4 * u) << 4) + li;
      abase[u] = arow[u] ? (m / Dl) * Dl * dDl + mo2[m % Dl] : 0;
    }
#pragma unroll
    for (int v = 0; v < kAbsNB2; ++v) {
      const int n = (v << 4) + li;
      bcol[v] = v < nb2 && n < Dl;
      bbase[v] = bcol[v] ? n2off[n] : 0;
    }
    v4d acc[kAbsRB][kAbsNB2];
#pragma unroll
    for (int u = 0; u < kAbsRB; ++u)
#pragma unroll
      for (int v = 0; v < kAbsNB2; ++v) acc[u][v] = v4d{0, 0, 0, 0};
    for (int t = 0; t < dDl; t += 4) {
      const int k = t + lk;
      const bool kin = k < dDl;
      const int kk = kin ? k : 0;
      const int ka = ko2[kk], kb = k2off[kk];
      double av[kAbsRB], bv[kAbsNB2];
#pragma unroll
      for (int u = 0; u < kAbsRB; ++u) av[u] = (arow[u] && kin) ? Xs[abase[u] + ka] : 0.0;
#pragma unroll
      for (int v = 0; v < kAbsNB2; ++v) bv[v] = (bcol[v] && kin) ? As[bbase[v] + kb] : 0.0;
#pragma unroll
      for (int u = 0; u < kAbsRB; ++u)
#pragma unroll
        for (int v = 0; v < kAbsNB2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
    }
    __syncthreads();   // every wavefront is done with X
#pragma unroll
    for (int u = 0; u < kAbsRB; ++u)
#pragma unroll
      for (int v = 0; v < kAbsNB2; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ((wave + 4 * u) << 4) + lk + 4 * r, col = (v << 4) + li;
          if (blk[u] && row < M && col < Dl) {
            const int g = row / Dl, o = row % Dl, o1k = o / D, o2k = o % D;
            const int o1b = col / D, o2b = col % D;
            Ws[(g * Dl + o1k * D + o1b) * Dl + o2k * D + o2b] = acc[u][v][r];
          }
        }
  }
  __syncthreads();
  // for the corners, rows (x, o1) of Ct hold the D^2 columns (y, o2) of one
  // pair contiguously
  TO* Ct = (TO*)a.Ct[corner];
  for (int i = tid; i < G * Dl * Dl; i += 256) {
    const int g = i / (Dl * Dl), rem = i % (Dl * Dl), o1 = rem / Dl, o2 = rem % Dl;
    Ct[rowoff[g] + o1 * a.so1 + o2 * a.so2] = (TO)Ws[i];
  }
}

}  // namespace

bool absorb_corner_fits(int D, int d) {
  return d >= 1 && D >= 2 && D * D <= kAbsMaxDl && d * D * D <= kAbsMaxN;
}

template <typename TO>
static void launch_absorb_t(const AbsArgs& a, dim3 grid, int D, hipStream_t s) {
  switch (D) {
    case 2: k_absorb_corner<2, TO><<<grid, 256, 0, s>>>(a); break;
    case 3: k_absorb_corner<3, TO><<<grid, 256, 0, s>>>(a); break;
    case 4: k_absorb_corner<4, TO><<<grid, 256, 0, s>>>(a); break;
    case 5: k_absorb_corner<5, TO><<<grid, 256, 0, s>>>(a); break;
    default: k_absorb_corner<6, TO><<<grid, 256, 0, s>>>(a); break;
  }
}

int launch_absorb(int count, const double* const* W, void* const* out, bool out_f32,
                  const double* const* A, const long (*legs)[4], long nR, int n2,
                  const long* ostr, int D, int d, hipStream_t s) {
  if (!absorb_corner_fits(D, d) || nR < 1 || n2 < 1 || count < 1 || count > kAbsMaxProb) {
    set_thread_error("single-layer absorption: D, d or the problem count outside its tiling");
    return 1;
  }
  AbsArgs a{};
  for (int i = 0; i < count; ++i) {
    a.W[i] = W[i];
    a.Ct[i] = out[i];
    a.A[i] = A[i];
    for (int j = 0; j < 4; ++j) a.sA[i][j] = legs[i][j];
  }
  a.nR = nR;
  a.n2 = n2;
  a.sR1 = ostr[0];
  a.sR2 = ostr[1];
  a.so1 = ostr[2];
  a.so2 = ostr[3];
  a.D = D;
  a.d = d;
  a.Dl = D * D;
  dim3 grid((unsigned)((nR + kAbsG - 1) / kAbsG), count);
  if (out_f32) launch_absorb_t<float>(a, grid, D, s);
  else launch_absorb_t<double>(a, grid, D, s);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int launch_absorb_corners(const double* const* W, void* const* Ct, bool out_f32, const double* A,
                          const long (*legs)[4], int chi, int D, int d, hipStream_t s) {
  const long Dl = (long)D * D, N1 = (long)chi * Dl;
  const long ostr[4] = {Dl * N1, Dl, N1, 1};
  const double* As[4] = {A, A, A, A};
  return launch_absorb(4, W, Ct, out_f32, As, legs, (long)chi * chi, chi, ostr, D, d, s);
}

}  // namespace sictm
