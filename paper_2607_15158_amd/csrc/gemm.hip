// Batched, index-mapped GEMM on the gfx950 matrix cores.
//
// Every contraction of a CTMRG move -- the enlarged-corner build, the
// applications of the enlarged corners to the N x k isometry blocks, the
// reduced matrix rho, the projector products and the renormalisation of C
// and T (Fig. 1; QR-based projector section) -- is one launch of this kernel
// family.  Leg permutations are folded into the operand strides and into the
// two-level output map, so no tensor is ever transposed in memory.
//
// Design: 256-thread workgroups (4 wavefronts of 64), one BM x BN output tile
// per workgroup, K staged through LDS in BK slices with a register prefetch
// of the next slice.  Wavefronts own (BM/WGM) x (BN/WGN) sub-tiles built
// from 16x16 MFMA blocks:
//   float64: v_mfma_f64_16x16x4_f64  (A: lane -> (row l%16, k l/16))
//   float32: v_mfma_f32_16x16x4_f32  (same operand layout)
//   bf16   : v_mfma_f32_16x16x32_bf16 (A: lane -> (row l%16, k 8*(l/16)..+7))
// and accumulate in float64 (f64 inputs) or float32 (f32/bf16 inputs).
// Result element r = 0..3 of lane l lies in column l%16 and in row
// l/16 + 4r for the float64 instruction, row 4(l/16) + r for the others
// (both measured on gfx950).
// Workgroup ids are remapped so that consecutive tiles share an XCD (and its
// L2), since the hardware deals consecutive workgroups round-robin to the 8
// XCDs.

#include "common.h"

#include <algorithm>

namespace sictm {
namespace {

template <typename Dst, typename Src>
__device__ __forceinline__ Dst cvt(Src x) { return (Dst)x; }
template <>
__device__ __forceinline__ __bf16 cvt<__bf16, double>(double x) { return (__bf16)(float)x; }
template <>
__device__ __forceinline__ __bf16 cvt<__bf16, float>(float x) { return (__bf16)x; }
template <>
__device__ __forceinline__ float cvt<float, __bf16>(__bf16 x) { return (float)x; }
template <>
__device__ __forceinline__ double cvt<double, __bf16>(__bf16 x) { return (double)(float)x; }

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ long map2(int i, int div, long s1, long s0) {
  return (long)(i / div) * s1 + (long)(i % div) * s0;
}

// ---------------------------------------------------------------------------
// 16x16x4 path (float64 or float32 compute type CT).
// ---------------------------------------------------------------------------
template <typename CT> struct Mfma4;
template <> struct Mfma4<double> {
  using acc_t = v4d;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma4<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kK4BK = 16, kK4Pad = 2;

// One BM x BN output tile (tm, tn) of problem `prob`, inner batch `batch`.
// The K loop runs in ascending 16-wide slices whatever the tile shape, so an
// output element gets the same bits from every tile shape and grid.  The
// slices are double-buffered in LDS: the global loads of slice kt + 1 are in
// flight while slice kt is multiplied, then stored into the other buffer,
// one barrier per slice.
template <typename TA, typename TB, typename TC, typename CT, int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void k4_tile(const GemmBatch& g, int prob, int batch, int tm, int tn,
                                        CT (*As)[kK4BK][BM + kK4Pad],
                                        CT (*Bs)[kK4BK][BN + kK4Pad]) {
  constexpr int BK = kK4BK;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int MI = WTM / 16, NI = WTN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(WGM * WGN == 4, "four wavefronts");
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile multiple of 16");
  static_assert((BM * BK) % 256 == 0 && (BN * BK) % 256 == 0, "tile loads");
  using Acc = typename Mfma4<CT>::acc_t;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const int trans = g.transA[prob];
  const TA* A = (const TA*)g.A[prob] + (long)batch * g.a_bs;
  const TB* B = (const TB*)g.B[prob] + (long)batch * g.b_bs;
  TC* C = (TC*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  CT ra[EA], rb[EB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int i = tid + e * 256;
      int m, kk;
      if (trans) { m = i % BM; kk = i / BM; } else { m = i / BK; kk = i % BK; }
      const int gm = m0 + m, gk = k0 + kk;
      CT v = (CT)0;
      if (gm < M && gk < K) v = cvt<CT>(trans ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk]);
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int i = tid + e * 256;
      const int n = i % BN, kk = i / BN;
      const int gn = n0 + n, gk = k0 + kk;
      CT v = (CT)0;
      if (gn < N && gk < K) v = cvt<CT>(B[(long)gk * ldb + gn]);
      rb[e] = v;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int i = tid + e * 256;
      int m, kk;
      if (trans) { m = i % BM; kk = i / BM; } else { m = i / BK; kk = i % BK; }
      As[buf][kk][m] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int i = tid + e * 256;
      Bs[buf][i / BN][i % BN] = rb[e];
    }
  };

  Acc acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      CT a[MI], b[NI];
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = As[buf][kr][wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = Mfma4<CT>::op(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) store_tiles(buf ^ 1);
    __syncthreads();
  }

  // epilogue: two-level output map
  long offn[NI];
  bool okn[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int n = n0 + wn * WTN + j * 16 + (lane & 15);
    okn[j] = n < N;
    offn[j] = okn[j] ? map2(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const double alpha = g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + Mfma4<CT>::row(lane, r);
      if (m >= M) continue;
      const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        TC* p = C + offm + offn[j];
        double v = alpha * (double)acc[i][j][r];
        if (g.accumulate) v += (double)*p;
        *p = cvt<TC>(v);
      }
    }
  }
}

template <typename TA, typename TB, typename TC, typename CT, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_k4(GemmBatch g, int tiles_m, int tiles_n) {
  __shared__ CT As[2][kK4BK][BM + kK4Pad];
  __shared__ CT Bs[2][kK4BK][BN + kK4Pad];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int prob = blockIdx.y / g.nbatch, batch = blockIdx.y % g.nbatch;
  k4_tile<TA, TB, TC, CT, BM, BN, WGM, WGN>(g, prob, batch, tile / tiles_n, tile % tiles_n, As, Bs);
}

// ---------------------------------------------------------------------------
// Skinny float64 path for C (M x N) = op(A) (M x K) B (K x N) with N <= BN:
// the enlarged corner applied to an N x k isometry block.  One workgroup owns
// a BM x BN tile (the whole width of B), so A is streamed from HBM exactly
// once; K is staged through double-buffered LDS in BK slices with 16-byte
// global loads, one barrier per slice.  The launch is flattened over
// (problem, tile) and dealt to the XCDs in contiguous chunks, so the
// workgroups of one problem share an L2 and its slice of B.
// ROLE only separates instantiations (and kernel names in profiles).
// ---------------------------------------------------------------------------
typedef double v2d __attribute__((ext_vector_type(2)));

// LDS layouts of the A slice: transposed operands arrive m-contiguous and are
// kept as [k][m] (rows padded by 16 doubles); plain ones arrive
// k-contiguous and are kept as [m][k] with rows of BK + 1 doubles, so that
// both the 16-byte row loads and the fragment reads (16 consecutive m at
// fixed k per lane group) avoid bank conflicts.
// Two adjacent doubles: one 16-byte load, or two 8-byte ones where odd
// leading dimensions leave every other row 8-byte aligned only.
template <bool ODD>
__device__ __forceinline__ v2d ld_pair(const double* p) {
  if (ODD) {
    v2d v;
    v.x = p[0];
    v.y = p[1];
    return v;
  }
  return *(const v2d*)p;
}

template <int BM, int BK>
struct SkinnyA {
  static constexpr int LT = BM + 16;          // [k][m] row length
  static constexpr int LN = BK + 1;           // [m][k] row length
  static constexpr int SIZE = (BK * LT > BM * LN) ? BK * LT : BM * LN;
};

template <int BM, int BN, int WGM, int WGN, bool TRANS, bool ODD = false>
__device__ __forceinline__ void skinny_tile(const GemmBatch& g, int tiles_m, int tiles_n, int lin,
                                            double (*As)[SkinnyA<BM, 16>::SIZE],
                                            double (*Bs)[16][BN + 16]) {
  constexpr int BK = 16;
  using AL = SkinnyA<BM, BK>;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int MI = WTM / 16, NI = WTN / 16;
  constexpr int NT = 64 * WGM * WGN;                   // threads per workgroup
  constexpr int NA = BM * BK / 2, NB = BN * BK / 2;    // 16-byte loads per slice
  constexpr int VA = (NA + NT - 1) / NT, VB = (NB + NT - 1) / NT;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile multiple of 16");

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int per_prob = tiles_m * tiles_n;
  const int pb = lin / per_prob, tile = lin % per_prob;
  const int prob = pb / g.nbatch, batch = pb % g.nbatch;
  const int tn = tile % tiles_n, tm = tile / tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const double* A = (const double*)g.A[prob] + (long)batch * g.a_bs;
  const double* B = (const double*)g.B[prob] + (long)batch * g.b_bs;
  double* C = (double*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  v2d ra[VA], rb[VB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      v2d v = {0.0, 0.0};
      if (i < NA) {
        if (TRANS) {
          const int gk = k0 + i / (BM / 2), gm = m0 + 2 * (i % (BM / 2));
          if (gk < K) {
            const double* p = A + (long)gk * lda + gm;
            if (gm + 1 < M) v = ld_pair<ODD>(p);
            else if (gm < M) v.x = p[0];
          }
        } else {
          const int gm = m0 + i / (BK / 2), gk = k0 + 2 * (i % (BK / 2));
          if (gm < M) {
            const double* p = A + (long)gm * lda + gk;
            if (gk + 1 < K) v = ld_pair<ODD>(p);
            else if (gk < K) v.x = p[0];
          }
        }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      const int gk = k0 + i / (BN / 2), gn = n0 + 2 * (i % (BN / 2));
      v2d v = {0.0, 0.0};
      if (i < NB && gk < K) {
        const double* p = B + (long)gk * ldb + gn;
        if (gn + 1 < N) v = ld_pair<ODD>(p);
        else if (gn < N) v.x = p[0];
      }
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      if (i < NA) {
        if (TRANS) {
          const int kk = i / (BM / 2), m = 2 * (i % (BM / 2));
          *(v2d*)&As[buf][kk * AL::LT + m] = ra[e];
        } else {
          const int m = i / (BK / 2), kk = 2 * (i % (BK / 2));
          As[buf][m * AL::LN + kk] = ra[e].x;
          As[buf][m * AL::LN + kk + 1] = ra[e].y;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      if (i < NB) *(v2d*)&Bs[buf][i / (BN / 2)][2 * (i % (BN / 2))] = rb[e];
    }
  };

  v4d acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = v4d{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[MI], b[NI];
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int m = wm * WTM + i * 16 + (lane & 15);
        a[i] = TRANS ? As[buf][kr * AL::LT + m] : As[buf][m * AL::LN + kr];
      }
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  long offn[NI];
  bool okn[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int n = n0 + wn * WTN + j * 16 + (lane & 15);
    okn[j] = n < N;
    offn[j] = okn[j] ? map2(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const double alpha = g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + (lane >> 4) + 4 * r;
      if (m >= M) continue;
      const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        double* p = C + offm + offn[j];
        double v = alpha * acc[i][j][r];
        if (g.accumulate) v += *p;
        *p = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Float32 form of the double-buffered skinny tile, for the float32
// contractions with long K (the site absorptions of the corners and of the
// edges' renormalisation, 20736 x 1296 x 1296 per corner at D = 6, and
// Zc = Ct P_l): operands of type TA / TB are rounded to float32 on their way
// into LDS and multiplied on v_mfma_f32_16x16x4f32 with float32
// accumulation (operand layout as the float64 instruction; result element r
// of lane l in row 4 (l / 16) + r).
// ---------------------------------------------------------------------------
template <int BM, int BK>
struct SkinnyAF {
  static constexpr int LT = BM + 16;
  static constexpr int LN = BK + 1;
  static constexpr int SIZE = (BK * LT > BM * LN) ? BK * LT : BM * LN;
};

template <typename TA, typename TB, typename TC, int BM, int BN, int WGM, int WGN, bool TRANS>
__device__ __forceinline__ void skinny_tile_f32(const GemmBatch& g, int tiles_m, int tiles_n,
                                                int lin, float (*As)[SkinnyAF<BM, 16>::SIZE],
                                                float (*Bs)[16][BN + 16]) {
  constexpr int BK = 16;
  using AL = SkinnyAF<BM, BK>;
  using VA2 = TA __attribute__((ext_vector_type(2)));
  using VB2 = TB __attribute__((ext_vector_type(2)));
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int MI = WTM / 16, NI = WTN / 16;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int NA = BM * BK / 2, NB = BN * BK / 2;
  constexpr int VA = (NA + NT - 1) / NT, VB = (NB + NT - 1) / NT;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile multiple of 16");

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int per_prob = tiles_m * tiles_n;
  const int pb = lin / per_prob, tile = lin % per_prob;
  const int prob = pb / g.nbatch, batch = pb % g.nbatch;
  const int tn = tile % tiles_n, tm = tile / tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const TA* A = (const TA*)g.A[prob] + (long)batch * g.a_bs;
  const TB* B = (const TB*)g.B[prob] + (long)batch * g.b_bs;
  TC* C = (TC*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  VA2 ra[VA];
  VB2 rb[VB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      VA2 v = {(TA)0, (TA)0};
      if (i < NA) {
        if (TRANS) {
          const int gk = k0 + i / (BM / 2), gm = m0 + 2 * (i % (BM / 2));
          if (gk < K) {
            const TA* p = A + (long)gk * lda + gm;
            if (gm + 1 < M) v = *(const VA2*)p;
            else if (gm < M) v.x = p[0];
          }
        } else {
          const int gm = m0 + i / (BK / 2), gk = k0 + 2 * (i % (BK / 2));
          if (gm < M) {
            const TA* p = A + (long)gm * lda + gk;
            if (gk + 1 < K) v = *(const VA2*)p;
            else if (gk < K) v.x = p[0];
          }
        }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      const int gk = k0 + i / (BN / 2), gn = n0 + 2 * (i % (BN / 2));
      VB2 v = {(TB)0, (TB)0};
      if (i < NB && gk < K) {
        const TB* p = B + (long)gk * ldb + gn;
        if (gn + 1 < N) v = *(const VB2*)p;
        else if (gn < N) v.x = p[0];
      }
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      if (i < NA) {
        if (TRANS) {
          const int kk = i / (BM / 2), m = 2 * (i % (BM / 2));
          As[buf][kk * AL::LT + m] = (float)ra[e].x;
          As[buf][kk * AL::LT + m + 1] = (float)ra[e].y;
        } else {
          const int m = i / (BK / 2), kk = 2 * (i % (BK / 2));
          As[buf][m * AL::LN + kk] = (float)ra[e].x;
          As[buf][m * AL::LN + kk + 1] = (float)ra[e].y;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      if (i < NB) {
        Bs[buf][i / (BN / 2)][2 * (i % (BN / 2))] = (float)rb[e].x;
        Bs[buf][i / (BN / 2)][2 * (i % (BN / 2)) + 1] = (float)rb[e].y;
      }
    }
  };

  v4f acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      float a[MI], b[NI];
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int m = wm * WTM + i * 16 + (lane & 15);
        a[i] = TRANS ? As[buf][kr * AL::LT + m] : As[buf][m * AL::LN + kr];
      }
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  long offn[NI];
  bool okn[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int n = n0 + wn * WTN + j * 16 + (lane & 15);
    okn[j] = n < N;
    offn[j] = okn[j] ? map2(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const double alpha = g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
      if (m >= M) continue;
      const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        TC* p = C + offm + offn[j];
        double v = alpha * (double)acc[i][j][r];
        if (g.accumulate) v += (double)*p;
        *p = cvt<TC>(v);
      }
    }
  }
}

template <typename TA, typename TB, typename TC, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN, 512 / (64 * WGM * WGN)) void gemm_skinny_f32x(
    GemmBatch g, int tiles_m, int tiles_n) {
  __shared__ float As[2][SkinnyAF<BM, 16>::SIZE];
  __shared__ float Bs[2][16][BN + 16];
  const int per_prob = tiles_m * tiles_n;
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int prob = lin / per_prob / g.nbatch;
  if (g.transA[prob])
    skinny_tile_f32<TA, TB, TC, BM, BN, WGM, WGN, true>(g, tiles_m, tiles_n, lin, As, Bs);
  else
    skinny_tile_f32<TA, TB, TC, BM, BN, WGM, WGN, false>(g, tiles_m, tiles_n, lin, As, Bs);
}

// ---------------------------------------------------------------------------
// Split form of the skinny tile for the SI applications (stream-K style).  A
// launch of one tile per workgroup leaves CUs idle or half loaded when the
// count x tiles_m tiles do not fill the chip evenly (432 tiles of 96 rows on
// 512 slots at D = 6).  Here one workgroup of 8 wavefronts per CU (192 x 160
// tiles: each B block is re-read by half as many tiles as with 96 rows) takes
// an equal, contiguous range of the (tile, K-slice) space.  A tile inside one
// range is written directly; a tile cut by range boundaries leaves partial
// tiles in scratch (slot 2w for the segment that starts range w, 2w+1 for the
// one that ends it), which a second kernel sums in workgroup order, so
// results do not depend on timing.
// ---------------------------------------------------------------------------
struct StreamK {
  long total;     // count * tiles_m * nslices
  int nslices;    // BK-slices of K per tile
  int tiles_m;
  int nwg;        // workgroups (ranges) of the main kernel
  double* part;   // 2 * nwg partial BM x BN tiles (row-major)
};

__device__ __forceinline__ long sk_begin(long w, const StreamK& sk) { return w * sk.total / sk.nwg; }

__device__ __forceinline__ int sk_owner(long p, const StreamK& sk) {
  int w = (int)((p * sk.nwg) / sk.total);
  while (w + 1 < sk.nwg && sk_begin(w + 1, sk) <= p) ++w;
  while (w > 0 && sk_begin(w, sk) > p) --w;
  return w;
}

// acc += op(A)[m0 .. m0+BM) x B over the K slices [s0, s1) of problem prob.
template <int BM, int BN, int WGM, int WGN, bool TRANS, bool BODD, int MI, int NI>
__device__ __forceinline__ void sk_segment(const GemmBatch& g, int prob, int m0, int s0, int s1,
                                           double (*As)[SkinnyA<BM, 16>::SIZE],
                                           double (*Bs)[16][BN + 16], v4d (&acc)[MI][NI]) {
  constexpr int BK = 16;
  using AL = SkinnyA<BM, BK>;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int NA = BM * BK / 2, NB = BN * BK / 2;
  constexpr int VA = (NA + NT - 1) / NT, VB = (NB + NT - 1) / NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int M = g.M, N = g.N, K = g.K;
  const double* A = (const double*)g.A[prob];
  const double* B = (const double*)g.B[prob];
  const long lda = g.lda, ldb = g.ldb;
  v2d ra[VA], rb[VB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      v2d v = {0.0, 0.0};
      if (i < NA) {
        if (TRANS) {
          const int gk = k0 + i / (BM / 2), gm = m0 + 2 * (i % (BM / 2));
          if (gk < K) {
            const double* p = A + (long)gk * lda + gm;
            if (gm + 1 < M) v = *(const v2d*)p;
            else if (gm < M) v.x = p[0];
          }
        } else {
          const int gm = m0 + i / (BK / 2), gk = k0 + 2 * (i % (BK / 2));
          if (gm < M) {
            const double* p = A + (long)gm * lda + gk;
            if (gk + 1 < K) v = *(const v2d*)p;
            else if (gk < K) v.x = p[0];
          }
        }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      const int gk = k0 + i / (BN / 2), gn = 2 * (i % (BN / 2));
      v2d v = {0.0, 0.0};
      if (i < NB && gk < K) {
        const double* p = B + (long)gk * ldb + gn;
        if (gn + 1 < N) {
          // an odd ldb leaves every other row 8-byte aligned only
          if (BODD) {
            v.x = p[0];
            v.y = p[1];
          } else {
            v = *(const v2d*)p;
          }
        } else if (gn < N) {
          v.x = p[0];
        }
      }
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      if (i < NA) {
        if (TRANS) {
          const int kk = i / (BM / 2), m = 2 * (i % (BM / 2));
          *(v2d*)&As[buf][kk * AL::LT + m] = ra[e];
        } else {
          const int m = i / (BK / 2), kk = 2 * (i % (BK / 2));
          As[buf][m * AL::LN + kk] = ra[e].x;
          As[buf][m * AL::LN + kk + 1] = ra[e].y;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      if (i < NB) *(v2d*)&Bs[buf][i / (BN / 2)][2 * (i % (BN / 2))] = rb[e];
    }
  };
  load(s0 * BK);
  store(0);
  __syncthreads();
  for (int kt = s0; kt < s1; ++kt) {
    const int buf = (kt - s0) & 1;
    if (kt + 1 < s1) load((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[MI], b[NI];
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int m = wm * WTM + i * 16 + (lane & 15);
        a[i] = TRANS ? As[buf][kr * AL::LT + m] : As[buf][m * AL::LN + kr];
      }
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < s1) store(buf ^ 1);
    __syncthreads();
  }
}

template <int BM, int BN, int WGM, int WGN, bool BODD>
__global__ __launch_bounds__(64 * WGM * WGN, 512 / (64 * WGM * WGN)) void gemm_streamk_f64(
    GemmBatch g, StreamK sk) {
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int MI = WTM / 16, NI = WTN / 16;
  __shared__ double As[2][SkinnyA<BM, 16>::SIZE];
  __shared__ double Bs[2][16][BN + 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const long begin = sk_begin(w, sk), end = sk_begin(w + 1, sk);
  const int M = g.M, N = g.N;
  // segments last to first: a range of L <= nslices slices then reads slice
  // t of its second tile, and later slice t + nslices - L of its first, at
  // step t, so the ranges sharing a problem (and an XCD) walk K in two
  // phases and reuse each B slice from L2
  long pend = end;
  while (pend > begin) {
    const long tile = (pend - 1) / sk.nslices;
    const long pos = tile * sk.nslices > begin ? tile * sk.nslices : begin;
    const int s0 = (int)(pos - tile * sk.nslices), s1 = (int)(pend - tile * sk.nslices);
    const int prob = (int)(tile / sk.tiles_m), m0 = (int)(tile % sk.tiles_m) * BM;
    v4d acc[MI][NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) acc[i][j] = v4d{0, 0, 0, 0};
    if (g.transA[prob])
      sk_segment<BM, BN, WGM, WGN, true, BODD, MI, NI>(g, prob, m0, s0, s1, As, Bs, acc);
    else
      sk_segment<BM, BN, WGM, WGN, false, BODD, MI, NI>(g, prob, m0, s0, s1, As, Bs, acc);
    if (s0 == 0 && s1 == sk.nslices) {
      // the whole tile: written here
      double* C = (double*)g.C[prob];
      long offn[NI];
      bool okn[NI];
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int n = wn * WTN + j * 16 + (lane & 15);
        okn[j] = n < N;
        offn[j] = okn[j] ? map2(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
      }
#pragma unroll
      for (int i = 0; i < MI; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * WTM + i * 16 + (lane >> 4) + 4 * r;
          if (m >= M) continue;
          const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
          for (int j = 0; j < NI; ++j) {
            if (!okn[j]) continue;
            double* p = C + offm + offn[j];
            double v = g.alpha * acc[i][j][r];
            if (g.accumulate) v += *p;
            *p = v;
          }
        }
      }
    } else {
      // part of a tile: into the slot of this segment
      double* P = sk.part + (long)(2 * w + (pos == begin ? 0 : 1)) * (BM * BN);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ml = wm * WTM + i * 16 + (lane >> 4) + 4 * r;
#pragma unroll
          for (int j = 0; j < NI; ++j) P[ml * BN + wn * WTN + j * 16 + (lane & 15)] = acc[i][j][r];
        }
    }
    pend = pos;
  }
}

// Float32 form of the split SI application (contraction precision f32): the
// same ranges of (tile, K-slice) space as gemm_streamk_f64 over 192 x 160
// tiles, with A (the enlarged corner) in float32, B (the float64 block)
// rounded to float32 on its way into LDS, 32-wide slices (the bytes of the
// float64 kernel's 16) and v_mfma_f32_16x16x4f32 with float32 accumulation.
// Whole tiles are widened to float64 on store; cut tiles leave their partial
// sums in float64 in the same scratch slots, summed by gemm_streamk_fixup.
namespace skf32 {
constexpr int BM = 192, BN = 160, BK = 32, WGM = 4, WGN = 2, NT = 64 * WGM * WGN;
constexpr int WTM = BM / WGM, WTN = BN / WGN;   // 48 x 80 per wavefront
constexpr int MI = WTM / 16, NI = WTN / 16;     // 3 x 5 accumulator blocks
constexpr int LT = BM + 16;                     // transposed A in LDS: [k][m]
constexpr int LN = BK + 1;                      // plain A in LDS: [m][k]
constexpr int ASZ = (BK * LT > BM * LN) ? BK * LT : BM * LN;
constexpr int LB = BN + 16;                     // B in LDS: [k][n]
constexpr int NA = BM * BK / 4;                 // 16-byte loads of A per slice (4 floats)
constexpr int NB = BK * BN / 2;                 // 16-byte loads of B per slice (2 doubles)
constexpr int VA = (NA + NT - 1) / NT, VB = (NB + NT - 1) / NT;
}  // namespace skf32

template <bool TRANS>
__device__ __forceinline__ void sk_segment_f32(const GemmBatch& g, int prob, int m0, int s0, int s1,
                                               float (*As)[skf32::ASZ],
                                               float (*Bs)[skf32::BK][skf32::LB],
                                               v4f (&acc)[skf32::MI][skf32::NI]) {
  using namespace skf32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int M = g.M, N = g.N, K = g.K;
  const float* A = (const float*)g.A[prob];
  const double* B = (const double*)g.B[prob];
  const long lda = g.lda, ldb = g.ldb;
  v4f ra[VA];
  v2d rb[VB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (i < NA) {
        if (TRANS) {
          const int gk = k0 + i / (BM / 4), gm = m0 + 4 * (i % (BM / 4));
          if (gk < K) {
            const float* q = A + (long)gk * lda + gm;
            if (gm + 3 < M) {
              v = *(const v4f*)q;
            } else {
              if (gm < M) v.x = q[0];
              if (gm + 1 < M) v.y = q[1];
              if (gm + 2 < M) v.z = q[2];
            }
          }
        } else {
          const int gm = m0 + i / (BK / 4), gk = k0 + 4 * (i % (BK / 4));
          if (gm < M) {
            const float* q = A + (long)gm * lda + gk;
            if (gk + 3 < K) {
              v = *(const v4f*)q;
            } else {
              if (gk < K) v.x = q[0];
              if (gk + 1 < K) v.y = q[1];
              if (gk + 2 < K) v.z = q[2];
            }
          }
        }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      const int gk = k0 + i / (BN / 2), gn = 2 * (i % (BN / 2));
      v2d v = {0.0, 0.0};
      if (i < NB && gk < K) {
        const double* q = B + (long)gk * ldb + gn;
        if (gn + 1 < N) v = *(const v2d*)q;
        else if (gn < N) v.x = q[0];
      }
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      if (i < NA) {
        if (TRANS) {
          const int kk = i / (BM / 4), m = 4 * (i % (BM / 4));
          *(v4f*)&As[buf][kk * LT + m] = ra[e];
        } else {
          const int m = i / (BK / 4), kk = 4 * (i % (BK / 4));
          float* q = &As[buf][m * LN + kk];
          q[0] = ra[e].x;
          q[1] = ra[e].y;
          q[2] = ra[e].z;
          q[3] = ra[e].w;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      if (i < NB) {
        float* q = &Bs[buf][i / (BN / 2)][2 * (i % (BN / 2))];
        q[0] = (float)rb[e].x;
        q[1] = (float)rb[e].y;
      }
    }
  };
  load(s0 * BK);
  store(0);
  __syncthreads();
  for (int kt = s0; kt < s1; ++kt) {
    const int buf = (kt - s0) & 1;
    if (kt + 1 < s1) load((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      float a[MI], b[NI];
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int m = wm * WTM + i * 16 + (lane & 15);
        a[i] = TRANS ? As[buf][kr * LT + m] : As[buf][m * LN + kr];
      }
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < s1) store(buf ^ 1);
    __syncthreads();
  }
}

__global__ __launch_bounds__(skf32::NT, 1) void gemm_streamk_f32(GemmBatch g, StreamK sk) {
  using namespace skf32;
  __shared__ float As[2][ASZ];
  __shared__ float Bs[2][BK][LB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const long begin = sk_begin(w, sk), end = sk_begin(w + 1, sk);
  const int M = g.M, N = g.N;
  // segments last to first, as in the float64 kernel
  long pend = end;
  while (pend > begin) {
    const long tile = (pend - 1) / sk.nslices;
    const long pos = tile * sk.nslices > begin ? tile * sk.nslices : begin;
    const int s0 = (int)(pos - tile * sk.nslices), s1 = (int)(pend - tile * sk.nslices);
    const int prob = (int)(tile / sk.tiles_m), m0 = (int)(tile % sk.tiles_m) * BM;
    v4f acc[MI][NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    if (g.transA[prob])
      sk_segment_f32<true>(g, prob, m0, s0, s1, As, Bs, acc);
    else
      sk_segment_f32<false>(g, prob, m0, s0, s1, As, Bs, acc);
    // float32 MFMA result element r of lane l: row 4 (l / 16) + r, column l % 16
    if (s0 == 0 && s1 == sk.nslices) {
      double* C = (double*)g.C[prob];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
          if (m >= M) continue;
          double* row = C + (long)m * g.cs_m0;
#pragma unroll
          for (int j = 0; j < NI; ++j) {
            const int n = wn * WTN + j * 16 + (lane & 15);
            if (n >= N) continue;
            double v = g.alpha * (double)acc[i][j][r];
            if (g.accumulate) v += row[n];
            row[n] = v;
          }
        }
      }
    } else {
      double* P = sk.part + (long)(2 * w + (pos == begin ? 0 : 1)) * (BM * BN);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ml = wm * WTM + i * 16 + 4 * (lane >> 4) + r;
#pragma unroll
          for (int j = 0; j < NI; ++j)
            P[ml * BN + wn * WTN + j * 16 + (lane & 15)] = (double)acc[i][j][r];
        }
    }
    pend = pos;
  }
}

// Sums the partial tiles of every tile cut by range boundaries, in
// workgroup order, and writes them through C's index map (alpha and
// accumulate as in the main kernel).  kFixRows-row strips of a tile per block
// of 256 threads, two adjacent columns per thread.  Ranges are never empty here (the
// split runs only with at least 8 slices per workgroup), so every workgroup
// between the first and the last owner of a tile left a partial in slot 2w.
constexpr int kFixRows = 24;

template <int BM, int BN>
__global__ __launch_bounds__(256) void gemm_streamk_fixup(GemmBatch g, StreamK sk) {
  static_assert(BM % kFixRows == 0 && BN % 2 == 0, "strip shape");
  const long tile = blockIdx.x / (BM / kFixRows);
  const int r0 = (blockIdx.x % (BM / kFixRows)) * kFixRows;
  const long t0 = tile * sk.nslices, t1 = t0 + sk.nslices;
  const int wf = sk_owner(t0, sk), wl = sk_owner(t1 - 1, sk);
  if (wf == wl) return;
  const int prob = (int)(tile / sk.tiles_m), m0 = (int)(tile % sk.tiles_m) * BM;
  const int first_slot = sk_begin(wf, sk) < t0 ? 2 * wf + 1 : 2 * wf;
  double* C = (double*)g.C[prob];
  constexpr int PR = BN / 2;   // column pairs per row
  for (int q = threadIdx.x; q < kFixRows * PR; q += 256) {
    const int ml = r0 + q / PR, n = 2 * (q % PR), m = m0 + ml;
    if (m >= g.M || n >= g.N) continue;
    const long e = (long)ml * BN + n;
    v2d v = *(const v2d*)&sk.part[(long)first_slot * (BM * BN) + e];
    for (int w = wf + 1; w <= wl; ++w) v += *(const v2d*)&sk.part[(long)(2 * w) * (BM * BN) + e];
    const bool two = n + 1 < g.N;
    const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
    double* p0 = C + offm + map2(n, g.cdiv_n, g.cs_n1, g.cs_n0);
    double* p1 = two ? C + offm + map2(n + 1, g.cdiv_n, g.cs_n1, g.cs_n0) : p0;
    double o0 = g.alpha * v.x, o1 = g.alpha * v.y;
    if (g.accumulate) {
      o0 += *p0;
      if (two) o1 += *p1;
    }
    *p0 = o0;
    if (two) *p1 = o1;
  }
}

template <int BM, int BN, int WGM, int WGN, int ROLE, bool ODD = false>
__global__ __launch_bounds__(64 * WGM * WGN, 512 / (64 * WGM * WGN)) void gemm_skinny_f64(
    GemmBatch g, int tiles_m, int tiles_n) {
  __shared__ double As[2][SkinnyA<BM, 16>::SIZE];
  __shared__ double Bs[2][16][BN + 16];
  const int per_prob = tiles_m * tiles_n;
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int prob = lin / per_prob / g.nbatch;
  if (g.transA[prob])
    skinny_tile<BM, BN, WGM, WGN, true, ODD>(g, tiles_m, tiles_n, lin, As, Bs);
  else
    skinny_tile<BM, BN, WGM, WGN, false, ODD>(g, tiles_m, tiles_n, lin, As, Bs);
}

// ---------------------------------------------------------------------------
// Grouped launches: the products of several GemmBatch descriptors of
// different shapes (one per context of a batched move) in one persistent
// launch.  The descriptors sit in device memory with the prefix sums of
// their work items (tiles x problems x inner batches); workgroup w takes
// items w, w + grid, ... and finds each one's descriptor by binary search.
// Every item runs the tile code of the ungrouped kernels, whose results do
// not depend on the grid, so a grouped product equals the same product
// launched alone, bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int group_of(const GroupItem* items, int n, long w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN, 512 / (64 * WGM * WGN)) void gemm_skinny_grouped(
    const GroupItem* items, int nitems, long total) {
  __shared__ double As[2][SkinnyA<BM, 16>::SIZE];
  __shared__ double Bs[2][16][BN + 16];
  for (long w = blockIdx.x; w < total; w += gridDim.x) {
    const GroupItem& it = items[group_of(items, nitems, w)];
    const int lin = (int)(w - it.first);
    const int prob = lin / (it.tiles_m * it.tiles_n) / it.g.nbatch;
    if (it.g.transA[prob])
      skinny_tile<BM, BN, WGM, WGN, true>(it.g, it.tiles_m, it.tiles_n, lin, As, Bs);
    else
      skinny_tile<BM, BN, WGM, WGN, false>(it.g, it.tiles_m, it.tiles_n, lin, As, Bs);
  }
}

template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_k4_grouped(const GroupItem* items, int nitems,
                                                       long total) {
  __shared__ double As[2][kK4BK][BM + kK4Pad];
  __shared__ double Bs[2][kK4BK][BN + kK4Pad];
  for (long w = blockIdx.x; w < total; w += gridDim.x) {
    const GroupItem& it = items[group_of(items, nitems, w)];
    const int lin = (int)(w - it.first);
    const int per = it.tiles_m * it.tiles_n;
    const int pb = lin / per, tile = lin % per;
    k4_tile<double, double, double, double, BM, BN, WGM, WGN>(
        it.g, pb / it.g.nbatch, pb % it.g.nbatch, tile / it.tiles_n, tile % it.tiles_n, As, Bs);
  }
}

// ---------------------------------------------------------------------------
// bf16 path: v_mfma_f32_16x16x32_bf16, float32 accumulation.
// LDS keeps k contiguous per row so that a lane reads its 8 k-values at once.
// ---------------------------------------------------------------------------
template <typename TA, typename TB, typename TC, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_bf16(GemmBatch g, int tiles_m, int tiles_n) {
  constexpr int BK = 32;
  constexpr int PAD = 8;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int MI = WTM / 16, NI = WTN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(WGM * WGN == 4, "four wavefronts");
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile multiple of 16");

  __shared__ __attribute__((aligned(16))) __bf16 As[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][BK + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = tile % tiles_n, tm = tile / tiles_n;
  const int prob = blockIdx.y / g.nbatch, batch = blockIdx.y % g.nbatch;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const int trans = g.transA[prob];
  const TA* A = (const TA*)g.A[prob] + (long)batch * g.a_bs;
  const TB* B = (const TB*)g.B[prob] + (long)batch * g.b_bs;
  TC* C = (TC*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  __bf16 ra[EA], rb[EB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int i = tid + e * 256;
      int m, kk;
      if (trans) { m = i % BM; kk = i / BM; } else { m = i / BK; kk = i % BK; }
      const int gm = m0 + m, gk = k0 + kk;
      __bf16 v = (__bf16)0.0f;
      if (gm < M && gk < K)
        v = cvt<__bf16>(trans ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk]);
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int i = tid + e * 256;
      const int n = i % BN, kk = i / BN;
      const int gn = n0 + n, gk = k0 + kk;
      __bf16 v = (__bf16)0.0f;
      if (gn < N && gk < K) v = cvt<__bf16>(B[(long)gk * ldb + gn]);
      rb[e] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int i = tid + e * 256;
      int m, kk;
      if (trans) { m = i % BM; kk = i / BM; } else { m = i / BK; kk = i % BK; }
      As[m][kk] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int i = tid + e * 256;
      Bs[i % BN][i / BN] = rb[e];
    }
  };

  v4f acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load_tiles(0);
  for (int kt = 0; kt < nk; ++kt) {
    store_tiles();
    __syncthreads();
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
    const int kc = 8 * (lane >> 4);
    v8bf a[MI], b[NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
      a[i] = *reinterpret_cast<const v8bf*>(&As[wm * WTM + i * 16 + (lane & 15)][kc]);
#pragma unroll
    for (int j = 0; j < NI; ++j)
      b[j] = *reinterpret_cast<const v8bf*>(&Bs[wn * WTN + j * 16 + (lane & 15)][kc]);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  long offn[NI];
  bool okn[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int n = n0 + wn * WTN + j * 16 + (lane & 15);
    okn[j] = n < N;
    offn[j] = okn[j] ? map2(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const float alpha = (float)g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
      if (m >= M) continue;
      const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        TC* p = C + offm + offn[j];
        float v = alpha * acc[i][j][r];
        if (g.accumulate) v += (float)*p;
        *p = cvt<TC>(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split bfloat16 path (three bf16 products per step): every operand value x
// is rounded to float32 and written as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (16 significant bits together); A B is then
// A_hi B_hi + A_hi B_lo + A_lo B_hi on v_mfma_f32_16x16x32_bf16 with float32
// accumulation, dropping only A_lo B_lo (relative 2^-16).  This keeps the
// bf16 matrix-core rate at close to float32 accuracy (Henry, Tang and
// Heinecke, ARITH 2019).  Same LDS layout as the bf16 path, hi and lo
// halves side by side.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <typename TA, typename TB, typename TC, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_bf16x3(GemmBatch g, int tiles_m, int tiles_n) {
  constexpr int BK = 32;
  constexpr int PAD = 8;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int MI = WTM / 16, NI = WTN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(WGM * WGN == 4, "four wavefronts");
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile multiple of 16");

  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Al[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[BN][BK + PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[BN][BK + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = tile % tiles_n, tm = tile / tiles_n;
  const int prob = blockIdx.y / g.nbatch, batch = blockIdx.y % g.nbatch;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const int trans = g.transA[prob];
  const TA* A = (const TA*)g.A[prob] + (long)batch * g.a_bs;
  const TB* B = (const TB*)g.B[prob] + (long)batch * g.b_bs;
  TC* C = (TC*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  float ra[EA], rb[EB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int i = tid + e * 256;
      int m, kk;
      if (trans) { m = i % BM; kk = i / BM; } else { m = i / BK; kk = i % BK; }
      const int gm = m0 + m, gk = k0 + kk;
      float v = 0.0f;
      if (gm < M && gk < K) v = (float)(trans ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk]);
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int i = tid + e * 256;
      const int n = i % BN, kk = i / BN;
      const int gn = n0 + n, gk = k0 + kk;
      float v = 0.0f;
      if (gn < N && gk < K) v = (float)B[(long)gk * ldb + gn];
      rb[e] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int i = tid + e * 256;
      int m, kk;
      if (trans) { m = i % BM; kk = i / BM; } else { m = i / BK; kk = i % BK; }
      split_bf16(ra[e], Ah[m][kk], Al[m][kk]);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int i = tid + e * 256;
      split_bf16(rb[e], Bh[i % BN][i / BN], Bl[i % BN][i / BN]);
    }
  };

  v4f acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load_tiles(0);
  for (int kt = 0; kt < nk; ++kt) {
    store_tiles();
    __syncthreads();
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
    const int kc = 8 * (lane >> 4);
    v8bf ah[MI], al[MI], bh[NI], bl[NI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      ah[i] = *reinterpret_cast<const v8bf*>(&Ah[wm * WTM + i * 16 + (lane & 15)][kc]);
      al[i] = *reinterpret_cast<const v8bf*>(&Al[wm * WTM + i * 16 + (lane & 15)][kc]);
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      bh[j] = *reinterpret_cast<const v8bf*>(&Bh[wn * WTN + j * 16 + (lane & 15)][kc]);
      bl[j] = *reinterpret_cast<const v8bf*>(&Bl[wn * WTN + j * 16 + (lane & 15)][kc]);
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }

  long offn[NI];
  bool okn[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int n = n0 + wn * WTN + j * 16 + (lane & 15);
    okn[j] = n < N;
    offn[j] = okn[j] ? map2(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const float alpha = (float)g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
      if (m >= M) continue;
      const long offm = map2(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        TC* p = C + offm + offn[j];
        float v = alpha * acc[i][j][r];
        if (g.accumulate) v += (float)*p;
        *p = cvt<TC>(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// tile selection
// ---------------------------------------------------------------------------
struct TileCfg {
  int bm, bn;
};

// Available (BM, BN) shapes; each has a fixed wavefront arrangement below.
constexpr TileCfg kTiles[] = {{128, 128}, {128, 144}, {64, 160}, {64, 80}, {64, 64}, {32, 32}};

int pick_tile(const GemmBatch& g) {
  int best = -1;
  double best_cost = 1e300;
  const long blocks_y = (long)g.count * g.nbatch;
  for (int c = 0; c < (int)(sizeof(kTiles) / sizeof(kTiles[0])); ++c) {
    const int bm = kTiles[c].bm, bn = kTiles[c].bn;
    const long tm = ceil_div(g.M, bm), tn = ceil_div(g.N, bn);
    const long wgs = tm * tn * blocks_y;
    // padded work, penalised when the grid cannot fill 256 compute units, and
    // slightly by the per-tile overhead of small tiles
    const double work = (double)tm * bm * tn * bn * blocks_y;
    const double fill = wgs >= 256 ? 1.0 : 256.0 / (double)wgs;
    const double small = 1.0 + 2048.0 / (double)(bm * bn);
    const double cost = work * fill * small;
    if (cost < best_cost) { best_cost = cost; best = c; }
  }
  return best;
}

template <typename TA, typename TB, typename TC, typename CT>
int launch_k4(const GemmBatch& g, hipStream_t s) {
  const int c = pick_tile(g);
  const int bm = kTiles[c].bm, bn = kTiles[c].bn;
  const int tm = ceil_div(g.M, bm), tn = ceil_div(g.N, bn);
  dim3 grid(tm * tn, g.count * g.nbatch), block(256);
  switch (c) {
    case 0: gemm_k4<TA, TB, TC, CT, 128, 128, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 1: gemm_k4<TA, TB, TC, CT, 128, 144, 4, 1><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 2: gemm_k4<TA, TB, TC, CT, 64, 160, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 3: gemm_k4<TA, TB, TC, CT, 64, 80, 4, 1><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 4: gemm_k4<TA, TB, TC, CT, 64, 64, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    default: gemm_k4<TA, TB, TC, CT, 32, 32, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
  }
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

template <typename TA, typename TB, typename TC>
int launch_b16(const GemmBatch& g, hipStream_t s) {
  const int c = pick_tile(g);
  const int bm = kTiles[c].bm, bn = kTiles[c].bn;
  const int tm = ceil_div(g.M, bm), tn = ceil_div(g.N, bn);
  dim3 grid(tm * tn, g.count * g.nbatch), block(256);
  switch (c) {
    case 0: gemm_bf16<TA, TB, TC, 128, 128, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 1: gemm_bf16<TA, TB, TC, 128, 144, 4, 1><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 2: gemm_bf16<TA, TB, TC, 64, 160, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 3: gemm_bf16<TA, TB, TC, 64, 80, 4, 1><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 4: gemm_bf16<TA, TB, TC, 64, 64, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    default: gemm_bf16<TA, TB, TC, 32, 32, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
  }
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

template <typename TA, typename TB, typename TC>
int launch_bx3(const GemmBatch& g, hipStream_t s) {
  const int c = pick_tile(g);
  const int bm = kTiles[c].bm, bn = kTiles[c].bn;
  const int tm = ceil_div(g.M, bm), tn = ceil_div(g.N, bn);
  dim3 grid(tm * tn, g.count * g.nbatch), block(256);
  switch (c) {
    case 0: gemm_bf16x3<TA, TB, TC, 128, 128, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 1: gemm_bf16x3<TA, TB, TC, 128, 144, 4, 1><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 2: gemm_bf16x3<TA, TB, TC, 64, 160, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 3: gemm_bf16x3<TA, TB, TC, 64, 80, 4, 1><<<grid, block, 0, s>>>(g, tm, tn); break;
    case 4: gemm_bf16x3<TA, TB, TC, 64, 64, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
    default: gemm_bf16x3<TA, TB, TC, 32, 32, 2, 2><<<grid, block, 0, s>>>(g, tm, tn); break;
  }
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

// The skinny kernel needs 16-byte aligned rows: even leading dimensions and
// batch strides, 16-byte aligned base pointers.
bool skinny_ok(const GemmBatch& g) {
  if ((g.lda & 1) || (g.ldb & 1) || (g.a_bs & 1) || (g.b_bs & 1)) return false;
  for (int i = 0; i < g.count; ++i)
    if (((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15)) return false;
  return true;
}

template <int BM, int BN, int WGM, int WGN, int ROLE, bool ODD = false>
int launch_skinny(const GemmBatch& g, hipStream_t s) {
  const int tm = ceil_div(g.M, BM), tn = ceil_div(g.N, BN);
  dim3 grid(tm * tn * g.count * g.nbatch), block(64 * WGM * WGN);
  gemm_skinny_f64<BM, BN, WGM, WGN, ROLE, ODD><<<grid, block, 0, s>>>(g, tm, tn);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace

int grouped_kind(const GemmBatch* gs, int n) {
  bool skinny = true;
  int big = 0;
  double most = -1.0;
  for (int i = 0; i < n; ++i) {
    skinny = skinny && gs[i].N <= 160 && skinny_ok(gs[i]);
    const double f = (double)gs[i].M * gs[i].N * (double)gs[i].K * gs[i].count * gs[i].nbatch;
    if (f > most) { most = f; big = i; }
  }
  if (skinny) return 0;
  return 1 + pick_tile(gs[big]);
}

long grouped_fill(const GemmBatch* gs, int n, int kind, GroupItem* items) {
  const int bm = kind == 0 ? 96 : kTiles[kind - 1].bm, bn = kind == 0 ? 160 : kTiles[kind - 1].bn;
  long total = 0;
  for (int i = 0; i < n; ++i) {
    items[i].g = gs[i];
    items[i].tiles_m = gs[i].M > 0 ? ceil_div(gs[i].M, bm) : 0;
    items[i].tiles_n = gs[i].N > 0 ? ceil_div(gs[i].N, bn) : 0;
    items[i].first = total;
    total += (long)items[i].tiles_m * items[i].tiles_n * gs[i].count * gs[i].nbatch;
  }
  return total;
}

int launch_gemm_grouped(const GroupItem* items, int n, long total, int kind, hipStream_t s) {
  if (n <= 0 || total <= 0) return 0;
  // persistent grid: at most two workgroups per CU of 256
  const int grid = (int)std::min<long>(total, 512);
  if (kind == 0) {
    gemm_skinny_grouped<96, 160, 2, 2><<<grid, 256, 0, s>>>(items, n, total);
  } else {
    switch (kind - 1) {
      case 0: gemm_k4_grouped<128, 128, 2, 2><<<grid, 256, 0, s>>>(items, n, total); break;
      case 1: gemm_k4_grouped<128, 144, 4, 1><<<grid, 256, 0, s>>>(items, n, total); break;
      case 2: gemm_k4_grouped<64, 160, 2, 2><<<grid, 256, 0, s>>>(items, n, total); break;
      case 3: gemm_k4_grouped<64, 80, 4, 1><<<grid, 256, 0, s>>>(items, n, total); break;
      case 4: gemm_k4_grouped<64, 64, 2, 2><<<grid, 256, 0, s>>>(items, n, total); break;
      default: gemm_k4_grouped<32, 32, 2, 2><<<grid, 256, 0, s>>>(items, n, total); break;
    }
  }
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int launch_gemm_si(const GemmBatch& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch <= 0) return 0;
  if (g.N > 160 || !skinny_ok(g)) return launch_gemm(g, DT::F64, DT::F64, DT::F64, s);
  return launch_skinny<96, 160, 2, 2, 1>(g, s);
}

size_t gemm_si_scratch_bytes() { return (size_t)2 * kSplitMaxCus * 192 * 160 * sizeof(double); }

// Ranges of the split: ncu, or fewer so that each holds at least 8 slices.
static int sk_ranges(long pairs, int ncu) { return (int)std::min<long>(ncu, pairs / 8); }

bool gemm_si_balanced_useful(int count, int M, int N, int K, int ncu) {
  // the split pays whenever each tile holds several slices: its ranges keep
  // every CU busy for the same time whatever the tile count, where the
  // plain kernel leaves CUs idle through whole K walks once the tiles are
  // fewer than the slots or do not divide them
  if (ncu < 1 || ncu > kSplitMaxCus || N > 160 || M <= 0 || count <= 0 || K <= 0) return false;
  const long tiles = (long)ceil_div(M, 192) * count, ns = ceil_div(K, 16);
  return ns >= 16 && sk_ranges(tiles * ns, ncu) >= 1;
}

// The split kernel's operands: A as the skinny kernel's (even lda, 16-byte
// aligned rows); B with an even ldb on 16-byte aligned bases, or with an odd
// one on 8-byte aligned bases (loaded one element at a time).
static bool streamk_ok(const GemmBatch& g) {
  if ((g.lda & 1) || (g.a_bs & 1)) return false;
  const uintptr_t balign = (g.ldb & 1) ? 7 : 15;
  for (int i = 0; i < g.count; ++i)
    if (((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & balign)) return false;
  return true;
}

bool gemm_si_balanced_applies(const GemmBatch& g, const void* scratch, int ncu) {
  if (!scratch || ((uintptr_t)scratch & 15) || g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch != 1)
    return false;
  return gemm_si_balanced_useful(g.count, g.M, g.N, g.K, ncu) && streamk_ok(g) &&
         (long)g.count * ceil_div(g.M, 192) * ceil_div(g.K, 16) <= (1L << 40);
}

template <int BN, bool BODD>
static int launch_streamk_f64(const GemmBatch& g, const StreamK& sk, hipStream_t s) {
  gemm_streamk_f64<192, BN, 4, 2, BODD><<<sk.nwg, 512, 0, s>>>(g, sk);
  CTM_HIP_TRY(hipGetLastError());
  gemm_streamk_fixup<192, BN><<<(int)((long)g.count * sk.tiles_m * (192 / kFixRows)), 256, 0, s>>>(g, sk);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int launch_gemm_si_balanced(const GemmBatch& g, double* scratch, int ncu, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch <= 0) return 0;
  if (!gemm_si_balanced_applies(g, scratch, ncu)) return launch_gemm_si(g, s);
  const int tm = ceil_div(g.M, 192);
  const int ns = ceil_div(g.K, 16);
  StreamK sk;
  sk.nslices = ns;
  sk.tiles_m = tm;
  sk.total = (long)g.count * tm * ns;
  sk.nwg = sk_ranges(sk.total, ncu);
  sk.part = scratch;
  // 128-wide tiles for N <= 128 (3 x 4 accumulator blocks of 16 x 16 per
  // wavefront): less of the MFMA work is padding
  const bool odd = g.ldb & 1;
  if (g.N <= 128) return odd ? launch_streamk_f64<128, true>(g, sk, s) : launch_streamk_f64<128, false>(g, sk, s);
  return odd ? launch_streamk_f64<160, true>(g, sk, s) : launch_streamk_f64<160, false>(g, sk, s);
}

int launch_gemm_f64_any(const GemmBatch& g, double* scratch, int ncu, hipStream_t s) {
  if (gemm_si_balanced_applies(g, scratch, ncu)) return launch_gemm_si_balanced(g, scratch, ncu, s);
  return launch_gemm(g, DT::F64, DT::F64, DT::F64, s);
}

bool gemm_si_f32_balanced_applies(const GemmBatch& g, const void* scratch, int ncu) {
  if (!scratch || ((uintptr_t)scratch & 15) || g.M <= 0 || g.N <= 0 || g.count <= 0 ||
      g.nbatch != 1 || g.N > skf32::BN)
    return false;
  if ((g.lda & 3) || (g.ldb & 1)) return false;
  for (int i = 0; i < g.count; ++i)
    if (((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15)) return false;
  const bool rowmajor_c = g.cdiv_m >= g.M && g.cdiv_n >= g.N && g.cs_n0 == 1;
  // at least 8 slices per range, so that no range is empty, and 8 per tile
  const long tiles = (long)g.count * ceil_div(g.M, skf32::BM), ns = ceil_div(g.K, skf32::BK);
  return rowmajor_c && ncu >= 1 && ncu <= kSplitMaxCus && ns >= 8 && tiles * ns >= 8L * ncu &&
         tiles * ns <= (1L << 40);
}

int launch_gemm_si_f32_balanced(const GemmBatch& g, double* scratch, int ncu, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch <= 0) return 0;
  if (!gemm_si_f32_balanced_applies(g, scratch, ncu)) return launch_gemm_si_f32(g, s);
  const int tm = ceil_div(g.M, skf32::BM);
  StreamK sk;
  sk.nslices = ceil_div(g.K, skf32::BK);
  sk.tiles_m = tm;
  sk.total = (long)g.count * tm * sk.nslices;
  sk.nwg = ncu;
  sk.part = scratch;
  gemm_streamk_f32<<<ncu, skf32::NT, 0, s>>>(g, sk);
  CTM_HIP_TRY(hipGetLastError());
  gemm_streamk_fixup<192, 160><<<(int)((long)g.count * tm * (192 / kFixRows)), 256, 0, s>>>(g, sk);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

namespace {
// 8-byte aligned pairs of float32 / float64 operands for the float32 skinny tile.
bool pairs_ok(const GemmBatch& g) {
  if ((g.lda & 1) || (g.ldb & 1) || (g.a_bs & 1) || (g.b_bs & 1)) return false;
  for (int i = 0; i < g.count; ++i)
    if (((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15)) return false;
  return true;
}

// float32 contractions long enough for the double-buffered float32 tile
// (the same shape rule as the float64 one below).
template <typename TA, typename TB, typename TC>
bool launch_f32_db(const GemmBatch& g, hipStream_t s, int* rc) {
  if (g.K < 512 || g.M < 256 || !pairs_ok(g)) return false;
  auto go = [&](auto kern, int bm, int bn, int threads) {
    const int tm = ceil_div(g.M, bm), tn = ceil_div(g.N, bn);
    kern<<<dim3(tm * tn * g.count * g.nbatch), dim3(threads), 0, s>>>(g, tm, tn);
    const hipError_t e = hipGetLastError();
    *rc = e == hipSuccess ? 0 : hip_fail(e, "float32 skinny tile", __LINE__);
  };
  if (g.N <= 160)
    go(gemm_skinny_f32x<TA, TB, TC, 96, 160, 2, 2>, 96, 160, 256);
  else if ((long)g.M * g.count * g.nbatch >= 16384)
    go(gemm_skinny_f32x<TA, TB, TC, 256, 144, 8, 1>, 256, 144, 512);
  else
    go(gemm_skinny_f32x<TA, TB, TC, 128, 144, 4, 1>, 128, 144, 256);
  return true;
}

// float64 GEMMs long enough for the double-buffered tiles: N <= 160 takes
// the 96 x 160 tile, wider N the 128 x 144 tile (144 divides the D^4 = 1296
// columns of the double-layer absorptions at D = 6).
bool launch_f64_db(const GemmBatch& g, hipStream_t s, int* rc) {
  // short K (a few slices per tile) gains nothing from the double buffer,
  // except on the wide products with many rows (the corner stems, K = chi),
  // which the 256 x 144 tile covers with fewer, fuller workgroups
  const bool wide = g.K >= 128 && g.N > 160 && (long)g.M * g.count * g.nbatch >= 16384;
  if ((g.K < 512 && !wide) || g.M < 256) return false;
  // odd leading dimensions or batch strides: the same tiles with operand
  // pairs loaded one element at a time
  if (!skinny_ok(g)) {
    if (g.N <= 160)
      *rc = launch_skinny<96, 160, 2, 2, 0, true>(g, s);
    else if ((long)g.M * g.count * g.nbatch >= 16384)
      *rc = launch_skinny<256, 144, 8, 1, 0, true>(g, s);
    else
      *rc = launch_skinny<128, 144, 4, 1, 0, true>(g, s);
    return true;
  }
  if (g.N <= 160)
    *rc = launch_skinny<96, 160, 2, 2, 0>(g, s);
  else if ((long)g.M * g.count * g.nbatch >= 16384)
    *rc = launch_skinny<256, 144, 8, 1, 0>(g, s);
  else
    *rc = launch_skinny<128, 144, 4, 1, 0>(g, s);
  return true;
}
}  // namespace

// Compute type: float64 when any operand is float64 and the mode is f64;
// the caller selects the mode through the operand types:
//   (F64, F64, *)   -> float64 MFMA
//   (F32, *, *)     -> float32 MFMA (f64 B operands are rounded to f32)
//   (BF16, *, *)    -> bf16 MFMA with f32 accumulation
int launch_gemm(const GemmBatch& g, DT ta, DT tb, DT tc, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch <= 0) return 0;
  if (g.K <= 0 && !g.accumulate) {
    // empty sum: the kernels still write zeros (load loop does not run)
  }
  if (g.split) {
    // split bfloat16 products of float32-stored contraction operands
    if (ta == DT::F64 && tb == DT::F32 && tc == DT::F32) return launch_bx3<double, float, float>(g, s);
    if (ta == DT::F32 && tb == DT::F64 && tc == DT::F64) return launch_bx3<float, double, double>(g, s);
    if (ta == DT::F32 && tb == DT::F32 && tc == DT::F64) return launch_bx3<float, float, double>(g, s);
    if (ta == DT::F64 && tb == DT::F32 && tc == DT::F64) return launch_bx3<double, float, double>(g, s);
    set_thread_error("launch_gemm: unsupported type combination for split bfloat16");
    return 1;
  }
  if (ta == DT::F64 && tb == DT::F64) {
    int rc = 0;
    if (tc == DT::F64 && launch_f64_db(g, s, &rc)) return rc;
    if (tc == DT::F64) return launch_k4<double, double, double, double>(g, s);
    if (tc == DT::F32) return launch_k4<double, double, float, double>(g, s);
  }
  {
    // the float32 contractions with long K on the double-buffered tile
    int rc = 0;
    if (ta == DT::F32 && tb == DT::F64 && tc == DT::F64 &&
        launch_f32_db<float, double, double>(g, s, &rc))
      return rc;
    if (ta == DT::F64 && tb == DT::F32 && tc == DT::F32 &&
        launch_f32_db<double, float, float>(g, s, &rc))
      return rc;
    if (ta == DT::F64 && tb == DT::F32 && tc == DT::F64 &&
        launch_f32_db<double, float, double>(g, s, &rc))
      return rc;
  }
  if (ta == DT::F32) {
    if (tb == DT::F64 && tc == DT::F64) return launch_k4<float, double, double, float>(g, s);
    if (tb == DT::F64 && tc == DT::F32) return launch_k4<float, double, float, float>(g, s);
    if (tb == DT::F32 && tc == DT::F32) return launch_k4<float, float, float, float>(g, s);
    if (tb == DT::F32 && tc == DT::F64) return launch_k4<float, float, double, float>(g, s);
  }
  if (ta == DT::F64 && tb == DT::F32) {
    if (tc == DT::F32) return launch_k4<double, float, float, float>(g, s);
    if (tc == DT::F64) return launch_k4<double, float, double, float>(g, s);
  }
  if (ta == DT::F64 && tb == DT::BF16) {
    if (tc == DT::BF16) return launch_b16<double, __bf16, __bf16>(g, s);
    if (tc == DT::F32) return launch_b16<double, __bf16, float>(g, s);
    if (tc == DT::F64) return launch_b16<double, __bf16, double>(g, s);
  }
  if (ta == DT::F64 && tb == DT::F32 && tc == DT::BF16) return launch_k4<double, float, __bf16, float>(g, s);
  if (ta == DT::BF16) {
    if (tb == DT::BF16 && tc == DT::F64) return launch_b16<__bf16, __bf16, double>(g, s);
    if (tb == DT::F64 && tc == DT::F64) return launch_b16<__bf16, double, double>(g, s);
    if (tb == DT::F64 && tc == DT::F32) return launch_b16<__bf16, double, float>(g, s);
    if (tb == DT::F32 && tc == DT::F32) return launch_b16<__bf16, float, float>(g, s);
    if (tb == DT::F32 && tc == DT::F64) return launch_b16<__bf16, float, double>(g, s);
  }
  if (ta == DT::F64 && tb == DT::F64 && tc == DT::BF16)
    return launch_k4<double, double, __bf16, double>(g, s);
  if (ta == DT::F64 && tb == DT::F64) return launch_k4<double, double, double, double>(g, s);
  set_thread_error("launch_gemm: unsupported type combination");
  return 1;
}

}  // namespace sictm
