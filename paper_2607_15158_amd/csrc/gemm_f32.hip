// Float32 and split-bfloat16 contractions of the enlarged-corner
// applications (the precision split of the contractions): C (float64, M x N) = op(A) B with A the
// enlarged corner stored in float32 (M x K, or K x M when transposed) and
// B the float64 isometry block (K x N, N <= 160), rounded to float32 on its
// way into LDS; v_mfma_f32_16x16x4f32 with float32 accumulation, the result
// widened to float64.  One workgroup owns a 96 x 160 tile (the whole width of
// the block), so A is streamed from HBM once per application; K is staged
// through double-buffered LDS in 32-wide slices (the same bytes per slice as
// the float64 tile's 16) with 16-byte global loads and one barrier per slice;
// the flattened (problem, tile) grid is dealt to the XCDs in contiguous
// chunks so that one problem's workgroups share an L2.

#include "common.h"

namespace sictm {
namespace {

typedef double v2d32 __attribute__((ext_vector_type(2)));
typedef float v2f32 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int xcd_chunk(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ long map2f(int i, int div, long s1, long s0) {
  return (long)(i / div) * s1 + (long)(i % div) * s0;
}

constexpr int BM = 96, BN = 160, BK = 32, WGM = 2, WGN = 2, NT = 256;
constexpr int WTM = BM / WGM, WTN = BN / WGN;   // 48 x 80 per wavefront
constexpr int MI = WTM / 16, NI = WTN / 16;     // 3 x 5 accumulator tiles
constexpr int LT = BM + 16;                     // transposed A in LDS: [k][m]
constexpr int LN = BK + 1;                      // plain A in LDS: [m][k]
constexpr int ASZ = (BK * LT > BM * LN) ? BK * LT : BM * LN;
constexpr int LB = BN + 16;                     // B in LDS: [k][n]
constexpr int NA = BM * BK / 4;                 // 16-byte loads of A per slice (4 floats)
constexpr int NB = BK * BN / 2;                 // 16-byte loads of B per slice (2 doubles)
constexpr int VA = (NA + NT - 1) / NT, VB = (NB + NT - 1) / NT;

template <bool TRANS>
__device__ __forceinline__ void tile32(const GemmBatch& g, int tiles_m, int tiles_n,
                                       float (*As)[ASZ], float (*Bs)[BK][LB]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int per_prob = tiles_m * tiles_n;
  const int lin = xcd_chunk(blockIdx.x, gridDim.x);
  const int pb = lin / per_prob, tile = lin % per_prob;
  const int prob = pb / g.nbatch, batch = pb % g.nbatch;
  const int tn = tile % tiles_n, tm = tile / tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const float* A = (const float*)g.A[prob] + (long)batch * g.a_bs;
  const double* B = (const double*)g.B[prob] + (long)batch * g.b_bs;
  double* C = (double*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  v4f ra[VA];
  v2d32 rb[VB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < VA; ++e) {
      const int i = tid + e * NT;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (i < NA) {
        if (TRANS) {
          const int gk = k0 + i / (BM / 4), gm = m0 + 4 * (i % (BM / 4));
          if (gk < K) {
            const float* p = A + (long)gk * lda + gm;
            if (gm + 3 < M) {
              v = *(const v4f*)p;
            } else {
              if (gm < M) v.x = p[0];
              if (gm + 1 < M) v.y = p[1];
              if (gm + 2 < M) v.z = p[2];
            }
          }
        } else {
          const int gm = m0 + i / (BK / 4), gk = k0 + 4 * (i % (BK / 4));
          if (gm < M) {
            const float* p = A + (long)gm * lda + gk;
            if (gk + 3 < K) {
              v = *(const v4f*)p;
            } else {
              if (gk < K) v.x = p[0];
              if (gk + 1 < K) v.y = p[1];
              if (gk + 2 < K) v.z = p[2];
            }
          }
        }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < VB; ++e) {
      const int i = tid + e * NT;
      const int gk = k0 + i / (BN / 2), gn = n0 + 2 * (i % (BN / 2));
      v2d32 v = {0.0, 0.0};
      if (i < NB && gk < K) {
        const double* p = B + (long)gk * ldb + gn;
        if (gn + 1 < N) v = *(const v2d32*)p;
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
        const v2f32 f = {(float)rb[e].x, (float)rb[e].y};
        *(v2f32*)&Bs[buf][i / (BN / 2)][2 * (i % (BN / 2))] = f;
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
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // epilogue: float32 MFMA result element r of lane l is row 4 (l / 16) + r,
  // column l % 16 of the 16 x 16 block; two-level output map, float64 store
  long offn[NI];
  bool okn[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int n = n0 + wn * WTN + j * 16 + (lane & 15);
    okn[j] = n < N;
    offn[j] = okn[j] ? map2f(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const double alpha = g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
      if (m >= M) continue;
      const long offm = map2f(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        double* p = C + offm + offn[j];
        double v = alpha * (double)acc[i][j][r];
        if (g.accumulate) v += *p;
        *p = v;
      }
    }
  }
}

__global__ __launch_bounds__(NT, 2) void gemm_skinny_f32(GemmBatch g, int tiles_m, int tiles_n) {
  __shared__ float As[2][ASZ];
  __shared__ float Bs[2][BK][LB];
  const int per_prob = tiles_m * tiles_n;
  const int prob = xcd_chunk(blockIdx.x, gridDim.x) / per_prob / g.nbatch;
  if (g.transA[prob])
    tile32<true>(g, tiles_m, tiles_n, As, Bs);
  else
    tile32<false>(g, tiles_m, tiles_n, As, Bs);
}

bool f32_ok(const GemmBatch& g) {
  if ((g.lda & 3) || (g.ldb & 1) || (g.a_bs & 3) || (g.b_bs & 1)) return false;
  for (int i = 0; i < g.count; ++i)
    if (((uintptr_t)g.A[i] & 15) || ((uintptr_t)g.B[i] & 15)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Split bfloat16 form of the same product (contraction precision
// CTM_PREC_BF16X3): A float32, B float64; every value is rounded to float32
// and written into LDS as hi = bf16(x) and lo = bf16(x - hi), k contiguous
// per row (the operand layout of v_mfma_f32_16x16x32_bf16: lane l reads 8
// consecutive k of row l % 16, starting at 8 (l / 16)); each 32-wide slice
// then takes three bf16 products per 16 x 16 block, lo*hi + hi*lo + hi*hi,
// accumulated in float32 (Henry, Tang and Heinecke, ARITH 2019).
// ---------------------------------------------------------------------------
typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf16 __attribute__((ext_vector_type(4)));
constexpr int XBK = 32;                 // k per slice (one bf16 MFMA step)
constexpr int XL = XBK + 8;             // LDS row length (bf16): 80 bytes
constexpr int XNA = BM * XBK / 4;       // 16-byte loads of A per slice
constexpr int XNB = XBK * BN / 2;       // 16-byte loads of B per slice
constexpr int XVA = (XNA + NT - 1) / NT, XVB = (XNB + NT - 1) / NT;

struct X3Lds {
  __bf16 ah[2][BM][XL], al[2][BM][XL];
  __bf16 bh[2][BN][XL], bl[2][BN][XL];
};

__device__ __forceinline__ void split2(float x, __bf16& h, __bf16& l) {
  h = (__bf16)x;
  l = (__bf16)(x - (float)h);
}

template <bool TRANS>
__device__ __forceinline__ void tile_x3(const GemmBatch& g, int tiles_m, int tiles_n, X3Lds& L) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int per_prob = tiles_m * tiles_n;
  const int lin = xcd_chunk(blockIdx.x, gridDim.x);
  const int pb = lin / per_prob, tile = lin % per_prob;
  const int prob = pb / g.nbatch, batch = pb % g.nbatch;
  const int tn = tile % tiles_n, tm = tile / tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = g.M, N = g.N, K = g.K;
  const float* A = (const float*)g.A[prob] + (long)batch * g.a_bs;
  const double* B = (const double*)g.B[prob] + (long)batch * g.b_bs;
  double* C = (double*)g.C[prob] + (long)batch * g.c_bs;
  const long lda = g.lda, ldb = g.ldb;

  v4f ra[XVA];
  v2d32 rb[XVB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < XVA; ++e) {
      const int i = tid + e * NT;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (i < XNA) {
        if (TRANS) {
          const int gk = k0 + i / (BM / 4), gm = m0 + 4 * (i % (BM / 4));
          if (gk < K) {
            const float* p = A + (long)gk * lda + gm;
            if (gm + 3 < M) {
              v = *(const v4f*)p;
            } else {
              if (gm < M) v.x = p[0];
              if (gm + 1 < M) v.y = p[1];
              if (gm + 2 < M) v.z = p[2];
            }
          }
        } else {
          const int gm = m0 + i / (XBK / 4), gk = k0 + 4 * (i % (XBK / 4));
          if (gm < M) {
            const float* p = A + (long)gm * lda + gk;
            if (gk + 3 < K) {
              v = *(const v4f*)p;
            } else {
              if (gk < K) v.x = p[0];
              if (gk + 1 < K) v.y = p[1];
              if (gk + 2 < K) v.z = p[2];
            }
          }
        }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < XVB; ++e) {
      const int i = tid + e * NT;
      const int gk = k0 + i / (BN / 2), gn = n0 + 2 * (i % (BN / 2));
      v2d32 v = {0.0, 0.0};
      if (i < XNB && gk < K) {
        const double* p = B + (long)gk * ldb + gn;
        if (gn + 1 < N) v = *(const v2d32*)p;
        else if (gn < N) v.x = p[0];
      }
      rb[e] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < XVA; ++e) {
      const int i = tid + e * NT;
      if (i < XNA) {
        const float x[4] = {ra[e].x, ra[e].y, ra[e].z, ra[e].w};
        if (TRANS) {
          const int kk = i / (BM / 4), m = 4 * (i % (BM / 4));
#pragma unroll
          for (int q = 0; q < 4; ++q) split2(x[q], L.ah[buf][m + q][kk], L.al[buf][m + q][kk]);
        } else {
          const int m = i / (XBK / 4), kk = 4 * (i % (XBK / 4));
          v4bf16 h, l;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            __bf16 hq, lq;
            split2(x[q], hq, lq);
            h[q] = hq;
            l[q] = lq;
          }
          *(v4bf16*)&L.ah[buf][m][kk] = h;
          *(v4bf16*)&L.al[buf][m][kk] = l;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < XVB; ++e) {
      const int i = tid + e * NT;
      if (i < XNB) {
        const int kk = i / (BN / 2), n = 2 * (i % (BN / 2));
        split2((float)rb[e].x, L.bh[buf][n][kk], L.bl[buf][n][kk]);
        split2((float)rb[e].y, L.bh[buf][n + 1][kk], L.bl[buf][n + 1][kk]);
      }
    }
  };

  v4f acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + XBK - 1) / XBK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * XBK);
    const int kc = 8 * (lane >> 4);
    v8bf16 ah[MI], al[MI], bh[NI], bl[NI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int m = wm * WTM + i * 16 + (lane & 15);
      ah[i] = *(const v8bf16*)&L.ah[buf][m][kc];
      al[i] = *(const v8bf16*)&L.al[buf][m][kc];
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int n = wn * WTN + j * 16 + (lane & 15);
      bh[j] = *(const v8bf16*)&L.bh[buf][n][kc];
      bl[j] = *(const v8bf16*)&L.bl[buf][n][kc];
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
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
    offn[j] = okn[j] ? map2f(n, g.cdiv_n, g.cs_n1, g.cs_n0) : 0;
  }
  const double alpha = g.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
      if (m >= M) continue;
      const long offm = map2f(m, g.cdiv_m, g.cs_m1, g.cs_m0);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if (!okn[j]) continue;
        double* p = C + offm + offn[j];
        double v = alpha * (double)acc[i][j][r];
        if (g.accumulate) v += *p;
        *p = v;
      }
    }
  }
}

__global__ __launch_bounds__(NT, 2) void gemm_skinny_bx3(GemmBatch g, int tiles_m, int tiles_n) {
  __shared__ X3Lds L;
  const int per_prob = tiles_m * tiles_n;
  const int prob = xcd_chunk(blockIdx.x, gridDim.x) / per_prob / g.nbatch;
  if (g.transA[prob])
    tile_x3<true>(g, tiles_m, tiles_n, L);
  else
    tile_x3<false>(g, tiles_m, tiles_n, L);
}

}  // namespace

int launch_gemm_si_bx3(const GemmBatch& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch <= 0) return 0;
  if (g.N > BN || !f32_ok(g)) {
    GemmBatch gs = g;
    gs.split = 1;
    return launch_gemm(gs, DT::F32, DT::F64, DT::F64, s);
  }
  const int tm = ceil_div(g.M, BM), tn = ceil_div(g.N, BN);
  dim3 grid(tm * tn * g.count * g.nbatch), block(NT);
  gemm_skinny_bx3<<<grid, block, 0, s>>>(g, tm, tn);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int launch_gemm_si_f32(const GemmBatch& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.count <= 0 || g.nbatch <= 0) return 0;
  if (g.N > BN || !f32_ok(g)) return launch_gemm(g, DT::F32, DT::F64, DT::F64, s);
  const int tm = ceil_div(g.M, BM), tn = ceil_div(g.N, BN);
  dim3 grid(tm * tn * g.count * g.nbatch), block(NT);
  gemm_skinny_f32<<<grid, block, 0, s>>>(g, tm, tn);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace sictm
