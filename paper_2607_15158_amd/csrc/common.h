// Shared definitions of the SI-CTMRG HIP library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>
#include <string>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Cross-lane sums of doubles without LDS round trips.  DPP moves act on
// 32-bit halves; the patterns below pair every lane with a partner, so each
// stage adds the same two values in every lane and all lanes end with
// bitwise identical sums.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// Sum over each aligned group of 16 lanes, in every lane of the group:
// quad_perm(1,0,3,2), quad_perm(2,3,0,1), row_half_mirror, row_mirror.
__device__ __forceinline__ double row_sum16(double x) {
  x += dpp_mov_f64<0xB1>(x);
  x += dpp_mov_f64<0x4E>(x);
  x += dpp_mov_f64<0x141>(x);
  x += dpp_mov_f64<0x140>(x);
  return x;
}

// Sum over the 64 lanes of a wavefront (uniform result).
__device__ __forceinline__ double wave_sum64(double x) {
  x = row_sum16(x);
  return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

// Exchange of two doubles between lanes L and L ^ 32 (gfx950 permlane32
// swap: the upper half of `a` trades places with the lower half of `b`).
// After the call a + b holds, in every lane, its own value of the half it
// keeps (a for lanes < 32, b for lanes >= 32) plus the partner's value of
// the same half.
__device__ __forceinline__ void swap_halves32(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// The same between L and L ^ 16 (permlane16 swap: the odd 16-lane rows of
// `a` trade places with the even rows of `b`).
__device__ __forceinline__ void swap_halves16(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// One halving level through a DPP pattern whose partner differs from the
// lane in bit `bit`: the lane keeps `lo` (bit clear) or `hi` (bit set) and
// adds the partner's value of the same half.
template <int CTRL>
__device__ __forceinline__ double dpp_halve(double lo, double hi, bool bit) {
  const double send = bit ? lo : hi;
  return (bit ? hi : lo) + dpp_mov_f64<CTRL>(send);
}

// Transpose-reduction of 32 per-lane values p(0..31) over the wavefront:
// lane L returns the sum over all 64 lanes of p(L >> 1).  Each level halves
// the values a lane holds by trading half of them with a partner lane: L^32
// and L^16 by the permlane swaps, then L^8 (row_ror:8), L^7 (row_half_mirror)
// and L^3 (quad_perm 3,2,1,0) by DPP, the kept half chosen by bits 5..1 of
// L; a last exchange with L^1 (quad_perm 1,0,3,2) completes the sum.  The
// six partner masks are linearly independent over GF(2), so every lane's
// contribution enters each result exactly once.  p(s) is evaluated in pairs
// (s, s + 16) as the first level consumes them.
template <typename PF>
__device__ __forceinline__ double wave_xsum32(const PF& p, int lane) {
  double q[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    double a = p(s), b = p(s + 16);
    swap_halves32(a, b);
    q[s] = a + b;
  }
  double r[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    double a = q[s], b = q[s + 8];
    swap_halves16(a, b);
    r[s] = a + b;
  }
  double t[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) t[s] = dpp_halve<0x128>(r[s], r[s + 4], (lane >> 3) & 1);
  double u[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) u[s] = dpp_halve<0x141>(t[s], t[s + 2], (lane >> 2) & 1);
  const double v = dpp_halve<0x1B>(u[0], u[1], (lane >> 1) & 1);
  return v + dpp_mov_f64<0xB1>(v);
}

#define CTM_HIP_TRY(expr)                                              \
  do {                                                                 \
    hipError_t _e = (expr);                                            \
    if (_e != hipSuccess) return ::sictm::hip_fail(_e, #expr, __LINE__); \
  } while (0)

namespace sictm {

// Records the failing call in a thread-local message and returns CTM_E_DEVICE.
int hip_fail(hipError_t e, const char* what, int line);
const std::string& thread_error();
void set_thread_error(const std::string& s);

constexpr int kWave = 64;

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// GEMM descriptor: C_p[map_c(m, n) + batch*c_bs] = alpha * sum_k A(m,k) B(k,n)
// for up to kMaxProb problems p with identical shapes.  A(m,k) is
// A_p[m*lda + k] (trans 0) or A_p[k*lda + m] (trans 1), per problem.  B(k,n)
// is B_p[k*ldb + n].  The output map is two-level in m and in n:
//   off(m) = (m / cdiv_m) * cs_m1 + (m % cdiv_m) * cs_m0, same for n.
// ---------------------------------------------------------------------------
constexpr int kMaxProb = 8;

struct GemmBatch {
  const void* A[kMaxProb];
  const void* B[kMaxProb];
  void* C[kMaxProb];
  int transA[kMaxProb];
  int count;          // problems
  int M, N, K;
  long lda, ldb;
  int cdiv_m;
  long cs_m1, cs_m0;
  int cdiv_n;
  long cs_n1, cs_n0;
  int nbatch;         // inner batch per problem
  long a_bs, b_bs, c_bs;
  double alpha;
  int accumulate;     // 1: C += alpha*AB
  int split;          // 1: float32 operands as hi + lo bfloat16, three bf16 products
};

// Element types of a GEMM launch.
enum class DT : int { F64 = 0, F32 = 1, BF16 = 2 };

// Plain row-major output helper.
inline void gemm_set_rowmajor_c(GemmBatch& g, long ldc) {
  g.cdiv_m = 1 << 30; g.cs_m1 = 0; g.cs_m0 = ldc;
  g.cdiv_n = 1 << 30; g.cs_n1 = 0; g.cs_n0 = 1;
}

// Launches a batched GEMM; ta = element type of A, tb of B, tc of C.
// Accumulation is float64 for F64 inputs and float32 otherwise.
int launch_gemm(const GemmBatch& g, DT ta, DT tb, DT tc, hipStream_t s);
// float64 C = op(A) B with N <= 160 (the enlarged corner applied to an
// isometry block); other shapes fall back to launch_gemm.
int launch_gemm_si(const GemmBatch& g, hipStream_t s);
// The same product with the (192-row tile, 16-wide K slice) space split
// evenly over ncu workgroups of 8 wavefronts (one per CU; at most
// kSplitMaxCus) and the cut tiles summed by a second kernel in a fixed order;
// scratch holds gemm_si_scratch_bytes().  Other shapes: launch_gemm_si.
constexpr int kSplitMaxCus = 256;
size_t gemm_si_scratch_bytes();
bool gemm_si_balanced_useful(int count, int M, int N, int K, int ncu);
bool gemm_si_balanced_applies(const GemmBatch& g, const void* scratch, int ncu);
int launch_gemm_si_balanced(const GemmBatch& g, double* scratch, int ncu, hipStream_t s);
// A float64 product on the split kernel where it applies (thin B, several
// K slices per tile), else on the tile kernels.
int launch_gemm_f64_any(const GemmBatch& g, double* scratch, int ncu, hipStream_t s);
// float32 contractions of the same shape: A float32, B and C float64 (B
// rounded to float32, float32 accumulation); other shapes fall back to
// launch_gemm.
int launch_gemm_si_f32(const GemmBatch& g, hipStream_t s);
// The same product in split bfloat16 (A float32, three bf16 products).
int launch_gemm_si_bx3(const GemmBatch& g, hipStream_t s);
// The float32 product split over ncu workgroups like launch_gemm_si_balanced
// (partial tiles in the same float64 scratch); launch_gemm_si_f32 when the
// split does not apply.
bool gemm_si_f32_balanced_applies(const GemmBatch& g, const void* scratch, int ncu);
int launch_gemm_si_f32_balanced(const GemmBatch& g, double* scratch, int ncu, hipStream_t s);

// Grouped float64 GEMMs: one persistent launch over the products of several
// descriptors of different shapes (see gemm.hip).  Each descriptor's work
// items are (tile, problem, inner batch) in the order of its own launch;
// `first` is the prefix sum over the descriptors before it.
struct GroupItem {
  GemmBatch g;
  int tiles_m, tiles_n;
  long first;
};
// Tile kernel for a group (0: the 96 x 160 skinny tile, which needs N <= 160
// and 16-byte aligned rows in every descriptor; else an index into the
// generic tile shapes), chosen from the descriptors.
int grouped_kind(const GemmBatch* gs, int n);
// Fills items[0..n) for the kind and returns the total number of work items.
long grouped_fill(const GemmBatch* gs, int n, int kind, GroupItem* items);
// Launches the group whose descriptors (filled by grouped_fill) are in
// device memory at dev_items.
int launch_gemm_grouped(const GroupItem* dev_items, int n, long total, int kind, hipStream_t s);

// Householder QR (in place, Q returned with R_ii >= 0) of `count` N x k
// row-major matrices.  ws must hold qr_workspace_bytes(count, N, k) bytes.
size_t qr_workspace_bytes(int count, int N, int k);
// True if N rows split into leaves of k .. 192 rows (every leaf holds a
// k x k triangle): the shapes launch_qr accepts.
bool qr_plan_ok(int N, int k);
int launch_qr(int count, double* const* W, int N, int k, void* ws, hipStream_t s);

// One-sided Jacobi SVD of `count` n x n row-major matrices (see ctm.h).
size_t svd_workspace_bytes(int count, int n);
int launch_svd(int count, const double* const* A, double* const* U, double* const* S,
               double* const* V, int n, void* ws, hipStream_t s);

}  // namespace sictm
