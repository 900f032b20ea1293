// Reverse-mode tape of float64 device computations (see tape.h).
//
// Vector-Jacobian products of the recorded operations:
//   GEMM C = alpha op(A) B (with the descriptor's two-level output map):
//     C_bar is gathered through the output map, then
//     A_bar += alpha C_bar B^T (or its transpose when A is stored
//     transposed) and B_bar += alpha op(A)^T C_bar;
//   permutation: the cotangent is scattered back through the same map;
//   thin QR H = Q R with only Q used (eq. xy_iter, stabilised):
//     H_bar += (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T,  R = Q^T H;
//   projector factors (eq. projectors_diag, eq. rho_hat_diag): the scaled
//     columns give u_bar, v_bar and s_bar through d(s^-1/2)/ds, then the
//     adjoint of rho = u s v^T (square, full u and v):
//     rho_bar = u [F o (u^T u_bar - u_bar^T u) s + diag(s_bar)
//                  + s F o (v^T v_bar - v_bar^T v)] v^T,  F_ij = 1 / (s_j^2 - s_i^2);
//   unit-norm scaling y = x / |x|:  x_bar += (y_bar - y <y, y_bar>) / |x|;
//   ratio e = <w1, E> / <w2, E>:  E_bar += e_bar (w1 - e w2) / <w2, E>.

#include "tape.h"

#include "../../include/ctm.h"

#include <algorithm>
#include <cmath>

#include "elem.h"

namespace sictm {
namespace {

constexpr int kMaxNd = 10;
constexpr int kDotParts = 128;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct NdArgs {
  int nd;
  int dims[kMaxNd];
  long strides[kMaxNd];
};

__device__ __forceinline__ long nd_offset(const NdArgs& a, long i) {
  long off = 0;
  for (int j = a.nd - 1; j >= 0; --j) {
    const long d = a.dims[j];
    off += (i % d) * a.strides[j];
    i /= d;
  }
  return off;
}

__global__ __launch_bounds__(256) void k_gather_nd(const double* __restrict__ src,
                                                   double* __restrict__ dst, NdArgs a, long total,
                                                   double alpha, int acc) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const double v = alpha * src[nd_offset(a, i)];
    dst[i] = acc ? dst[i] + v : v;
  }
}

// src_bar[map(i)] += dst_bar[i] for a bijective map (no two i share a target).
__global__ __launch_bounds__(256) void k_scatter_add_nd(const double* __restrict__ g,
                                                        double* __restrict__ out, NdArgs a,
                                                        long total) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256)
    out[nd_offset(a, i)] += g[i];
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ x, long n, double v) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) x[i] = v;
}

__global__ void k_add_scalar(double* x, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) x[0] += v;
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

// out[t] = <x_t, y_t>: block (b, t) sums a fixed strided subset into
// part[t][b]; the final pass adds the partial sums in block order, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_dots_part(DotArgs a, double* part) {
  __shared__ double sh[4];
  const int t = blockIdx.y;
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n[t]; i += (long)kDotParts * 256)
    acc += a.x[t][i] * a.y[t][i];
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

struct ScaleArgs {
  const double* x[8];
  double* y[8];
  long n[8];
  const double* sq;   // squared norms
  double* nrm;        // norms (written by block 0 of each tensor)
};

__global__ __launch_bounds__(256) void k_unit_scale(ScaleArgs a) {
  const int t = blockIdx.y;
  const double nr = sqrt(a.sq[t]);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.nrm[t] = nr;
  const double inv = 1.0 / nr;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n[t]; i += (long)gridDim.x * 256)
    a.y[t][i] = a.x[t][i] * inv;
}

struct NormBwdArgs {
  const double* y[8];
  const double* yb[8];
  double* xb[8];
  long n[8];
  const double* dot;   // <y_t, yb_t>
  const double* nrm;
};

__global__ __launch_bounds__(256) void k_norm_bwd_acc(NormBwdArgs a) {
  const int t = blockIdx.y;
  const double dt = a.dot[t], inv = 1.0 / a.nrm[t];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n[t]; i += (long)gridDim.x * 256)
    a.xb[t][i] += (a.yb[t][i] - a.y[t][i] * dt) * inv;
}

struct SmallArgs {
  const double* in[8];
  double* out[8];
  int n;
};

// out = tril(in) + tril(in, -1)^T
__global__ __launch_bounds__(256) void k_copyltu(SmallArgs a) {
  const int b = blockIdx.y, n = a.n;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n * n; idx += gridDim.x * 256) {
    const int i = idx / n, j = idx % n;
    a.out[b][idx] = i >= j ? a.in[b][idx] : a.in[b][j * n + i];
  }
}

// Inverse of an upper-triangular n x n matrix (n <= 192): back substitution
// row by row with the triangle of the result in LDS; thread j owns column j.
// A zero diagonal entry gives a zero row.
constexpr int kTriMax = 192;
__global__ __launch_bounds__(256) void k_tri_inv(SmallArgs a) {
  __shared__ double Xs[kTriMax * (kTriMax + 1) / 2];
  __shared__ double Rrow[kTriMax];
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
  const double* vscb[4];
  const double* uscb[4];
  double* ub[4];   // in: cotangent of us; out: with the projector terms
  double* vb[4];
  double* sb[4];
  int k, keep;
};

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
  const double* Ju[4];
  const double* Jv[4];
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

// num_den[0] / num_den[1] -> out
__global__ void k_ratio(const double* nd, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = nd[0] / nd[1];
}

// E_bar += e_bar (w1 - e w2) / den
__global__ __launch_bounds__(256) void k_ratio_bwd(const double* w1, const double* w2,
                                                   const double* nd, const double* e,
                                                   const double* eb, double* Eb, long n) {
  const double f = eb[0] / nd[1], ev = e[0];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    Eb[i] += f * (w1[i] - ev * w2[i]);
}

int grid_of(long n, int cap = 2048) { return (int)std::max<long>(1, std::min<long>(cap, (n + 255) / 256)); }

long map_extent(int n, int div, long s1, long s0) {
  if (n <= 0) return 0;
  return (long)((n - 1) / div) * s1 + (long)std::min(div - 1, n - 1) * s0;
}

}  // namespace

Tape::~Tape() {
  if (mem_) (void)hipFree(mem_);
}

int Tape::fail(int code, const std::string& msg) {
  err_ = msg;
  set_thread_error(msg);
  return code;
}

void Tape::begin_dry() {
  dry_ = true;
  regions_.clear();
  scratch_regions_.clear();
  back_.clear();
  val_base_ = reinterpret_cast<char*>(size_t(1) << 20);   // placeholder addresses
  val_off_ = val_need_ = 0;
  grad_need_ = 0;
  tmp_need_ = 0;
  qr_need_ = svd_need_ = 0;
  err_.clear();
}

int Tape::reserve() {
  const size_t need = align_up(val_need_) + align_up(grad_need_) + align_up(tmp_need_) +
                      align_up(qr_need_) + align_up(svd_need_) + align_up(gemm_si_scratch_bytes()) +
                      align_up(8 * kDotParts * sizeof(double)) + 4 * kAlign;
  if (!mem_ || cap_ < need) {
    if (mem_) (void)hipFree(mem_);
    mem_ = nullptr;
    cap_ = 0;
    if (hipMalloc((void**)&mem_, need) != hipSuccess)
      return fail(CTM_E_NOMEM, "hipMalloc of the adjoint tape (" + std::to_string(need >> 20) +
                                   " MiB) failed");
    cap_ = need;
  }
  // the partition follows the last dry pass (the memory may be larger)
  char* p = mem_;
  val_base_ = p;
  p += align_up(val_need_);
  grad_base_ = p;
  p += align_up(grad_need_);
  tmp_base_ = p;
  tmp_cap_ = align_up(tmp_need_);
  p += tmp_cap_;
  qr_ws_ = p;
  p += align_up(qr_need_);
  svd_ws_ = p;
  p += align_up(svd_need_);
  sk_part_ = reinterpret_cast<double*>(p);
  p += align_up(gemm_si_scratch_bytes());
  part_ = reinterpret_cast<double*>(p);
  return 0;
}

void Tape::begin() {
  dry_ = false;
  regions_.clear();
  scratch_regions_.clear();
  back_.clear();
  val_base_ = mem_;
  val_off_ = 0;
  grad_off_ = 0;
  tmp_off_ = 0;
  err_.clear();
  scratch_regions_.push_back({(uintptr_t)grad_base_, (uintptr_t)grad_base_ + align_up(grad_need_)});
  scratch_regions_.push_back({(uintptr_t)tmp_base_, (uintptr_t)tmp_base_ + tmp_cap_});
}

double* Tape::alloc(long n) {
  const size_t bytes = align_up((size_t)std::max<long>(n, 1) * sizeof(double));
  if (!dry_ && val_off_ + bytes > align_up(val_need_)) {
    fail(CTM_E_NOMEM, "adjoint tape: a value does not fit the reserved memory");
    return nullptr;
  }
  double* p = reinterpret_cast<double*>(val_base_ + val_off_);
  val_off_ += bytes;
  if (dry_) {
    val_need_ = val_off_;
    grad_need_ += bytes;
  }
  regions_[(uintptr_t)p] = Region{(uintptr_t)p + (size_t)n * sizeof(double), false, nullptr, nullptr};
  return p;
}

double* Tape::upload(const double* host, long n) {
  double* p = alloc(n);
  if (!p) return nullptr;
  regions_[(uintptr_t)p].constant = true;
  if (!dry_ && hipMemcpyAsync(p, host, (size_t)n * 8, hipMemcpyHostToDevice, st_) != hipSuccess) {
    fail(CTM_E_DEVICE, "upload of a constant failed");
    return nullptr;
  }
  return p;
}

void Tape::external(const double* p, long n, bool constant) {
  regions_[(uintptr_t)p] = Region{(uintptr_t)p + (size_t)n * sizeof(double), constant, nullptr, nullptr};
  if (dry_ && !constant) grad_need_ += align_up((size_t)n * sizeof(double));
}

void Tape::external_grad(const double* p, double* g) {
  auto it = regions_.find((uintptr_t)p);
  if (it == regions_.end()) return;
  it->second.ext_g = g;
  const long n = (long)((it->second.end - it->first) / sizeof(double));
  scratch_regions_.push_back({(uintptr_t)g, (uintptr_t)g + (size_t)n * sizeof(double)});
  if (!dry_) fill(g, n, 0.0);
}

const Tape::Region* Tape::find(const void* p, uintptr_t* base) const {
  const uintptr_t a = (uintptr_t)p;
  auto it = regions_.upper_bound(a);
  if (it == regions_.begin()) return nullptr;
  --it;
  if (a >= it->second.end) return nullptr;
  *base = it->first;
  return &it->second;
}

Tape::Region* Tape::find(const void* p, uintptr_t* base) {
  return const_cast<Region*>(static_cast<const Tape*>(this)->find(p, base));
}

bool Tape::inside(const void* p, size_t bytes) const {
  const uintptr_t a = (uintptr_t)p;
  uintptr_t b0;
  const Region* r = find(p, &b0);
  if (r && a + bytes <= r->end) return true;
  for (const auto& s : scratch_regions_)
    if (a >= s.first && a + bytes <= s.second) return true;
  return false;
}

double* Tape::grad_if(const double* p) const {
  uintptr_t base;
  const Region* r = find(p, &base);
  if (!r || r->constant) return nullptr;
  double* g = r->ext_g ? r->ext_g : r->g;
  if (!g) return nullptr;
  return g + ((uintptr_t)p - base) / sizeof(double);
}

double* Tape::grad(const double* p) {
  uintptr_t base;
  Region* r = find(p, &base);
  if (!r || r->constant) return nullptr;
  if (!r->ext_g && !r->g) {
    const size_t bytes = align_up(r->end - base);
    if (grad_off_ + bytes > align_up(grad_need_)) {
      fail(CTM_E_NOMEM, "adjoint tape: a cotangent does not fit the reserved memory");
      return nullptr;
    }
    r->g = reinterpret_cast<double*>(grad_base_ + grad_off_);
    grad_off_ += bytes;
    fill(r->g, (long)((r->end - base) / sizeof(double)), 0.0);
  }
  double* g = r->ext_g ? r->ext_g : r->g;
  return g + ((uintptr_t)p - base) / sizeof(double);
}

double* Tape::tmp(long n) {
  const size_t bytes = align_up((size_t)std::max<long>(n, 1) * sizeof(double));
  if (tmp_off_ + bytes > tmp_cap_) {
    fail(CTM_E_NOMEM, "adjoint tape: backward scratch exhausted");
    return nullptr;
  }
  double* p = reinterpret_cast<double*>(tmp_base_ + tmp_off_);
  tmp_off_ += bytes;
  return p;
}

int Tape::fill(double* x, long n, double v) {
  if (n <= 0 || dry_) return 0;
  k_fill<<<grid_of(n), 256, 0, st_>>>(x, n, v);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int Tape::copy(const double* src, double* dst, long n) {
  if (dry_ || n <= 0) return 0;
  if (!inside(src, (size_t)n * 8) || !inside(dst, (size_t)n * 8))
    return fail(CTM_E_SHAPE, "adjoint copy outside its buffers; refused");
  CTM_HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n * 8, hipMemcpyDeviceToDevice, st_));
  return 0;
}

int Tape::gather(const double* src, double* dst, int nd, const int* dims, const long* strides,
                 bool acc, double alpha) {
  if (nd < 1 || nd > kMaxNd) return fail(CTM_E_ARG, "adjoint gather: 1..10 dimensions");
  NdArgs a{};
  a.nd = nd;
  long total = 1, ext = 0;
  for (int j = 0; j < nd; ++j) {
    a.dims[j] = dims[j];
    a.strides[j] = strides[j];
    total *= dims[j];
    ext += (long)(dims[j] - 1) * strides[j];
  }
  if (total <= 0 || dry_) return 0;
  if (!inside(src, (size_t)(ext + 1) * 8) || !inside(dst, (size_t)total * 8))
    return fail(CTM_E_SHAPE, "adjoint gather outside its buffers; refused");
  k_gather_nd<<<grid_of(total, 4096), 256, 0, st_>>>(src, dst, a, total, alpha, acc ? 1 : 0);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int Tape::scatter_add(const double* src, double* dst, int nd, const int* dims, const long* strides) {
  NdArgs a{};
  a.nd = nd;
  long total = 1, ext = 0;
  for (int j = 0; j < nd; ++j) {
    a.dims[j] = dims[j];
    a.strides[j] = strides[j];
    total *= dims[j];
    ext += (long)(dims[j] - 1) * strides[j];
  }
  if (total <= 0 || dry_) return 0;
  if (!inside(src, (size_t)total * 8) || !inside(dst, (size_t)(ext + 1) * 8))
    return fail(CTM_E_SHAPE, "adjoint scatter outside its buffers; refused");
  k_scatter_add_nd<<<grid_of(total, 4096), 256, 0, st_>>>(src, dst, a, total);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int Tape::dots(int count, const double* const* x, const double* const* y, const long* n,
               double* out) {
  if (dry_ || count <= 0) return 0;
  DotArgs a{};
  for (int t = 0; t < count; ++t) {
    a.x[t] = x[t];
    a.y[t] = y[t];
    a.n[t] = n[t];
    if (!inside(x[t], (size_t)n[t] * 8) || !inside(y[t], (size_t)n[t] * 8))
      return fail(CTM_E_SHAPE, "adjoint dot product outside its buffers; refused");
  }
  a.out = out;
  k_dots_part<<<dim3(kDotParts, count), 256, 0, st_>>>(a, part_);
  CTM_HIP_TRY(hipGetLastError());
  k_dots_final<<<count, 256, 0, st_>>>(a, part_);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int Tape::check_gemm(const GemmBatch& g) const {
  if (g.M <= 0 || g.N <= 0) return 0;
  for (int i = 0; i < g.count; ++i) {
    const long ea = g.K <= 0 ? 0
                    : (g.transA[i] ? (long)(g.K - 1) * g.lda + (g.M - 1)
                                   : (long)(g.M - 1) * g.lda + (g.K - 1)) +
                          (long)(g.nbatch - 1) * g.a_bs;
    const long eb = g.K <= 0 ? 0 : (long)(g.K - 1) * g.ldb + (g.N - 1) + (long)(g.nbatch - 1) * g.b_bs;
    const long ec = map_extent(g.M, g.cdiv_m, g.cs_m1, g.cs_m0) +
                    map_extent(g.N, g.cdiv_n, g.cs_n1, g.cs_n0) + (long)(g.nbatch - 1) * g.c_bs;
    if (!(g.K <= 0 || inside(g.A[i], (size_t)(ea + 1) * 8)) ||
        !(g.K <= 0 || inside(g.B[i], (size_t)(eb + 1) * 8)) || !inside(g.C[i], (size_t)(ec + 1) * 8))
      return CTM_E_SHAPE;
  }
  return 0;
}

int Tape::launch(const GemmBatch& g) {
  if (dry_ || g.count == 0) return 0;
  if (check_gemm(g))
    return fail(CTM_E_SHAPE, "adjoint GEMM operand outside its buffers (M=" + std::to_string(g.M) +
                                 " N=" + std::to_string(g.N) + " K=" + std::to_string(g.K) +
                                 "); launch refused");
  const int rc = launch_gemm_f64_any(g, sk_part_, kSplitMaxCus, st_);
  if (rc) return fail(rc == 1 ? CTM_E_ARG : rc, thread_error());
  return 0;
}

// ---------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------
int Tape::gemm(const GemmBatch& g) {
  if (g.accumulate) return fail(CTM_E_ARG, "taped GEMMs do not accumulate");
  const int rc = launch(g);
  if (rc) return rc;
  // scratch of the backward pass: per problem C_bar and one transposed operand
  const long MN = (long)g.M * g.N;
  const long T = std::max<long>((long)g.N * g.K, MN);
  note_tmp((size_t)g.count * align_up((size_t)MN * 8) + (size_t)g.count * align_up((size_t)T * 8));
  back_.push_back([this, g]() { return gemm_bwd(g); });
  return 0;
}

int Tape::gemm_bwd(const GemmBatch& g) {
  const int M = g.M, N = g.N, K = g.K;
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  const bool plain = g.cdiv_m >= M && g.cs_m0 == N && g.cdiv_n >= N && g.cs_n0 == 1 && g.alpha == 1.0;
  const int Mr = std::min(g.cdiv_m, M), Nr = std::min(g.cdiv_n, N);
  if (M % Mr || N % Nr) return fail(CTM_E_SHAPE, "adjoint of a GEMM with a ragged output map");
  for (int b = 0; b < g.nbatch; ++b) {
    tmp_reset();
    const double* A[kMaxProb];
    const double* B[kMaxProb];
    const double* Cb[kMaxProb];
    double* Ag[kMaxProb];
    double* Bg[kMaxProb];
    int live[kMaxProb];
    int nl = 0;
    for (int p = 0; p < g.count; ++p) {
      const double* C = (const double*)g.C[p] + (long)b * g.c_bs;
      const double* cg = grad_if(C);
      if (!cg) continue;
      A[nl] = (const double*)g.A[p] + (long)b * g.a_bs;
      B[nl] = (const double*)g.B[p] + (long)b * g.b_bs;
      if (plain) {
        Cb[nl] = cg;
      } else {
        double* t = tmp(M * (long)N);
        if (!t) return CTM_E_NOMEM;
        const int dims[4] = {M / Mr, Mr, N / Nr, Nr};
        const long strides[4] = {g.cs_m1, g.cs_m0, g.cs_n1, g.cs_n0};
        const int rc = gather(cg, t, 4, dims, strides, false, g.alpha);
        if (rc) return rc;
        Cb[nl] = t;
      }
      Ag[nl] = grad(A[nl]);
      Bg[nl] = grad(B[nl]);
      live[nl] = p;
      ++nl;
    }
    if (nl == 0) continue;
    // A side: grouped by transposition, destinations distinct within a launch
    for (int tr = 0; tr < 2; ++tr) {
      GemmBatch ga{};
      auto flush = [&]() -> int {
        if (ga.count == 0) return 0;
        const int rc = launch(ga);
        ga.count = 0;
        return rc;
      };
      for (int q = 0; q < nl; ++q) {
        const int p = live[q];
        if (!Ag[q] || (g.transA[p] != 0) != (tr == 1)) continue;
        for (int o = 0; o < ga.count; ++o)
          if (ga.C[o] == Ag[q]) {
            const int rc = flush();
            if (rc) return rc;
            break;
          }
        if (ga.count == kMaxProb) {
          const int rc = flush();
          if (rc) return rc;
        }
        if (ga.count == 0) {
          if (tr == 0) {
            // A_bar (M x K) += C_bar (M x N) B^T (N x K)
            ga = GemmBatch{};
            ga.M = M; ga.N = K; ga.K = N; ga.lda = N; ga.ldb = K;
          } else {
            // A stored K x M: A_bar^T (K x M) += B (K x N) C_bar^T (N x M)
            ga = GemmBatch{};
            ga.M = K; ga.N = M; ga.K = N; ga.lda = g.ldb; ga.ldb = M;
          }
          ga.cdiv_m = 1 << 30; ga.cs_m1 = 0; ga.cs_m0 = g.lda;
          ga.cdiv_n = 1 << 30; ga.cs_n1 = 0; ga.cs_n0 = 1;
          ga.nbatch = 1;
          ga.alpha = 1.0;
          ga.accumulate = 1;
        }
        double* t = tmp(tr == 0 ? (long)N * K : (long)N * M);
        if (!t) return CTM_E_NOMEM;
        if (tr == 0) {
          const int dims[2] = {N, K};
          const long strides[2] = {1, g.ldb};
          const int rc = gather(B[q], t, 2, dims, strides, false);
          if (rc) return rc;
          ga.A[ga.count] = Cb[q];
          ga.B[ga.count] = t;
        } else {
          const int dims[2] = {N, M};
          const long strides[2] = {1, N};
          const int rc = gather(Cb[q], t, 2, dims, strides, false);
          if (rc) return rc;
          ga.A[ga.count] = B[q];
          ga.B[ga.count] = t;
        }
        ga.transA[ga.count] = 0;
        ga.C[ga.count] = Ag[q];
        ++ga.count;
      }
      const int rc = flush();
      if (rc) return rc;
    }
    // B side: B_bar (K x N) += op(A)^T (K x M) C_bar (M x N)
    {
      GemmBatch gb{};
      auto flush = [&]() -> int {
        if (gb.count == 0) return 0;
        const int rc = launch(gb);
        gb.count = 0;
        return rc;
      };
      for (int q = 0; q < nl; ++q) {
        const int p = live[q];
        if (!Bg[q]) continue;
        for (int o = 0; o < gb.count; ++o)
          if (gb.C[o] == Bg[q]) {
            const int rc = flush();
            if (rc) return rc;
            break;
          }
        if (gb.count == kMaxProb) {
          const int rc = flush();
          if (rc) return rc;
        }
        if (gb.count == 0) {
          gb = GemmBatch{};
          gb.M = K; gb.N = N; gb.K = M; gb.lda = g.lda; gb.ldb = N;
          gb.cdiv_m = 1 << 30; gb.cs_m1 = 0; gb.cs_m0 = g.ldb;
          gb.cdiv_n = 1 << 30; gb.cs_n1 = 0; gb.cs_n0 = 1;
          gb.nbatch = 1;
          gb.alpha = 1.0;
          gb.accumulate = 1;
        }
        gb.A[gb.count] = A[q];
        gb.transA[gb.count] = g.transA[p] ? 0 : 1;
        gb.B[gb.count] = Cb[q];
        gb.C[gb.count] = Bg[q];
        ++gb.count;
      }
      const int rc = flush();
      if (rc) return rc;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// permutation
// ---------------------------------------------------------------------------
int Tape::permute(const double* src, double* dst, int nd, const int* dims, const long* strides) {
  int rc = gather(src, dst, nd, dims, strides, false);
  if (rc) return rc;
  std::vector<int> d(dims, dims + nd);
  std::vector<long> s(strides, strides + nd);
  back_.push_back([this, src, dst, d, s]() -> int {
    const double* gd = grad_if(dst);
    if (!gd) return 0;
    double* gs = grad(src);
    if (!gs) return 0;
    return scatter_add(gd, gs, (int)d.size(), d.data(), s.data());
  });
  return 0;
}

// ---------------------------------------------------------------------------
// thin QR
// ---------------------------------------------------------------------------
int Tape::qr(int count, const double* const* H, double* const* Q, int n, int k) {
  if (count < 1 || count > kMaxProb) return fail(CTM_E_ARG, "adjoint QR: 1..8 blocks");
  if (!qr_plan_ok(n, k)) return fail(CTM_E_SHAPE, "adjoint QR: no leaf partition for the block");
  const size_t ws = qr_workspace_bytes(count, n, k);
  if (dry_) {
    qr_need_ = std::max(qr_need_, ws);
  } else {
    if (ws > qr_need_) return fail(CTM_E_NOMEM, "adjoint QR workspace exceeds the reservation");
    for (int j = 0; j < count; ++j) {
      const int rc = copy(H[j], Q[j], (long)n * k);
      if (rc) return rc;
    }
    const int rc = launch_qr(count, Q, n, k, qr_ws_, st_);
    if (rc) return fail(rc == 1 ? CTM_E_ARG : rc, thread_error());
  }
  const long kk = (long)k * k, nk = (long)n * k;
  note_tmp((size_t)count * (5 * align_up((size_t)kk * 8) + align_up((size_t)nk * 8)));
  std::vector<const double*> h(H, H + count);
  std::vector<double*> q(Q, Q + count);
  back_.push_back([this, h, q, n, k, kk, nk]() -> int {
    const int cnt = (int)h.size();
    std::vector<int> live;
    std::vector<const double*> qb(cnt, nullptr);
    std::vector<double*> hg(cnt, nullptr);
    for (int j = 0; j < cnt; ++j) {
      qb[j] = grad_if(q[j]);
      if (!qb[j]) continue;
      hg[j] = grad(h[j]);
      if (hg[j]) live.push_back(j);
    }
    if (live.empty()) return 0;
    const int nl = (int)live.size();
    std::vector<double*> R(nl), Mm(nl), Mc(nl), Ri(nl), RiT(nl), Y(nl);
    for (int i = 0; i < nl; ++i) {
      R[i] = tmp(kk); Mm[i] = tmp(kk); Mc[i] = tmp(kk); Ri[i] = tmp(kk); RiT[i] = tmp(kk); Y[i] = tmp(nk);
      if (!R[i] || !Mm[i] || !Mc[i] || !Ri[i] || !RiT[i] || !Y[i]) return CTM_E_NOMEM;
    }
    auto rm = [&](int M_, int N_, int K_, long lda, long ldb, long ldc) {
      GemmBatch g{};
      g.M = M_; g.N = N_; g.K = K_; g.lda = lda; g.ldb = ldb;
      gemm_set_rowmajor_c(g, ldc);
      g.nbatch = 1;
      g.alpha = 1.0;
      return g;
    };
    // R = Q^T H, Mm = -Q_bar^T Q
    GemmBatch g1 = rm(k, k, n, k, k, k), g2 = rm(k, k, n, k, k, k);
    g2.alpha = -1.0;
    for (int i = 0; i < nl; ++i) {
      const int j = live[i];
      g1.A[i] = q[j]; g1.transA[i] = 1; g1.B[i] = h[j]; g1.C[i] = R[i];
      g2.A[i] = qb[j]; g2.transA[i] = 1; g2.B[i] = q[j]; g2.C[i] = Mm[i];
    }
    g1.count = g2.count = nl;
    int rc = launch(g1);
    if (!rc) rc = launch(g2);
    if (rc) return rc;
    SmallArgs sa{};
    for (int i = 0; i < nl; ++i) {
      sa.in[i] = Mm[i];
      sa.out[i] = Mc[i];
    }
    sa.n = k;
    k_copyltu<<<dim3((unsigned)((kk + 255) / 256), nl), 256, 0, st_>>>(sa);
    CTM_HIP_TRY(hipGetLastError());
    for (int i = 0; i < nl; ++i) {
      sa.in[i] = R[i];
      sa.out[i] = Ri[i];
    }
    k_tri_inv<<<nl, 256, 0, st_>>>(sa);
    CTM_HIP_TRY(hipGetLastError());
    for (int i = 0; i < nl; ++i) {
      const int dims[2] = {k, k};
      const long strides[2] = {1, k};
      rc = gather(Ri[i], RiT[i], 2, dims, strides, false);
      if (!rc) rc = copy(qb[live[i]], Y[i], nk);
      if (rc) return rc;
    }
    // Y = Q_bar + Q Mc;  H_bar += Y R^-T
    GemmBatch g3 = rm(n, k, k, k, k, k), g4 = rm(n, k, k, k, k, k);
    g3.accumulate = 1;
    g4.accumulate = 1;
    for (int i = 0; i < nl; ++i) {
      const int j = live[i];
      g3.A[i] = q[j]; g3.B[i] = Mc[i]; g3.C[i] = Y[i];
      g4.A[i] = Y[i]; g4.B[i] = RiT[i]; g4.C[i] = hg[j];
    }
    g3.count = g4.count = nl;
    rc = launch(g3);
    if (!rc) rc = launch(g4);
    return rc;
  });
  return 0;
}

// ---------------------------------------------------------------------------
// projector factors from the SVD of rho
// ---------------------------------------------------------------------------
int Tape::svdproj(int count, const double* const* rho, const double* const* Yt, int nrows, int k,
                  int keep, double rtol, double* const* us, double* const* vs, double* const* vsc,
                  double* const* usc) {
  if (count < 1 || count > 4) return fail(CTM_E_ARG, "adjoint projector factors: 1..4 at once");
  std::vector<double*> u(count), v(count), s(count), sg(count), sinv(count), ytu(count);
  for (int j = 0; j < count; ++j) {
    ytu[j] = alloc((long)nrows * k);
    u[j] = alloc((long)k * k);
    v[j] = alloc((long)k * k);
    s[j] = alloc(k);
    sg[j] = alloc(k);
    sinv[j] = alloc(k);
    if (!u[j] || !v[j] || !s[j] || !sg[j] || !sinv[j]) return CTM_E_NOMEM;
  }
  const size_t ws = svd_workspace_bytes(count, k);
  if (dry_) {
    svd_need_ = std::max(svd_need_, ws);
  } else {
    if (ws > svd_need_) return fail(CTM_E_NOMEM, "adjoint SVD workspace exceeds the reservation");
    int rc = launch_svd(count, rho, u.data(), s.data(), v.data(), k, svd_ws_, st_);
    if (rc) return fail(rc == 1 ? CTM_E_ARG : rc, thread_error());
    // the sign source Yt u (a constant: not recorded)
    GemmBatch gy{};
    gy.M = nrows; gy.N = k; gy.K = k; gy.lda = k; gy.ldb = k;
    gemm_set_rowmajor_c(gy, k);
    gy.nbatch = 1;
    gy.alpha = 1.0;
    for (int j = 0; j < count; ++j) {
      gy.A[j] = Yt[j];
      gy.B[j] = u[j];
      gy.C[j] = ytu[j];
    }
    gy.count = count;
    rc = launch(gy);
    if (rc) return rc;
    SignArgs sa{};
    sa.N = nrows;
    sa.k = k;
    sa.ld = k;
    for (int j = 0; j < count; ++j) {
      sa.Y[j] = ytu[j];
      sa.sg[j] = sg[j];
    }
    rc = elem_col_sign(sa, count, st_);
    if (rc) return fail(rc == 1 ? CTM_E_ARG : rc, thread_error());
    PrepArgs pa{};
    for (int j = 0; j < count; ++j) {
      pa.u[j] = u[j]; pa.v[j] = v[j]; pa.s[j] = s[j]; pa.sg[j] = sg[j];
      pa.us[j] = us[j]; pa.vs[j] = vs[j]; pa.sinv[j] = sinv[j];
      pa.vsc[j] = vsc[j]; pa.usc[j] = usc[j];
    }
    pa.k = k;
    pa.keep = keep;
    pa.rtol = rtol;
    k_prep<<<dim3((unsigned)((k * k + 255) / 256), count), 256, 0, st_>>>(pa);
    CTM_HIP_TRY(hipGetLastError());
  }
  const long kk = (long)k * k;
  note_tmp((size_t)count * (7 * align_up((size_t)kk * 8) + 2 * align_up((size_t)k * keep * 8) +
                            align_up((size_t)k * 8)));
  std::vector<const double*> rh(rho, rho + count);
  std::vector<double*> US(us, us + count), VS(vs, vs + count), VSC(vsc, vsc + count),
      USC(usc, usc + count);
  back_.push_back([=]() -> int {
    const int cnt = (int)rh.size();
    std::vector<double*> ub(cnt), vb(cnt), sb(cnt), vscb(cnt), uscb(cnt), Ju(cnt), Jv(cnt), Km(cnt),
        uK(cnt), vsT(cnt);
    bool any = false;
    for (int j = 0; j < cnt; ++j)
      any = any || grad_if(US[j]) || grad_if(VS[j]) || grad_if(VSC[j]) || grad_if(USC[j]);
    if (!any) return 0;
    for (int j = 0; j < cnt; ++j) {
      ub[j] = tmp(kk); vb[j] = tmp(kk); sb[j] = tmp(k); vscb[j] = tmp((long)k * keep);
      uscb[j] = tmp((long)k * keep); Ju[j] = tmp(kk); Jv[j] = tmp(kk); Km[j] = tmp(kk);
      uK[j] = tmp(kk); vsT[j] = tmp(kk);
      if (!vsT[j]) return CTM_E_NOMEM;
      int rc = 0;
      auto init = [&](const double* gsrc, double* dst, long n) {
        return gsrc ? copy(gsrc, dst, n) : fill(dst, n, 0.0);
      };
      rc = init(grad_if(US[j]), ub[j], kk);
      if (!rc) rc = init(grad_if(VS[j]), vb[j], kk);
      if (!rc) rc = init(grad_if(VSC[j]), vscb[j], (long)k * keep);
      if (!rc) rc = init(grad_if(USC[j]), uscb[j], (long)k * keep);
      if (rc) return rc;
    }
    ProjBwdArgs pb{};
    for (int j = 0; j < cnt; ++j) {
      pb.us[j] = US[j]; pb.vs[j] = VS[j]; pb.sinv[j] = sinv[j];
      pb.vscb[j] = vscb[j]; pb.uscb[j] = uscb[j];
      pb.ub[j] = ub[j]; pb.vb[j] = vb[j]; pb.sb[j] = sb[j];
    }
    pb.k = k;
    pb.keep = keep;
    k_proj_bwd<<<cnt, 256, 0, st_>>>(pb);
    CTM_HIP_TRY(hipGetLastError());
    auto rm = [&](int M_, int N_, int K_) {
      GemmBatch g{};
      g.M = M_; g.N = N_; g.K = K_; g.lda = K_; g.ldb = N_;
      gemm_set_rowmajor_c(g, N_);
      g.nbatch = 1;
      g.alpha = 1.0;
      return g;
    };
    GemmBatch g1 = rm(k, k, k);
    g1.lda = k;
    for (int j = 0; j < cnt; ++j) {
      g1.A[2 * j] = US[j]; g1.transA[2 * j] = 1; g1.B[2 * j] = ub[j]; g1.C[2 * j] = Ju[j];
      g1.A[2 * j + 1] = VS[j]; g1.transA[2 * j + 1] = 1; g1.B[2 * j + 1] = vb[j]; g1.C[2 * j + 1] = Jv[j];
    }
    g1.count = 2 * cnt;
    int rc = launch(g1);
    if (rc) return rc;
    KmatArgs ka{};
    for (int j = 0; j < cnt; ++j) {
      ka.Ju[j] = Ju[j]; ka.Jv[j] = Jv[j]; ka.s[j] = s[j]; ka.sb[j] = sb[j]; ka.K[j] = Km[j];
    }
    ka.n = k;
    k_svd_kmat<<<dim3((unsigned)((kk + 255) / 256), cnt), 256, 0, st_>>>(ka);
    CTM_HIP_TRY(hipGetLastError());
    GemmBatch g2 = rm(k, k, k);
    for (int j = 0; j < cnt; ++j) {
      g2.A[j] = US[j]; g2.B[j] = Km[j]; g2.C[j] = uK[j];
      const int dims[2] = {k, k};
      const long strides[2] = {1, k};
      rc = gather(VS[j], vsT[j], 2, dims, strides, false);
      if (rc) return rc;
    }
    g2.count = cnt;
    rc = launch(g2);
    if (rc) return rc;
    GemmBatch g3 = rm(k, k, k);
    g3.accumulate = 1;
    int nc = 0;
    for (int j = 0; j < cnt; ++j) {
      double* rg = grad(rh[j]);
      if (!rg) continue;
      g3.A[nc] = uK[j]; g3.B[nc] = vsT[j]; g3.C[nc] = rg;
      ++nc;
    }
    g3.count = nc;
    return launch(g3);
  });
  return 0;
}

// ---------------------------------------------------------------------------
// unit-norm scaling
// ---------------------------------------------------------------------------
int Tape::normalize(int count, const double* const* x, double* const* y, const long* n) {
  if (count < 1 || count > 8) return fail(CTM_E_ARG, "adjoint normalisation: 1..8 tensors");
  double* sq = alloc(8);
  double* nrm = alloc(8);
  if (!sq || !nrm) return CTM_E_NOMEM;
  long mx = 0;
  for (int t = 0; t < count; ++t) mx = std::max(mx, n[t]);
  if (!dry_) {
    int rc = dots(count, x, x, n, sq);
    if (rc) return rc;
    ScaleArgs a{};
    for (int t = 0; t < count; ++t) {
      a.x[t] = x[t];
      a.y[t] = y[t];
      a.n[t] = n[t];
      if (!inside(y[t], (size_t)n[t] * 8)) return fail(CTM_E_SHAPE, "normalisation outside its buffer");
    }
    a.sq = sq;
    a.nrm = nrm;
    k_unit_scale<<<dim3(grid_of(mx, 512), count), 256, 0, st_>>>(a);
    CTM_HIP_TRY(hipGetLastError());
  }
  note_tmp(2 * align_up(8 * 8));
  std::vector<const double*> xs(x, x + count);
  std::vector<double*> ys(y, y + count);
  std::vector<long> ns(n, n + count);
  back_.push_back([this, xs, ys, ns, nrm, mx]() -> int {
    const int cnt = (int)xs.size();
    NormBwdArgs a{};
    const double* yy[8];
    const double* yb[8];
    long nn[8];
    int nl = 0;
    int idx[8];
    for (int t = 0; t < cnt; ++t) {
      const double* g = grad_if(ys[t]);
      if (!g) continue;
      double* xg = grad(xs[t]);
      if (!xg) continue;
      yy[nl] = ys[t];
      yb[nl] = g;
      nn[nl] = ns[t];
      a.y[nl] = ys[t];
      a.yb[nl] = g;
      a.xb[nl] = xg;
      a.n[nl] = ns[t];
      idx[nl] = t;
      ++nl;
    }
    if (nl == 0) return 0;
    double* dt = tmp(8);
    double* nr = tmp(8);
    if (!dt || !nr) return CTM_E_NOMEM;
    int rc = dots(nl, yy, yb, nn, dt);
    if (rc) return rc;
    for (int i = 0; i < nl; ++i) {
      const int dims[1] = {1};
      const long strides[1] = {0};
      rc = gather(nrm + idx[i], nr + i, 1, dims, strides, false);
      if (rc) return rc;
    }
    a.dot = dt;
    a.nrm = nr;
    k_norm_bwd_acc<<<dim3(grid_of(mx, 512), nl), 256, 0, st_>>>(a);
    CTM_HIP_TRY(hipGetLastError());
    return 0;
  });
  return 0;
}

// ---------------------------------------------------------------------------
// ratio of two linear forms (a bond value from its unnormalised density matrix)
// ---------------------------------------------------------------------------
int Tape::ratio(const double* E, const double* w1, const double* w2, long n, double* out) {
  double* nd = alloc(2);
  if (!nd) return CTM_E_NOMEM;
  if (!dry_) {
    const double* xs[2] = {w1, w2};
    const double* ys[2] = {E, E};
    const long ns[2] = {n, n};
    int rc = dots(2, xs, ys, ns, nd);
    if (rc) return rc;
    k_ratio<<<1, 64, 0, st_>>>(nd, out);
    CTM_HIP_TRY(hipGetLastError());
  }
  back_.push_back([this, E, w1, w2, n, nd, out]() -> int {
    const double* eb = grad_if(out);
    if (!eb) return 0;
    double* Eg = grad(E);
    if (!Eg) return 0;
    if (!inside(Eg, (size_t)n * 8) || !inside(w1, (size_t)n * 8) || !inside(w2, (size_t)n * 8))
      return fail(CTM_E_SHAPE, "adjoint ratio outside its buffers; refused");
    k_ratio_bwd<<<grid_of(n), 256, 0, st_>>>(w1, w2, nd, out, eb, Eg, n);
    CTM_HIP_TRY(hipGetLastError());
    return 0;
  });
  return 0;
}

// ---------------------------------------------------------------------------
// backward pass
// ---------------------------------------------------------------------------
int Tape::accumulate_grad(const double* p, double* dst, long n) {
  const double* g = grad_if(p);
  if (!g || dry_) return 0;
  scratch_regions_.push_back({(uintptr_t)dst, (uintptr_t)dst + (size_t)n * sizeof(double)});
  const int dims[1] = {(int)n};
  const long strides[1] = {1};
  const int rc = gather(g, dst, 1, dims, strides, true);
  scratch_regions_.pop_back();
  return rc;
}

int Tape::copy_out(const double* src, double* dst, long n) {
  if (dry_) return 0;
  scratch_regions_.push_back({(uintptr_t)dst, (uintptr_t)dst + (size_t)n * sizeof(double)});
  const int rc = copy(src, dst, n);
  scratch_regions_.pop_back();
  return rc;
}

int Tape::seed(const double* p, const double* g, long n) {
  double* d = grad(p);
  if (!d || dry_) return 0;
  scratch_regions_.push_back({(uintptr_t)g, (uintptr_t)g + (size_t)n * sizeof(double)});
  const int dims[1] = {(int)n};
  const long strides[1] = {1};
  const int rc = gather(g, d, 1, dims, strides, true);
  scratch_regions_.pop_back();
  return rc;
}

int Tape::seed_scalar(const double* p, double alpha) {
  double* d = grad(p);
  if (!d || dry_) return 0;
  k_add_scalar<<<1, 64, 0, st_>>>(d, alpha);
  CTM_HIP_TRY(hipGetLastError());
  return 0;
}

int Tape::backward() {
  if (dry_) return 0;
  for (size_t i = back_.size(); i-- > 0;) {
    tmp_reset();
    const int rc = back_[i]();
    if (rc) return rc;
    if (!err_.empty()) return CTM_E_NOMEM;
  }
  return 0;
}

}  // namespace sictm

// ---------------------------------------------------------------------------
// self-check entry points: one operation and its vector-Jacobian product
// ---------------------------------------------------------------------------
namespace {

using sictm::Tape;

struct CheckRun {
  Tape t{nullptr};
  int run(const std::function<int(Tape&)>& fwd, const std::function<int(Tape&)>& seeds) {
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 0) {
        t.begin_dry();
      } else {
        const int rc = t.reserve();
        if (rc) return rc;
        t.begin();
      }
      const int rc = fwd(t);
      if (rc) return rc;
    }
    int rc = seeds(t);
    if (!rc) rc = t.backward();
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = CTM_E_DEVICE;
    if (!rc && !t.error().empty()) rc = CTM_E_NOMEM;
    return rc;
  }
};

}  // namespace

extern "C" {

ctm_status ctm_tape_check_gemm(const int* dims, const long* strides, double alpha, const double* A,
                               long nA, const double* B, long nB, double* C, long nC,
                               const double* Cbar, double* Abar, double* Bbar) {
  if (!dims || !strides || !A || !B || !C || !Cbar || !Abar || !Bbar) return CTM_E_ARG;
  sictm::GemmBatch g{};
  g.count = 1;
  g.M = dims[0];
  g.N = dims[1];
  g.K = dims[2];
  g.transA[0] = dims[3];
  g.cdiv_m = dims[4];
  g.cdiv_n = dims[5];
  g.nbatch = dims[6];
  g.lda = strides[0];
  g.ldb = strides[1];
  g.cs_m1 = strides[2];
  g.cs_m0 = strides[3];
  g.cs_n1 = strides[4];
  g.cs_n0 = strides[5];
  g.a_bs = strides[6];
  g.b_bs = strides[7];
  g.c_bs = strides[8];
  g.alpha = alpha;
  g.A[0] = A;
  g.B[0] = B;
  CheckRun cr;
  double* out = nullptr;
  const int rc = cr.run(
      [&](Tape& t) {
        t.external(A, nA, false);
        t.external(B, nB, false);
        if (!t.dry()) {
          t.external_grad(A, Abar);
          t.external_grad(B, Bbar);
        }
        out = t.alloc(nC);
        if (!out) return (int)CTM_E_NOMEM;
        if (!t.dry() && hipMemset(out, 0, (size_t)nC * 8) != hipSuccess) return (int)CTM_E_DEVICE;
        g.C[0] = out;
        return t.gemm(g);
      },
      [&](Tape& t) {
        const int r = t.seed(out, Cbar, nC);
        return r ? r : t.copy_out(out, C, nC);
      });
  return (ctm_status)rc;
}

ctm_status ctm_tape_check_qr(int count, int n, int k, const double* H, double* Q, const double* Qbar,
                             double* Hbar) {
  if (count < 1 || count > 8 || !H || !Q || !Qbar || !Hbar) return CTM_E_ARG;
  const long nk = (long)n * k;
  CheckRun cr;
  std::vector<double*> q(count);
  const int rc = cr.run(
      [&](Tape& t) {
        t.external(H, count * nk, false);
        if (!t.dry()) t.external_grad(H, Hbar);
        std::vector<const double*> h(count);
        for (int j = 0; j < count; ++j) {
          h[j] = H + j * nk;
          q[j] = t.alloc(nk);
          if (!q[j]) return (int)CTM_E_NOMEM;
        }
        return t.qr(count, h.data(), q.data(), n, k);
      },
      [&](Tape& t) {
        for (int j = 0; j < count; ++j) {
          int r = t.seed(q[j], Qbar + j * nk, nk);
          if (!r) r = t.copy_out(q[j], Q + j * nk, nk);
          if (r) return r;
        }
        return 0;
      });
  return (ctm_status)rc;
}

ctm_status ctm_tape_check_svdproj(int k, int keep, int nrows, double rtol, const double* rho,
                                  const double* Yt, double* outs, const double* bars,
                                  double* rhobar) {
  if (!rho || !Yt || !outs || !bars || !rhobar || keep < 1 || keep > k) return CTM_E_ARG;
  const long kk = (long)k * k, kp = (long)k * keep;
  CheckRun cr;
  double *us = nullptr, *vs = nullptr, *vsc = nullptr, *usc = nullptr;
  const int rc = cr.run(
      [&](Tape& t) {
        t.external(rho, kk, false);
        t.external(Yt, (long)nrows * k, true);
        if (!t.dry()) t.external_grad(rho, rhobar);
        us = t.alloc(kk);
        vs = t.alloc(kk);
        vsc = t.alloc(kp);
        usc = t.alloc(kp);
        if (!us || !vs || !vsc || !usc) return (int)CTM_E_NOMEM;
        return t.svdproj(1, &rho, &Yt, nrows, k, keep, rtol, &us, &vs, &vsc, &usc);
      },
      [&](Tape& t) {
        // outs and bars: us (k x k), vs (k x k), vsc (k x keep), usc (k x keep)
        const double* src[4] = {us, vs, vsc, usc};
        const long ns[4] = {kk, kk, kp, kp};
        long off = 0;
        for (int j = 0; j < 4; ++j) {
          int r = t.seed(src[j], bars + off, ns[j]);
          if (!r) r = t.copy_out(src[j], outs + off, ns[j]);
          if (r) return r;
          off += ns[j];
        }
        return 0;
      });
  return (ctm_status)rc;
}

ctm_status ctm_tape_check_normalize(int count, const long* n, const double* x, double* y,
                                    const double* ybar, double* xbar) {
  if (count < 1 || count > 8 || !n || !x || !y || !ybar || !xbar) return CTM_E_ARG;
  long tot = 0;
  for (int t = 0; t < count; ++t) tot += n[t];
  CheckRun cr;
  std::vector<double*> ys(count);
  const int rc = cr.run(
      [&](Tape& t) {
        t.external(x, tot, false);
        if (!t.dry()) t.external_grad(x, xbar);
        std::vector<const double*> xs(count);
        long off = 0;
        for (int j = 0; j < count; ++j) {
          xs[j] = x + off;
          ys[j] = t.alloc(n[j]);
          if (!ys[j]) return (int)CTM_E_NOMEM;
          off += n[j];
        }
        return t.normalize(count, xs.data(), ys.data(), n);
      },
      [&](Tape& t) {
        long off = 0;
        for (int j = 0; j < count; ++j) {
          int r = t.seed(ys[j], ybar + off, n[j]);
          if (!r) r = t.copy_out(ys[j], y + off, n[j]);
          if (r) return r;
          off += n[j];
        }
        return 0;
      });
  return (ctm_status)rc;
}

}  // extern "C"
