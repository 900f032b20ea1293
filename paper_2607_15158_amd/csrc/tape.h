// Reverse-mode tape of float64 device computations (internal).
//
// A forward pass written against the tape allocates every result in a fresh
// device buffer (nothing is overwritten, so every value the backward pass
// needs is still there), launches its kernels and records, per operation, a
// closure that propagates cotangents.  backward() runs the closures in
// reverse order: each reads the cotangents of its outputs and adds the
// cotangents of its inputs (vector-Jacobian products).  Discrete choices of
// the forward pass (QR diagonal signs, the sign rule, the pseudo-inverse
// mask) are held fixed, as in any reverse-mode treatment of them.
//
// Sizing: a dry pass (begin_dry) runs the same forward code without device
// memory or launches and measures the value, cotangent and scratch bytes it
// needs; reserve() then allocates them and a real pass (begin) follows.
#pragma once

#include <functional>
#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace sictm {

class Tape {
 public:
  explicit Tape(hipStream_t s) : st_(s) {}
  ~Tape();
  Tape(const Tape&) = delete;
  Tape& operator=(const Tape&) = delete;

  // --- passes ---------------------------------------------------------------
  void begin_dry();                  // sizing pass: no memory, no launches
  int reserve();                     // allocates what the dry pass measured
  void begin();                      // clears the tape for a real pass
  bool dry() const { return dry_; }
  size_t bytes_reserved() const { return cap_; }

  // --- values ---------------------------------------------------------------
  double* alloc(long n);                                   // fresh, uninitialised
  // A constant value uploaded from host memory (n doubles).
  double* upload(const double* host, long n);
  // Registers caller memory read by the pass; constant: no cotangent.
  void external(const double* p, long n, bool constant);
  // Registers caller memory that receives the cotangent of the external at p
  // (written by backward(), zero-filled first).
  void external_grad(const double* p, double* g);

  // --- operations (forward launch + backward record) ------------------------
  // Float64 GEMM with the library's descriptor (no accumulate); every output
  // must be a fresh value.  Thin products with long K take the split kernel.
  int gemm(const GemmBatch& g);
  // dst (row-major over dims) = src[sum_i idx_i strides_i]; a bijection.
  int permute(const double* src, double* dst, int nd, const int* dims, const long* strides);
  // Q_i = the thin Householder QR of H_i (R_ii >= 0), n x k each.
  int qr(int count, const double* const* H, double* const* Q, int n, int k);
  // Projector factors of rho_i = u s v^T (QR-based projector section, steps
  // 2-3): the signs sg_i of the sign rule on the columns of Yt_i u (nrows x
  // k; held constant), us = u sg, vs = v sg, and the kept scaled columns
  // vsc = vs[:, :keep] sinv, usc = us[:, :keep] sinv with sinv = s^-1/2 cut
  // at rtol s_1.
  int svdproj(int count, const double* const* rho, const double* const* Yt, int nrows, int k,
              int keep, double rtol, double* const* us, double* const* vs, double* const* vsc,
              double* const* usc);
  // y_t = x_t / |x_t| for up to 8 tensors of n_t doubles.
  int normalize(int count, const double* const* x, double* const* y, const long* n);
  // out = <w1, E> / <w2, E> (one double, device), w1 and w2 constants.
  int ratio(const double* E, const double* w1, const double* w2, long n, double* out);

  // --- backward -------------------------------------------------------------
  // Adds the device vector g (n doubles) to the cotangent of the value at p.
  int seed(const double* p, const double* g, long n);
  // Adds alpha to the cotangent of the one-double value at p.
  int seed_scalar(const double* p, double alpha);
  int backward();
  // Cotangent of the value at p (allocated and zero-filled on first use);
  // nullptr for constants.
  double* grad(const double* p);
  // Cotangent if one exists already, else nullptr.
  double* grad_if(const double* p) const;
  // dst (caller device memory, n doubles) += cotangent of the value at p.
  int accumulate_grad(const double* p, double* dst, long n);
  // dst (caller device memory) = the value at src.
  int copy_out(const double* src, double* dst, long n);

  const std::string& error() const { return err_; }
  double* sk_part() const { return sk_part_; }

 private:
  struct Region {
    uintptr_t end;
    bool constant;
    double* g;        // cotangent, or null
    double* ext_g;    // caller's cotangent buffer for an external
  };
  int fail(int code, const std::string& msg);
  const Region* find(const void* p, uintptr_t* base) const;
  Region* find(const void* p, uintptr_t* base);
  bool inside(const void* p, size_t bytes) const;
  int check_gemm(const GemmBatch& g) const;
  int launch(const GemmBatch& g);
  double* tmp(long n);        // backward scratch, released by tmp_reset()
  void tmp_reset() { tmp_off_ = 0; }
  int fill(double* x, long n, double v);
  int copy(const double* src, double* dst, long n);
  int gather(const double* src, double* dst, int nd, const int* dims, const long* strides, bool acc,
             double alpha = 1.0);
  int scatter_add(const double* src, double* dst, int nd, const int* dims, const long* strides);
  int dots(int count, const double* const* x, const double* const* y, const long* n, double* out);
  int gemm_bwd(const GemmBatch& g);
  void note_tmp(size_t bytes) {
    if (bytes > tmp_need_) tmp_need_ = bytes;
  }

  hipStream_t st_;
  bool dry_ = false;
  // device memory: [values | cotangents | scratch | workspaces]
  char* mem_ = nullptr;
  size_t cap_ = 0;
  char* val_base_ = nullptr;
  size_t val_off_ = 0, val_need_ = 0;
  char* grad_base_ = nullptr;
  size_t grad_off_ = 0, grad_need_ = 0;
  char* tmp_base_ = nullptr;
  size_t tmp_off_ = 0, tmp_need_ = 0, tmp_cap_ = 0;
  void* qr_ws_ = nullptr;
  void* svd_ws_ = nullptr;
  double* sk_part_ = nullptr;
  double* part_ = nullptr;
  size_t qr_need_ = 0, svd_need_ = 0;
  std::map<uintptr_t, Region> regions_;          // values, externals
  std::vector<std::pair<uintptr_t, uintptr_t>> scratch_regions_;   // cotangents, scratch
  std::vector<std::function<int()>> back_;
  std::string err_;
};

}  // namespace sictm
