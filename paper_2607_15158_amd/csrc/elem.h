// Element-wise kernels of a CTMRG move (internal).
#pragma once

#include "common.h"

namespace sictm {

// Partial sums per tensor of the norm reduction (fixed, so that the norms do
// not depend on the launch).
constexpr int kNormBlocks = 128;

struct NormArgs {
  double* x[8];
  long n[8];
  double* out;    // 8 norms
  int* bad;       // set to 1 on a zero / non-finite norm
  double* part;   // 8 * kNormBlocks partial sums of squares (workspace)
};

struct SignArgs {
  double* Y[4];
  double* sg[4];
  int N, k;
  long ld;
};

struct ProjPrepArgs {
  const double* u[4];
  const double* v[4];
  const double* s[4];
  const double* sg[4];
  double* vs[4];
  double* vsc[4];
  double* usc[4];
  double* gap;   // [4] or null
  int k, keep;
  double rtol;
};

struct OverlapArgs {
  const double* G[8];   // chi x chi products Q_old^T Q_new of orthonormal blocks
  int count, chi;
  double* out;          // largest over the blocks of the mean sin^2
};

struct SpecArgs {
  const double* s[4];
  const double* old_spec;  // [4][chi]
  double* new_spec;        // [4][chi]
  double* delta;
  int x, chi;
};

// a = sum_{s,t} A[s,ket] O[t,s] A[t,bra]; O == null: identity; s_fix >= 0: the single
// (ket s_fix, bra t_fix) term (an open physical leg).
int elem_double_layer(const double* A, const double* O, double* a, int d, int D, hipStream_t s,
                      int s_fix = -1, int t_fix = -1);
int elem_pair_dot(const double* X, const double* Y, long stride, int ni, int nj, int x, int m,
                  int rev, double* out, hipStream_t s);
int elem_kappa(const double* z, double* out, hipStream_t s);
int elem_bond_value(const double* E, const double* op, int d, double* out, hipStream_t s);
// out[j] = <X, Y_j> over n doubles for ny <= kMaxDots vectors, in a fixed
// summation order; part holds kDotBlocks * ny doubles of partial sums.
constexpr int kMaxDots = 9;
constexpr int kDotBlocks = 1024;
int elem_dots(const double* X, const double* const* Y, int ny, long n, double* part,
              double* out, hipStream_t s);
// dst (cols x rows) = src (rows x cols)^T
int elem_transpose(const double* src, double* dst, long rows, long cols, hipStream_t s);
// out[0] = -1/ln(|l2|/|l1|), out[1] = |l2|/|l1|, out[2] = l1 for the two
// eigenvalues of largest modulus of the m x m row-major matrix H
// (m <= kMaxSmallEig; l1 simple and dominant).
constexpr int kMaxSmallEig = 16;
int elem_xi_from_ritz(const double* H, int m, int squarings, double* out, hipStream_t s);
int elem_ratio(const double* a, const double* b, double* out, hipStream_t s);
int elem_permute4(const double* src, void* dst, DT t, int n, long s0, long s1, long s2, long s3,
                  hipStream_t s);
int elem_init_env(const double* a, const double* e, int n, double* const* C, double* const* T,
                  hipStream_t s);
int elem_normalize(const NormArgs& na, int count, hipStream_t s);
int elem_norms(const NormArgs& na, int count, hipStream_t s);
int elem_col_sign(const SignArgs& sa, int count, hipStream_t s);
int elem_scale_cols(const SignArgs& sa, int count, hipStream_t s);
int elem_proj_prep(const ProjPrepArgs& pa, int count, hipStream_t s);

// Site absorption of the four enlarged corners through the single-layer
// tensor A ([s][u][l][d][r], real): Ct_i[(x, o1), (y, o2)] =
// sum_(p, q) W_i[(x, y), p, q] a_i[(p, q), (o1, o2)] with a_i the corner-i leg
// permutation of the double layer, given per corner as the strides in A of
// the legs (p, q, o1, o2).  float64 arithmetic, output in float64 or (out_f32)
// float32; D^2 <= 36 and d D^2 <= 72.
bool absorb_corner_fits(int D, int d);
int launch_absorb_corners(const double* const* W, void* const* Ct, bool out_f32, const double* A,
                          const long (*legs)[4], int chi, int D, int d, hipStream_t s);
// The same absorption for 1..8 problems of nR rows (W_i [nR][Dl][Dl], site
// tensor A_i) with output element (R, o1, o2) at (R / n2) ostr[0] +
// (R % n2) ostr[1] + o1 ostr[2] + o2 ostr[3] (the edges' Z2 = Z1 a of the
// renormalisation, the unit cell's corners).
int launch_absorb(int count, const double* const* W, void* const* out, bool out_f32,
                  const double* const* A, const long (*legs)[4], long nR, int n2,
                  const long* ostr, int D, int d, hipStream_t s);
// The first m singular triples of a dense SVD in descending order of the
// singular value (stable): s_out[j], U_out[:, j], Vt_out[j, :] (row-major,
// leading dimension n); perm holds n ints.
int elem_sort_triples(const double* s, const double* U, const double* Vt, int n, int m, int* perm,
                      double* s_out, double* U_out, double* Vt_out, hipStream_t st);
int elem_proj_prep_full(const double* U, const double* Vt, const double* sv, const double* sg,
                        int N, int keep, double rtol, double* Us, double* Vs, double* gap,
                        hipStream_t s);
int elem_identity(double* P, int n, int m, hipStream_t s);
int elem_zero_int(int* x, hipStream_t s);
int elem_symmetrize(double* A, int n, hipStream_t s);
int elem_symmetrize_edge(double* T, int x, int Dl, hipStream_t s);
int elem_c4v_order(const double* w, const double* V, int n, int keep, double* P, hipStream_t s);
int elem_copy_cols(const double* X, int n, long ld, int keep, double* P, hipStream_t s);
int elem_spectra_delta(const SpecArgs& sp, hipStream_t s);
int elem_sin2(const OverlapArgs& oa, hipStream_t s);
int elem_gauss(double* x, long n, uint64_t seed, hipStream_t s);
int elem_dot_rev(const double* X, const double* Y, int x, int m, double* out, hipStream_t s);
int elem_dot_rev_batched(const double* X, long xs, const double* Y, long ys, int nb, int x, int m,
                         double* out, hipStream_t s);
int elem_trace(const double* A, int n, double* out, hipStream_t s);
int elem_dot(const double* X, const double* Y, long n, double* out, hipStream_t s);

}  // namespace sictm
