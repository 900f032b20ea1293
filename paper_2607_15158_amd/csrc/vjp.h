// Internal view of a context for the adjoint of the move (vjp.hip).
#pragma once

#include <string>

#include "../../include/ctm.h"
#include "common.h"

namespace sictm {

struct VjpView {
  ctm_config cfg;
  int d, D, Dl, chi, k, N;
  hipStream_t st;
  const double* A_site;   // d x D^4 site tensor
  const double* a;        // double layer, Dl^4
  const double* ap[4];    // the corner permutations of a (float64 contractions)
  long ap_strides[4][4];  // ap[i][i0,i1,i2,i3] = a[sum_j i_j * ap_strides[i][j]]
  double* sk_part;        // partial tiles of balanced SI products (or null)
  int sk_cus;             // CUs such a launch spreads over
};

// Fills v after completing a move still in flight; 0 or a ctm_status.
int vjp_view(ctm_ctx* c, VjpView* v);
// Records msg as the context's last error and returns code.
int vjp_fail(ctm_ctx* c, int code, const std::string& msg);
// Physical dimension d of the context's site tensor.
int ctx_phys_dim(const ctm_ctx* c);

}  // namespace sictm
