// CTMRG of an Lx x Ly unit cell on one GPU (End Matter, larger unit cells)
// and the ctm_cell_* entry points of include/ctm.h.
//
// Site (x, y) is column x and row y, periodic in both; every site carries
// its own environment C1..C4, T1..T4 in the single-site index conventions,
// each tensor with its own dimensions (they differ while the environment
// grows).  One iteration is a left, a top, a right and a bottom move; the
// move in direction d is the left move of the cell turned d times by 90
// degrees.  The turn moves no data: site (x', y') of the turned cell is a
// site of the cell, its tensor in slot i is the site's tensor in slot
// (i + d) mod 4, and enlarged corner i of the turned site is enlarged
// corner (i + d) mod 4 of the site (the corner and edge contractions are
// covariant under the turn).  A left move takes the columns in turn; for
// column x it
//   1. builds the four enlarged corners of every cluster (x, y) (sites
//      (x, y), (x+1, y), (x+1, y+1), (x, y+1); the contraction of the
//      single-site move with each site's own tensors);
//   2. builds the projectors of every cluster's left cut from
//      M = Ct3 Ct4 Ct1 Ct2 (L = Ct3 Ct4, R = Ct1 Ct2; the single-site bond
//      3): subspace iteration on the cut's own X, Y blocks (from fixed start
//      blocks in the randomized-SVD warm-up, recycled afterwards), the full
//      SVD of M, or identities while the cut is not larger than chi;
//   3. moves the left environment of column x one column to the right:
//      C1' = P_r (C1 T1), T4' = P_r (T4 a) P_l, C4' = (T3 C4) P_l, with the
//      projectors of the cuts above and below the site, each normalised to
//      unit Frobenius norm.
// Cuts of a column with equal shapes run batched (the X and Y blocks of up
// to four cuts per launch).  All launches are ordered on the cell's stream.

#include "cell.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <limits>

#include "elem.h"

using namespace sictm;

namespace {

struct CellCarver {
  char* base = nullptr;
  size_t off = 0;
  std::vector<std::pair<uintptr_t, uintptr_t>>* reg = nullptr;
  double* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    if (base && reg) reg->push_back({(uintptr_t)p, (uintptr_t)p + count * sizeof(double)});
    off += count * sizeof(double);
    return p;
  }
  void* take_bytes(size_t bytes) { return (void*)take((bytes + 7) / 8); }
};

// One cut of a column step: the four cluster corners and what the cut's
// projectors need.
struct Cut {
  int j;                 // row of the cut in the turned cell
  int site[4];           // sites of the cluster corners
  int r[4], cc[4];       // rows, cols of the corners
  int mode;              // CTM_CELL_GROW / _SVD / _RSVD / _SI
  int keep;
  int cid;               // index of the cut's blocks in its direction
};

int cfail(ctm_cell* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  set_thread_error(msg);
  return code;
}

#define CTRY(expr)                                                         \
  do {                                                                     \
    int _r = (expr);                                                       \
    if (_r != 0) {                                                         \
      if (c->err.empty()) c->err = thread_error().empty() ? #expr : thread_error(); \
      return _r == 1 ? (int)CTM_E_ARG : _r;                                \
    }                                                                      \
  } while (0)

bool inside(const ctm_cell* c, const void* p, size_t bytes) {
  const uintptr_t a = (uintptr_t)p;
  auto it = std::upper_bound(c->bufs.begin(), c->bufs.end(),
                             std::make_pair(a, std::numeric_limits<uintptr_t>::max()));
  if (it == c->bufs.begin()) return false;
  --it;
  return a >= it->first && a + bytes <= it->second;
}

long map_extent(int n, int div, long s1, long s0) {
  if (n <= 0) return 0;
  return (long)((n - 1) / div) * s1 + (long)std::min(div - 1, n - 1) * s0;
}

// Host-side bounds check of every operand of a float64 GEMM launch against
// the carved buffer that holds its base pointer; refuses to launch on a
// violation.
int check_gemm(ctm_cell* c, const GemmBatch& g) {
  if (g.M <= 0 || g.N <= 0) return 0;
  for (int i = 0; i < g.count; ++i) {
    const long ea = g.K <= 0 ? 0
                    : (g.transA[i] ? (long)(g.K - 1) * g.lda + (g.M - 1)
                                   : (long)(g.M - 1) * g.lda + (g.K - 1)) +
                          (long)(g.nbatch - 1) * g.a_bs;
    const long eb = g.K <= 0 ? 0 : (long)(g.K - 1) * g.ldb + (g.N - 1) + (long)(g.nbatch - 1) * g.b_bs;
    const long ec = map_extent(g.M, g.cdiv_m, g.cs_m1, g.cs_m0) +
                    map_extent(g.N, g.cdiv_n, g.cs_n1, g.cs_n0) + (long)(g.nbatch - 1) * g.c_bs;
    const bool ok = (g.K <= 0 || inside(c, g.A[i], (size_t)(ea + 1) * 8)) &&
                    (g.K <= 0 || inside(c, g.B[i], (size_t)(eb + 1) * 8)) &&
                    inside(c, g.C[i], (size_t)(ec + 1) * 8);
    if (!ok)
      return cfail(c, CTM_E_SHAPE,
                   "cell GEMM operand out of its buffer (M=" + std::to_string(g.M) + " N=" +
                       std::to_string(g.N) + " K=" + std::to_string(g.K) + " problem " +
                       std::to_string(i) + "); launch refused");
  }
  return 0;
}

// Launches a float64 GEMM: the split kernel of the SI applications wherever
// it applies (thin products with long K: the SI applications, rho, the
// corner and edge renormalisations), else the tile kernels.
int run(ctm_cell* c, const GemmBatch& g) {
  if (g.count == 0) return 0;
  CTRY(check_gemm(c, g));
  CTRY(launch_gemm_f64_any(g, c->sk_part, kSplitMaxCus, c->st));
  return 0;
}

// ---------------------------------------------------------------------------
// enlarged corners: Ct_i = T_(i-1) C_i T_i a, the three products of the
// single-site move with the site's own dimensions
// ---------------------------------------------------------------------------
struct CornerJob {
  int site, i;
  double* out;
  double* stem;   // W_i
  double* ct;     // C_i T_i
};

void corner_dims(const SiteEnv& e, int i, int* xin, int* ca, int* cb, int* ty) {
  const int im = (i + 3) & 3;
  *xin = e.Td[im][0];
  *ca = e.Cd[i][0];
  *cb = e.Cd[i][1];
  *ty = e.Td[i][1];
}

int check_corner(ctm_cell* c, const SiteEnv& e, int i) {
  const int im = (i + 3) & 3;
  if (e.Td[im][1] != e.Cd[i][0] || e.Cd[i][1] != e.Td[i][0])
    return cfail(c, CTM_E_SHAPE, "inconsistent environment dimensions around corner " +
                                     std::to_string(i + 1));
  return 0;
}

int build_corners(ctm_cell* c, const std::vector<CornerJob>& jobs) {
  const int Dl = c->Dl;
  for (const auto& jb : jobs) CTRY(check_corner(c, c->env[jb.site], jb.i));
  // jobs with equal dimensions share a launch (at most 8 problems)
  std::vector<bool> done(jobs.size(), false);
  for (size_t s0 = 0; s0 < jobs.size(); ++s0) {
    if (done[s0]) continue;
    int xin, ca, cb, ty;
    corner_dims(c->env[jobs[s0].site], jobs[s0].i, &xin, &ca, &cb, &ty);
    std::vector<size_t> grp;
    for (size_t t = s0; t < jobs.size() && grp.size() < 8; ++t) {
      if (done[t]) continue;
      int a1, a2, a3, a4;
      corner_dims(c->env[jobs[t].site], jobs[t].i, &a1, &a2, &a3, &a4);
      if (a1 == xin && a2 == ca && a3 == cb && a4 == ty) {
        grp.push_back(t);
        done[t] = true;
      }
    }
    // CT_i[a, (y, q)] = C_i[a, b] T_i[b, q, y]
    GemmBatch g1 = gemm_of(ca, Dl * ty, cb, cb, (long)Dl * ty, 0);
    g1.cdiv_m = 1 << 30; g1.cs_m1 = 0; g1.cs_m0 = (long)Dl * ty;
    g1.cdiv_n = ty; g1.cs_n1 = 1; g1.cs_n0 = Dl;
    // W_i[(x_in, y), (p, q)] = T_(i-1)[(x_in, p), a] CT_i[a, (y, q)]
    GemmBatch g2 = gemm_of(xin * Dl, Dl * ty, ca, ca, (long)Dl * ty, 0);
    g2.cdiv_m = Dl; g2.cs_m1 = (long)ty * Dl * Dl; g2.cs_m0 = Dl;
    g2.cdiv_n = Dl; g2.cs_n1 = (long)Dl * Dl; g2.cs_n0 = 1;
    // Ct_i[(x_in, o1), (y, o2)] = W_i[(x_in, y), (p, q)] site_i[(p, q), (o1, o2)]
    GemmBatch g3 = gemm_of(xin * ty, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
    g3.cdiv_m = ty; g3.cs_m1 = (long)Dl * ty * Dl; g3.cs_m0 = Dl;
    g3.cdiv_n = Dl; g3.cs_n1 = (long)ty * Dl; g3.cs_n0 = 1;
    for (size_t t : grp) {
      const CornerJob& jb = jobs[t];
      const SiteEnv& e = c->env[jb.site];
      add(g1, e.C[jb.i], e.T[jb.i], jb.ct);
      add(g2, e.T[(jb.i + 3) & 3], jb.ct, jb.stem);
      add(g3, jb.stem, c->ap[jb.site * 4 + jb.i], jb.out);
    }
    CTRY(run(c, g1));
    CTRY(run(c, g2));
    CTRY(run(c, g3));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// projectors of a group of cuts with equal shapes
// ---------------------------------------------------------------------------
// Applies op(Q) to the X-side and Y-side blocks of the cuts: X side through
// corner qx (transposed if tx), Y side through qy (ty).
int apply_pair(ctm_cell* c, const std::vector<const Cut*>& g, int qx, int tx, int qy, int ty_,
               double* const* xin, double* const* xout, double* const* yin, double* const* yout) {
  const Cut& c0 = *g[0];
  const int k = c->k;
  const int Mx = tx ? c0.cc[qx] : c0.r[qx], Kx = tx ? c0.r[qx] : c0.cc[qx];
  const int My = ty_ ? c0.cc[qy] : c0.r[qy], Ky = ty_ ? c0.r[qy] : c0.cc[qy];
  const long ldx = c0.cc[qx], ldy = c0.cc[qy];
  const int n = (int)g.size();
  if (Mx == My && Kx == Ky && ldx == ldy) {
    GemmBatch gb = gemm_of(Mx, k, Kx, ldx, k, k);
    for (int i = 0; i < n; ++i) add(gb, c->Q[g[i]->j * 4 + qx], xin[i], xout[i], tx);
    for (int i = 0; i < n; ++i) add(gb, c->Q[g[i]->j * 4 + qy], yin[i], yout[i], ty_);
    return run(c, gb);
  }
  GemmBatch gx = gemm_of(Mx, k, Kx, ldx, k, k);
  for (int i = 0; i < n; ++i) add(gx, c->Q[g[i]->j * 4 + qx], xin[i], xout[i], tx);
  CTRY(run(c, gx));
  GemmBatch gy = gemm_of(My, k, Ky, ldy, k, k);
  for (int i = 0; i < n; ++i) add(gy, c->Q[g[i]->j * 4 + qy], yin[i], yout[i], ty_);
  return run(c, gy);
}

int qr_blocks(ctm_cell* c, std::vector<double*> w, int n) {
  if (!qr_plan_ok(n, c->k))
    return cfail(c, CTM_E_SHAPE, "no QR leaf partition for a cut block of " + std::to_string(n) +
                                     " x " + std::to_string(c->k));
  CTRY(launch_qr((int)w.size(), w.data(), n, c->k, c->qr_ws, c->st));
  return 0;
}

// SI projectors (QR-based projector section, steps 1-3, with the blocks
// of each cut); recycle: the blocks are the cut's current ones and X v,
// Y^T u replace them (eq. xy_recycle), else the start blocks, unchanged
// (the randomized SVD of the warm-up).
int si_group(ctm_cell* c, int d, const std::vector<const Cut*>& g, bool recycle) {
  const int k = c->k, n = (int)g.size();
  const Cut& c0 = *g[0];
  const int nb = c0.cc[1];          // rows of the blocks (= r[2])
  const int ncut = c0.cc[3];        // the cut (= r[0])
  std::vector<double*> xc(n), yc(n), xo(n), yo(n), tmpx(n), tmpy(n), Am(n), Bt(n);
  // per-cut work blocks: B[j*6 + 0/1] X chain, 2/3 Y chain, 4 A, 5 B^T
  auto blk = [&](int i, int s) { return c->B[g[i]->j * 6 + s]; };
  for (int i = 0; i < n; ++i) {
    const int id = d * c->ns + g[i]->cid;
    xc[i] = recycle ? c->X[id] : c->X0[id];
    yc[i] = recycle ? c->Y[id] : c->Y0[id];
  }
  auto other = [&](int i, double* cur, int s0) { return cur == blk(i, s0) ? blk(i, s0 + 1) : blk(i, s0); };
  // one half step: X through M (or M^T), Y through the other; results in
  // work blocks, then orthonormalised when asked
  auto half = [&](bool x_with_M, bool qr) -> int {
    // M W = Q3 Q4 Q1 Q2 W; M^T W = Q2^T Q1^T Q4^T Q3^T W
    const int mq[4] = {1, 0, 3, 2}, tq[4] = {2, 3, 0, 1};
    for (int t = 0; t < 4; ++t) {
      std::vector<double*> xi(n), xq(n), yi(n), yq(n);
      for (int i = 0; i < n; ++i) {
        xi[i] = xc[i];
        xq[i] = other(i, xc[i], 0);
        yi[i] = yc[i];
        yq[i] = other(i, yc[i], 2);
      }
      const int qx = x_with_M ? mq[t] : tq[t], tx = x_with_M ? 0 : 1;
      const int qy = x_with_M ? tq[t] : mq[t], tyy = x_with_M ? 1 : 0;
      CTRY(apply_pair(c, g, qx, tx, qy, tyy, xi.data(), xq.data(), yi.data(), yq.data()));
      xc = xq;
      yc = yq;
    }
    if (qr) {
      std::vector<double*> w;
      for (int i = 0; i < n; ++i) {
        w.push_back(xc[i]);
        w.push_back(yc[i]);
      }
      CTRY(qr_blocks(c, w, nb));
    }
    return 0;
  };
  for (int step = 0; step < c->cfg.n_si; ++step) {
    if (c->cfg.stabilized) {
      CTRY(half(true, true));
      CTRY(half(false, true));
    } else {
      CTRY(half(true, false));
      CTRY(half(false, true));
    }
  }
  // A = Q1 (Q2 X), B^T = Q4^T (Q3^T Y^T)
  for (int i = 0; i < n; ++i) {
    tmpx[i] = other(i, xc[i], 0);
    tmpy[i] = other(i, yc[i], 2);
    Am[i] = blk(i, 4);
    Bt[i] = blk(i, 5);
  }
  CTRY(apply_pair(c, g, 1, 0, 2, 1, xc.data(), tmpx.data(), yc.data(), tmpy.data()));
  CTRY(apply_pair(c, g, 0, 0, 3, 1, tmpx.data(), Am.data(), tmpy.data(), Bt.data()));
  // rho = (B^T)^T A
  {
    GemmBatch gr = gemm_of(k, k, ncut, k, k, k);
    for (int i = 0; i < n; ++i) add(gr, Bt[i], Am[i], c->rho[g[i]->j], 1);
    CTRY(run(c, gr));
  }
  {
    std::vector<const double*> rp(n);
    std::vector<double*> up(n), sp(n), vp(n);
    for (int i = 0; i < n; ++i) {
      rp[i] = c->rho[g[i]->j];
      up[i] = c->u[g[i]->j];
      sp[i] = c->s[g[i]->j];
      vp[i] = c->v[g[i]->j];
    }
    CTRY(launch_svd(n, rp.data(), up.data(), sp.data(), vp.data(), k, c->svd_ws, c->st));
  }
  // Y^T u (its column signs are the sign rule's), into the spare Y block
  {
    GemmBatch gy = gemm_of(nb, k, k, k, k, k);
    for (int i = 0; i < n; ++i) add(gy, yc[i], c->u[g[i]->j], tmpy[i]);
    CTRY(run(c, gy));
  }
  SignArgs sa{};
  sa.N = nb;
  sa.k = k;
  sa.ld = k;
  for (int i = 0; i < n; ++i) {
    sa.Y[i] = tmpy[i];
    sa.sg[i] = c->sg[g[i]->j];
  }
  CTRY(elem_col_sign(sa, n, c->st));
  CTRY(elem_scale_cols(sa, n, c->st));
  const int keep = c0.keep;
  ProjPrepArgs pa{};
  pa.k = k;
  pa.keep = keep;
  pa.rtol = c->cfg.pinv_rtol;
  pa.gap = nullptr;
  for (int i = 0; i < n; ++i) {
    const int j = g[i]->j;
    pa.u[i] = c->u[j];
    pa.v[i] = c->v[j];
    pa.s[i] = c->s[j];
    pa.sg[i] = c->sg[j];
    pa.vs[i] = c->vs[j];
    pa.vsc[i] = c->vsc[j];
    pa.usc[i] = c->usc[j];
  }
  CTRY(elem_proj_prep(pa, n, c->st));
  // P_l = A vsc, P_r^T = B^T usc
  {
    GemmBatch gp = gemm_of(ncut, keep, k, k, keep, keep);
    for (int i = 0; i < n; ++i) {
      add(gp, Am[i], c->vsc[g[i]->j], c->Pl[g[i]->j]);
      add(gp, Bt[i], c->usc[g[i]->j], c->Prt[g[i]->j]);
    }
    CTRY(run(c, gp));
  }
  if (recycle) {
    // X <- X vs into the spare X block; the blocks become the cut's own
    GemmBatch gx = gemm_of(nb, k, k, k, k, k);
    for (int i = 0; i < n; ++i) add(gx, xc[i], c->vs[g[i]->j], tmpx[i]);
    CTRY(run(c, gx));
    for (int i = 0; i < n; ++i) {
      const int id = d * c->ns + g[i]->cid;
      // swap the pointers of the new blocks and the cut's old ones
      for (int s = 0; s < 6; ++s) {
        double*& w = c->B[g[i]->j * 6 + s];
        if (w == tmpx[i]) w = c->X[id];
        else if (w == tmpy[i]) w = c->Y[id];
      }
      c->X[id] = tmpx[i];
      c->Y[id] = tmpy[i];
    }
  }
  return 0;
}

// Projectors from the full SVD of M (Standard CTMRG section) for one cut.
int svd_cut(ctm_cell* c, const Cut& q) {
  const int j = q.j, nb = q.cc[1], keep = q.keep;
  double *R = c->F[0], *L = c->F[1], *M = c->F[2], *Ut = c->F[3], *Uv = c->F[4], *Us2 = c->F[5],
         *Vt2 = c->F[6], *Us = c->F[7], *Vs = c->F[8];
  if (!c->rb) {
    if (rocblas_create_handle(&c->rb) != rocblas_status_success)
      return cfail(c, CTM_E_DEVICE, "rocblas_create_handle failed");
    rocblas_set_stream(c->rb, c->st);
  }
  {
    GemmBatch g = gemm_of(q.r[0], q.cc[1], q.cc[0], q.cc[0], q.cc[1], q.cc[1]);
    add(g, c->Q[j * 4 + 0], c->Q[j * 4 + 1], R);
    CTRY(run(c, g));
  }
  {
    GemmBatch g = gemm_of(q.r[2], q.cc[3], q.cc[2], q.cc[2], q.cc[3], q.cc[3]);
    add(g, c->Q[j * 4 + 2], c->Q[j * 4 + 3], L);
    CTRY(run(c, g));
  }
  {
    GemmBatch g = gemm_of(q.r[2], q.cc[1], q.cc[3], q.cc[3], q.cc[1], q.cc[1]);
    add(g, L, R, M);
    CTRY(run(c, g));
  }
  // rocSOLVER is column-major: it decomposes M^T = V S U^T, so its left
  // vectors are V^T of M and its right vectors U of M, both row-major
  const rocblas_status st =
      rocsolver_dgesvd(c->rb, rocblas_svect_singular, rocblas_svect_singular, nb, nb, M, nb, c->fs,
                       Ut, nb, Uv, nb, c->fE, rocblas_outofplace, c->finfo);
  if (st != rocblas_status_success)
    return cfail(c, CTM_E_DEVICE, "rocSOLVER SVD failed: " + std::to_string((int)st));
  const int m = std::min(nb, keep + 1);
  CTRY(elem_sort_triples(c->fs, Uv, Ut, nb, m, c->fperm, c->fE, Us2, Vt2, c->st));
  SignArgs sa{};
  sa.N = nb;
  sa.k = keep;
  sa.ld = nb;
  sa.Y[0] = Us2;
  sa.sg[0] = c->fsg;
  CTRY(elem_col_sign(sa, 1, c->st));
  CTRY(elem_proj_prep_full(Us2, Vt2, c->fE, c->fsg, nb, keep, c->cfg.pinv_rtol, Us, Vs, nullptr,
                           c->st));
  // P_l = R Vs, P_r^T = L^T Us
  {
    GemmBatch g = gemm_of(q.r[0], keep, nb, nb, keep, keep);
    add(g, R, Vs, c->Pl[j]);
    CTRY(run(c, g));
  }
  {
    GemmBatch g = gemm_of(q.cc[3], keep, nb, q.cc[3], keep, keep);
    add(g, L, Us, c->Prt[j], 1);
    CTRY(run(c, g));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// one column of a left move in the turned cell of direction d
// ---------------------------------------------------------------------------
int column_step(ctm_cell* c, int d, int xt, int mode) {
  const int H = height(c, d), W = width(c, d), Dl = c->Dl, chi = c->chi, k = c->k;
  std::vector<Cut> cuts(H);
  std::vector<CornerJob> jobs;
  for (int y = 0; y < H; ++y) {
    Cut& q = cuts[y];
    q.j = y;
    q.cid = y * W + xt;
    q.site[0] = site_of(c, d, xt, y);
    q.site[1] = site_of(c, d, xt + 1, y);
    q.site[2] = site_of(c, d, xt + 1, y + 1);
    q.site[3] = site_of(c, d, xt, y + 1);
    for (int i = 0; i < 4; ++i) {
      const int ci = (i + d) & 3;
      const SiteEnv& e = c->env[q.site[i]];
      int xin, ca, cb, ty;
      corner_dims(e, ci, &xin, &ca, &cb, &ty);
      q.r[i] = xin * Dl;
      q.cc[i] = ty * Dl;
      jobs.push_back(CornerJob{q.site[i], ci, c->Q[y * 4 + i], c->Wst[y * 4 + i], c->CT[y * 4 + i]});
    }
    for (int i = 0; i < 4; ++i)
      if (q.cc[i] != q.r[(i + 1) & 3])
        return cfail(c, CTM_E_SHAPE, "cluster corners of a cut do not chain");
  }
  CTRY(build_corners(c, jobs));
  // the mode of every cut
  for (auto& q : cuts) {
    const int ncut = q.cc[3], nb = q.cc[1];
    const int x_env = c->env[q.site[0]].Cd[d & 3][0];
    if (ncut <= chi) {
      q.mode = CTM_CELL_GROW;
      q.keep = ncut;
    } else if (mode == CTM_CELL_SVD || (mode == CTM_CELL_SI && x_env != chi) ||
               (mode == CTM_CELL_RSVD && std::min(nb, q.r[2]) < k)) {
      q.mode = CTM_CELL_SVD;
      q.keep = std::min(chi, nb);
    } else {
      q.mode = mode;
      q.keep = std::min(chi, k);
    }
  }
  // projectors: identities, full SVDs, and SI groups of equal shapes
  std::vector<bool> done(H, false);
  for (int y = 0; y < H; ++y) {
    if (done[y]) continue;
    const Cut& q = cuts[y];
    if (q.mode == CTM_CELL_GROW) {
      CTRY(elem_identity(c->Pl[y], q.keep, q.keep, c->st));
      CTRY(elem_identity(c->Prt[y], q.keep, q.keep, c->st));
      done[y] = true;
      continue;
    }
    if (q.mode == CTM_CELL_SVD) {
      CTRY(svd_cut(c, q));
      done[y] = true;
      continue;
    }
    std::vector<const Cut*> grp;
    for (int t = y; t < H && (int)grp.size() < kCutsPerLaunch; ++t) {
      const Cut& o = cuts[t];
      if (done[t] || o.mode != q.mode) continue;
      bool same = true;
      for (int i = 0; i < 4; ++i) same = same && o.r[i] == q.r[i] && o.cc[i] == q.cc[i];
      if (same) {
        grp.push_back(&o);
        done[t] = true;
      }
    }
    CTRY(si_group(c, d, grp, q.mode == CTM_CELL_SI));
  }
  // move the left environment of column xt to column xt + 1
  const int sC1 = d & 3, sT1 = d & 3, sT3 = (2 + d) & 3, sC4 = (3 + d) & 3, sT4 = (3 + d) & 3;
  std::vector<std::array<int, 6>> nd(H);   // new dims: C1 (2), T4 (2), C4 (2)
  NormArgs na{};
  int nn = 0;
  auto flush_norms = [&]() -> int {
    if (nn == 0) return 0;
    na.out = c->scal;
    na.bad = c->bad;
    na.part = c->norm_part;
    CTRY(elem_normalize(na, nn, c->st));
    nn = 0;
    return 0;
  };
  for (int y = 0; y < H; ++y) {
    const int yu = imod(y - 1, H);
    const Cut& up = cuts[yu];
    const Cut& dn = cuts[y];
    const SiteEnv& e = c->env[dn.site[0]];
    const int p0 = e.Cd[sC1][0], p1 = e.Cd[sC1][1], p2 = e.Td[sT1][1];
    const int q5 = e.Td[sT3][0], q6 = e.Td[sT3][1], q7 = e.Cd[sC4][1];
    const int t_in = e.Td[sT4][0], t_out = e.Td[sT4][1];
    const int ku = up.keep, ky = dn.keep;
    if (e.Td[sT1][0] != p1 || e.Cd[sC4][0] != q6 || up.cc[3] != p0 * Dl || up.r[0] != t_out * Dl ||
        dn.r[0] != q7 * Dl || dn.cc[3] != t_in * Dl)
      return cfail(c, CTM_E_SHAPE, "projector and environment dimensions disagree in a left move");
    double* nC1 = c->spare[y * 3 + 0];
    double* nT4 = c->spare[y * 3 + 1];
    double* nC4 = c->spare[y * 3 + 2];
    double* tmp = c->Z1[y];
    double* tmp2 = c->Z2[y];
    // C1' = P_r(up)^T (C1 T1):  (C1 T1)[(a, u), g]
    {
      GemmBatch g = gemm_of(p0, Dl * p2, p1, p1, (long)Dl * p2, (long)Dl * p2);
      add(g, e.C[sC1], e.T[sT1], tmp);
      CTRY(run(c, g));
      GemmBatch g2 = gemm_of(ku, p2, p0 * Dl, ku, p2, p2);
      add(g2, c->Prt[yu], tmp, nC1, 1);
      CTRY(run(c, g2));
    }
    // C4' = (T3 C4) P_l(dn): Y[z, t, d] = T3[(z, d), n] C4[n, t]
    {
      GemmBatch g = gemm_of(q5 * Dl, q7, q6, q6, q7, 0);
      g.cdiv_m = Dl; g.cs_m1 = (long)q7 * Dl; g.cs_m0 = 1;
      g.cdiv_n = 1 << 30; g.cs_n1 = 0; g.cs_n0 = Dl;
      add(g, e.T[sT3], e.C[sC4], tmp);
      CTRY(run(c, g));
      GemmBatch g2 = gemm_of(q5, ky, q7 * Dl, (long)q7 * Dl, ky, ky);
      add(g2, tmp, c->Pl[y], nC4);
      CTRY(run(c, g2));
    }
    // T4' = P_r(dn)^T (T4 a) P_l(up), as the single-site edge renormalisation
    {
      // Z1[(b, g'), (r, u)] = sum_g T4[(b, u), g] P_l[(g, r), g']   (batched over r)
      GemmBatch g = gemm_of(t_in * Dl, ku, t_out, t_out, (long)Dl * ku, 0);
      g.cdiv_m = Dl; g.cs_m1 = (long)ku * Dl * Dl; g.cs_m0 = 1;
      g.cdiv_n = 1 << 30; g.cs_n1 = 0; g.cs_n0 = (long)Dl * Dl;
      g.nbatch = Dl; g.a_bs = 0; g.b_bs = ku; g.c_bs = Dl;
      add(g, e.T[sT4], c->Pl[yu], tmp);
      CTRY(run(c, g));
      // Z2[(b, l), d, g'] = Z1[(b, g'), (r, u)] apr[(r, u), (l, d)]
      GemmBatch g2 = gemm_of(t_in * ku, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
      g2.cdiv_m = ku; g2.cs_m1 = (long)Dl * Dl * ku; g2.cs_m0 = 1;
      g2.cdiv_n = Dl; g2.cs_n1 = (long)Dl * ku; g2.cs_n0 = ku;
      add(g2, tmp, c->apr[dn.site[0] * 4 + ((sT4 + 1) & 3)], tmp2);
      CTRY(run(c, g2));
      // T4'[b', (d, g')] = sum_(b, l) P_r^T[(b, l), b'] Z2[(b, l), (d, g')], as its transpose
      GemmBatch g3 = gemm_of(Dl * ku, ky, t_in * Dl, (long)Dl * ku, ky, 0);
      g3.cdiv_m = 1 << 30; g3.cs_m1 = 0; g3.cs_m0 = 1;
      g3.cdiv_n = 1 << 30; g3.cs_n1 = 0; g3.cs_n0 = (long)Dl * ku;
      add(g3, tmp2, c->Prt[y], nT4, 1);
      CTRY(run(c, g3));
    }
    nd[y] = {ku, p2, ky, ku, q5, ky};
    if (nn + 3 > 8) CTRY(flush_norms());
    na.x[nn] = nC1; na.n[nn] = (long)ku * p2; ++nn;
    na.x[nn] = nT4; na.n[nn] = (long)ky * Dl * ku; ++nn;
    na.x[nn] = nC4; na.n[nn] = (long)q5 * ky; ++nn;
  }
  CTRY(flush_norms());
  // the new tensors become those of column xt + 1 (old buffers become spares)
  for (int y = 0; y < H; ++y) {
    SiteEnv& t = c->env[site_of(c, d, xt + 1, y)];
    std::swap(t.C[sC1], c->spare[y * 3 + 0]);
    std::swap(t.T[sT4], c->spare[y * 3 + 1]);
    std::swap(t.C[sC4], c->spare[y * 3 + 2]);
    t.Cd[sC1][0] = nd[y][0]; t.Cd[sC1][1] = nd[y][1];
    t.Td[sT4][0] = nd[y][2]; t.Td[sT4][1] = nd[y][3];
    t.Cd[sC4][0] = nd[y][4]; t.Cd[sC4][1] = nd[y][5];
  }
  return 0;
}

// ---------------------------------------------------------------------------
// corner spectra of every site and the convergence measure
// ---------------------------------------------------------------------------
__global__ void k_pad(const double* __restrict__ src, int r, int cols, double* __restrict__ dst, int S) {
  const long total = (long)S * S;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int a = (int)(i / S), b = (int)(i % S);
    dst[i] = (a < r && b < cols) ? src[(long)a * cols + b] : 0.0;
  }
}

// Spectra of the current corners into spec[1 - spec_cur]; the largest change
// against spec[spec_cur] in *delta (host), or no comparison when delta is null.
int spectra(ctm_cell* c, double* delta) {
  const int chi = c->chi, nc = c->ns * 4;
  for (int s = 0; s < c->ns; ++s)
    for (int i = 0; i < 4; ++i) {
      const SiteEnv& e = c->env[s];
      k_pad<<<std::min(1024, (chi * chi + 255) / 256), 256, 0, c->st>>>(
          e.C[i], e.Cd[i][0], e.Cd[i][1], c->cpad[s * 4 + i], chi);
    }
  CTM_HIP_TRY(hipGetLastError());
  for (int b = 0; b < nc; b += 8) {
    const int cnt = std::min(8, nc - b);
    CTRY(launch_svd(cnt, (const double* const*)&c->cpad[b], nullptr, &c->csv[b], nullptr, chi,
                    c->svd_ws, c->st));
  }
  for (int s = 0; s < c->ns; ++s) {
    SpecArgs sp{};
    for (int i = 0; i < 4; ++i) sp.s[i] = c->csv[s * 4 + i];
    sp.old_spec = c->spec[c->spec_cur] + (long)s * 4 * chi;
    sp.new_spec = c->spec[1 - c->spec_cur] + (long)s * 4 * chi;
    sp.delta = c->scal + 64 + s;
    sp.x = chi;
    sp.chi = chi;
    CTRY(elem_spectra_delta(sp, c->st));
  }
  std::vector<double> dl(c->ns);
  int badv = 0;
  CTM_HIP_TRY(hipMemcpyAsync(dl.data(), c->scal + 64, c->ns * 8, hipMemcpyDeviceToHost, c->st));
  CTM_HIP_TRY(hipMemcpyAsync(&badv, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->st));
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  c->spec_cur = 1 - c->spec_cur;
  if (badv) return cfail(c, CTM_E_NUMERIC, "zero or non-finite norm of a new environment tensor");
  if (delta) {
    double m = 0.0;
    for (double x : dl) m = std::max(m, x);
    *delta = m;
  }
  return 0;
}

int iteration(ctm_cell* c, int mode, double* delta) {
  if (mode == CTM_CELL_SI && c->last_mode != CTM_CELL_SI) {
    // the subspace iteration starts from the start blocks
    const size_t nk = (size_t)c->Nf * c->k * 8;
    for (int i = 0; i < 4 * c->ns; ++i) {
      CTM_HIP_TRY(hipMemcpyAsync(c->X[i], c->X0[i], nk, hipMemcpyDeviceToDevice, c->st));
      CTM_HIP_TRY(hipMemcpyAsync(c->Y[i], c->Y0[i], nk, hipMemcpyDeviceToDevice, c->st));
    }
  }
  for (int d = 0; d < 4; ++d)
    for (int xt = 0; xt < width(c, d); ++xt) CTRY(column_step(c, d, xt, mode));
  CTRY(spectra(c, delta));
  c->last_mode = mode;
  ++c->iterations;
  return 0;
}

// ---------------------------------------------------------------------------
// initial environment: every tensor from the neighbour in its direction with
// its outer legs closed by the boundary vectors of that neighbour
// ---------------------------------------------------------------------------
struct InitArgs {
  const double* a[8];    // neighbour network tensors, in the order C1 T1 C2 T2 C3 T3 C4 T4
  const double* e[8][2]; // closing vectors (legs in the order of the contraction)
  double* out[8];
  int Dl;
};

// C1[d,r] = a[u,l,d,r] e_u e_l     T1[l,d,r] = a[u,l,d,r] e_u
// C2[l,d] = a[u,l,d,r] e_u e_r     T2[u,l,d] = a[u,l,d,r] e_r
// C3[u,l] = a[u,l,d,r] e_d e_r     T3[r,u,l] = a[u,l,d,r] e_d
// C4[r,u] = a[u,l,d,r] e_l e_d     T4[d,r,u] = a[u,l,d,r] e_l
__global__ void k_cell_init(InitArgs ia) {
  const int t = blockIdx.y, n = ia.Dl;
  const long n2 = (long)n * n, n3 = n2 * n;
  const bool corner = (t % 2) == 0;
  const long total = corner ? n2 : n3;
  const double* a = ia.a[t];
  const long su = n3, sl = n2, sd = n, sr = 1;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    if (corner) {
      const int o1 = (int)(i / n), o2 = (int)(i % n);
      const double* e0 = ia.e[t][0];
      const double* e1 = ia.e[t][1];
      for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
          long off;
          switch (t) {
            case 0: off = p * su + q * sl + o1 * sd + o2 * sr; break;   // u, l | d, r
            case 2: off = p * su + q * sr + o1 * sl + o2 * sd; break;   // u, r | l, d
            case 4: off = p * sd + q * sr + o1 * su + o2 * sl; break;   // d, r | u, l
            default: off = p * sl + q * sd + o1 * sr + o2 * su; break;  // l, d | r, u
          }
          acc += a[off] * e0[p] * e1[q];
        }
    } else {
      const int o1 = (int)(i / n2), o2 = (int)((i / n) % n), o3 = (int)(i % n);
      const double* e0 = ia.e[t][0];
      for (int p = 0; p < n; ++p) {
        long off;
        switch (t) {
          case 1: off = p * su + o1 * sl + o2 * sd + o3 * sr; break;   // u | l, d, r
          case 3: off = p * sr + o1 * su + o2 * sl + o3 * sd; break;   // r | u, l, d
          case 5: off = p * sd + o1 * sr + o2 * su + o3 * sl; break;   // d | r, u, l
          default: off = p * sl + o1 * sd + o2 * sr + o3 * su; break;  // l | d, r, u
        }
        acc += a[off] * e0[p];
      }
    }
    ia.out[t][i] = acc;
  }
}

int init_env(ctm_cell* c, const double* bvec) {
  const int Dl = c->Dl;
  // neighbour offsets of C1 T1 C2 T2 C3 T3 C4 T4 and the legs they close
  // (leg index: 0 u, 1 l, 2 d, 3 r)
  const int off[8][2] = {{-1, -1}, {0, -1}, {1, -1}, {1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}};
  const int legs[8][2] = {{0, 1}, {0, 0}, {0, 3}, {3, 3}, {2, 3}, {2, 2}, {1, 2}, {1, 1}};
  for (int y = 0; y < c->Ly; ++y)
    for (int x = 0; x < c->Lx; ++x) {
      const int s = y * c->Lx + x;
      InitArgs ia{};
      ia.Dl = Dl;
      for (int t = 0; t < 8; ++t) {
        const int nx = imod(x + off[t][0], c->Lx), ny = imod(y + off[t][1], c->Ly);
        const int ns = ny * c->Lx + nx;
        ia.a[t] = c->a[ns];
        for (int l = 0; l < 2; ++l) ia.e[t][l] = bvec + ((long)ns * 4 + legs[t][l]) * Dl;
        ia.out[t] = (t % 2 == 0) ? c->env[s].C[t / 2] : c->env[s].T[t / 2];
      }
      const long n3 = (long)Dl * Dl * Dl;
      k_cell_init<<<dim3((unsigned)std::min<long>(1024, (n3 + 255) / 256), 8), 256, 0, c->st>>>(ia);
      CTM_HIP_TRY(hipGetLastError());
      SiteEnv& e = c->env[s];
      for (int i = 0; i < 4; ++i) {
        e.Cd[i][0] = e.Cd[i][1] = Dl;
        e.Td[i][0] = e.Td[i][1] = Dl;
      }
      NormArgs na{};
      for (int i = 0; i < 4; ++i) {
        na.x[i] = e.C[i];
        na.n[i] = (long)Dl * Dl;
        na.x[4 + i] = e.T[i];
        na.n[4 + i] = (long)Dl * Dl * Dl;
      }
      na.out = c->scal;
      na.bad = c->bad;
      na.part = c->norm_part;
      CTRY(elem_normalize(na, 8, c->st));
    }
  return 0;
}

int validate_cell(const ctm_cell_config* cfg) {
  if (!cfg) return cfail(nullptr, CTM_E_ARG, "null cell config");
  if (cfg->Lx < 1 || cfg->Ly < 1 || cfg->Lx > kCellMaxSide || cfg->Ly > kCellMaxSide)
    return cfail(nullptr, CTM_E_SHAPE, "need 1 <= Lx, Ly <= 16");
  if (cfg->d < 0 || cfg->D < 1 || cfg->chi < 1 || cfg->p < 0 || cfg->n_si < 0)
    return cfail(nullptr, CTM_E_SHAPE, "need d >= 0, D >= 1, chi >= 1, p >= 0, n_si >= 0");
  if (!(cfg->pinv_rtol >= 0.0)) return cfail(nullptr, CTM_E_ARG, "pinv_rtol must be >= 0");
  const int Dl = cfg->d > 0 ? cfg->D * cfg->D : cfg->D;
  if (cfg->chi < Dl)
    return cfail(nullptr, CTM_E_SHAPE, "the cell needs chi >= the network bond dimension");
  const long N = (long)cfg->chi * Dl;
  const long k = std::min<long>(cfg->chi + cfg->p, N);
  if (k > 192 || cfg->chi > 192) return cfail(nullptr, CTM_E_SHAPE, "need chi + p <= 192");
  if (N > 65536) return cfail(nullptr, CTM_E_SHAPE, "chi * Dl must be <= 65536");
  return CTM_OK;
}

size_t carve_cell(ctm_cell* c, char* base) {
  CellCarver cv;
  cv.base = base;
  c->bufs.clear();
  cv.reg = &c->bufs;
  const size_t Dl = c->Dl, chi = c->chi, N = c->Nf, k = c->k, ns = c->ns, L = c->Lmax;
  const size_t Dl4 = Dl * Dl * Dl * Dl;
  const size_t envsz = chi * Dl * chi;   // every environment buffer holds an edge
  const int dd = std::max(1, c->cfg.d);
  for (size_t s = 0; s < ns; ++s) {
    c->A[s] = cv.take(c->cfg.d > 0 ? (size_t)dd * c->cfg.D * c->cfg.D * c->cfg.D * c->cfg.D : 1);
    c->a[s] = cv.take(Dl4);
    for (int i = 0; i < 4; ++i) {
      c->ap[s * 4 + i] = cv.take(Dl4);
      c->apr[s * 4 + i] = cv.take(Dl4);
      c->env[s].C[i] = cv.take(envsz);
      c->env[s].T[i] = cv.take(envsz);
    }
  }
  for (size_t i = 0; i < L * 3; ++i) c->spare[i] = cv.take(envsz);
  for (size_t i = 0; i < 4 * ns; ++i) {
    c->X0[i] = cv.take(N * k);
    c->Y0[i] = cv.take(N * k);
    c->X[i] = cv.take(N * k);
    c->Y[i] = cv.take(N * k);
  }
  for (size_t i = 0; i < L * 4; ++i) {
    c->Q[i] = cv.take(N * N);
    c->Wst[i] = cv.take(N * N);
    c->CT[i] = cv.take(envsz);
  }
  for (size_t i = 0; i < L * 6; ++i) c->B[i] = cv.take(N * k);
  for (size_t j = 0; j < L; ++j) {
    c->rho[j] = cv.take(k * k);
    c->u[j] = cv.take(k * k);
    c->v[j] = cv.take(k * k);
    c->vs[j] = cv.take(k * k);
    c->s[j] = cv.take(k);
    c->sg[j] = cv.take(k);
    c->vsc[j] = cv.take(k * chi);
    c->usc[j] = cv.take(k * chi);
    c->Pl[j] = cv.take(N * chi);
    c->Prt[j] = cv.take(N * chi);
    c->Z1[j] = cv.take(chi * chi * Dl * Dl);
    c->Z2[j] = cv.take(chi * chi * Dl * Dl);
  }
  for (int i = 0; i < 9; ++i) c->F[i] = cv.take(N * N);
  c->fs = cv.take(N);
  c->fE = cv.take(N);
  c->fsg = cv.take(N);
  c->finfo = (int*)cv.take(8);
  c->fperm = (int*)cv.take((N + 1) / 2);
  for (size_t i = 0; i < 4 * ns; ++i) {
    c->cpad[i] = cv.take(chi * chi);
    c->csv[i] = cv.take(chi);
  }
  c->spec[0] = cv.take(4 * ns * chi);
  c->spec[1] = cv.take(4 * ns * chi);
  c->bvec = cv.take(ns * 4 * Dl);
  c->scal = cv.take(64 + ns);
  c->bad = (int*)cv.take(8);
  c->norm_part = cv.take(8 * kNormBlocks);
  c->qr_ws = cv.take_bytes(qr_workspace_bytes(8, (int)N, (int)k));
  c->svd_ws = cv.take_bytes(svd_workspace_bytes(8, (int)std::max(k, chi)));
  c->sk_part = (double*)cv.take_bytes(gemm_si_scratch_bytes());
  std::sort(c->bufs.begin(), c->bufs.end());
  return cv.off + 256;
}

void size_vectors(ctm_cell* c) {
  const size_t ns = c->ns, L = c->Lmax;
  c->A.assign(ns, nullptr);
  c->a.assign(ns, nullptr);
  c->ap.assign(ns * 4, nullptr);
  c->apr.assign(ns * 4, nullptr);
  c->env.assign(ns, SiteEnv{});
  c->spare.assign(L * 3, nullptr);
  c->X0.assign(4 * ns, nullptr);
  c->Y0.assign(4 * ns, nullptr);
  c->X.assign(4 * ns, nullptr);
  c->Y.assign(4 * ns, nullptr);
  c->Q.assign(L * 4, nullptr);
  c->Wst.assign(L * 4, nullptr);
  c->CT.assign(L * 4, nullptr);
  c->B.assign(L * 6, nullptr);
  for (auto* v : {&c->rho, &c->u, &c->v, &c->vs, &c->s, &c->sg, &c->vsc, &c->usc, &c->Pl, &c->Prt,
                  &c->Z1, &c->Z2})
    v->assign(L, nullptr);
  c->F.assign(9, nullptr);
  c->cpad.assign(ns * 4, nullptr);
  c->csv.assign(ns * 4, nullptr);
}

void set_cell_dims(ctm_cell* c, const ctm_cell_config* cfg) {
  c->cfg = *cfg;
  c->Lx = cfg->Lx;
  c->Ly = cfg->Ly;
  c->ns = cfg->Lx * cfg->Ly;
  c->Lmax = std::max(cfg->Lx, cfg->Ly);
  c->Dl = cfg->d > 0 ? cfg->D * cfg->D : cfg->D;
  c->chi = cfg->chi;
  c->Nf = c->chi * c->Dl;
  c->k = std::min(c->chi + cfg->p, c->Nf);
}

size_t env_doubles(const ctm_cell* c) {
  const size_t chi = c->chi, Dl = c->Dl;
  return (size_t)c->ns * (4 * chi * chi + 4 * chi * Dl * chi);
}

}  // namespace

extern "C" {

const char* ctm_cell_last_error(const ctm_cell* cell) {
  return cell ? cell->err.c_str() : thread_error().c_str();
}

ctm_status ctm_cell_workspace_bytes(const ctm_cell_config* cfg, size_t* bytes) {
  const int r = validate_cell(cfg);
  if (r) return (ctm_status)r;
  if (!bytes) return (ctm_status)cfail(nullptr, CTM_E_ARG, "null bytes");
  ctm_cell tmp;
  set_cell_dims(&tmp, cfg);
  size_vectors(&tmp);
  *bytes = carve_cell(&tmp, nullptr);
  return CTM_OK;
}

ctm_status ctm_cell_create(ctm_cell** out, const ctm_cell_config* cfg, const double* sites_dev,
                           const double* boundary_dev) {
  if (!out || !sites_dev) return (ctm_status)cfail(nullptr, CTM_E_ARG, "null argument");
  *out = nullptr;
  int r = validate_cell(cfg);
  if (r) return (ctm_status)r;
  ctm_cell* c = new ctm_cell();
  set_cell_dims(c, cfg);
  size_vectors(c);
  auto bail = [&](int code) {
    if (c->mem) (void)hipFree(c->mem);
    if (c->st) (void)hipStreamDestroy(c->st);
    if (c->rb) rocblas_destroy_handle(c->rb);
    delete c;
    return (ctm_status)code;
  };
  const size_t bytes = carve_cell(c, nullptr);
  if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess)
    return bail(cfail(nullptr, CTM_E_DEVICE, "hipStreamCreate failed"));
  if (hipMalloc((void**)&c->mem, bytes) != hipSuccess)
    return bail(cfail(nullptr, CTM_E_NOMEM, "hipMalloc of the cell workspace failed"));
  carve_cell(c, c->mem);
  const int Dl = c->Dl;
  const long Dl4 = (long)Dl * Dl * Dl * Dl;
  const long site_n = cfg->d > 0 ? (long)cfg->d * cfg->D * cfg->D * cfg->D * cfg->D : Dl4;
  for (int s = 0; s < c->ns && !r; ++s) {
    if (cfg->d > 0) {
      if (hipMemcpyAsync(c->A[s], sites_dev + s * site_n, site_n * 8, hipMemcpyDeviceToDevice,
                         c->st) != hipSuccess)
        return bail(cfail(nullptr, CTM_E_DEVICE, "copy of a site tensor failed"));
      r = elem_double_layer(c->A[s], nullptr, c->a[s], cfg->d, cfg->D, c->st);
    } else if (hipMemcpyAsync(c->a[s], sites_dev + s * site_n, site_n * 8,
                              hipMemcpyDeviceToDevice, c->st) != hipSuccess) {
      return bail(cfail(nullptr, CTM_E_DEVICE, "copy of a site tensor failed"));
    }
    // corner permutations of a (a[u,l,d,r]): corner 0: (l,u),(d,r); 1: (u,r),(l,d);
    // 2: (r,d),(u,l); 3: (d,l),(r,u); apr: the two leading legs swapped
    const long su = (long)Dl * Dl * Dl, sl = (long)Dl * Dl, sd = Dl, sr = 1;
    const long perm[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
    for (int i = 0; i < 4 && !r; ++i) {
      r = elem_permute4(c->a[s], c->ap[s * 4 + i], DT::F64, Dl, perm[i][0], perm[i][1], perm[i][2],
                        perm[i][3], c->st);
      if (!r)
        r = elem_permute4(c->a[s], c->apr[s * 4 + i], DT::F64, Dl, perm[i][1], perm[i][0],
                          perm[i][2], perm[i][3], c->st);
    }
  }
  if (r) return bail(cfail(nullptr, r == 1 ? CTM_E_ARG : r, thread_error()));
  // boundary vectors (default: the delta vector of each ket-bra pair, or the
  // uniform one of a classical network)
  double* bvec = c->bvec;
  {
    std::vector<double> hb((size_t)c->ns * 4 * Dl, 0.0);
    if (boundary_dev) {
      if (hipMemcpyAsync(bvec, boundary_dev, hb.size() * 8, hipMemcpyDeviceToDevice, c->st) !=
          hipSuccess)
        return bail(cfail(nullptr, CTM_E_DEVICE, "copy of the boundary vectors failed"));
    } else {
      for (size_t v = 0; v < (size_t)c->ns * 4; ++v)
        for (int i = 0; i < Dl; ++i)
          hb[v * Dl + i] = cfg->d > 0 ? ((i / cfg->D == i % cfg->D) ? 1.0 : 0.0) : 1.0;
      if (hipMemcpy(bvec, hb.data(), hb.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bail(cfail(nullptr, CTM_E_DEVICE, "copy of the boundary vectors failed"));
    }
  }
  if (hipMemsetAsync(c->bad, 0, sizeof(int), c->st) != hipSuccess ||
      hipMemsetAsync(c->spec[0], 0, (size_t)4 * c->ns * c->chi * 8, c->st) != hipSuccess ||
      hipMemsetAsync(c->spec[1], 0, (size_t)4 * c->ns * c->chi * 8, c->st) != hipSuccess)
    return bail(cfail(nullptr, CTM_E_DEVICE, "memset failed"));
  r = init_env(c, bvec);
  if (!r) r = spectra(c, nullptr);
  if (r) return bail(cfail(nullptr, r, c->err));
  *out = c;
  return CTM_OK;
}

void ctm_cell_destroy(ctm_cell* cell) {
  if (!cell) return;
  (void)hipStreamSynchronize(cell->st);
  if (cell->rb) rocblas_destroy_handle(cell->rb);
  if (cell->mem) (void)hipFree(cell->mem);
  if (cell->st) (void)hipStreamDestroy(cell->st);
  delete cell;
}

ctm_status ctm_cell_set_blocks(ctm_cell* cell, const double* X_dev, const double* Yt_dev) {
  if (!cell || !X_dev || !Yt_dev) return (ctm_status)cfail(cell, CTM_E_ARG, "null argument");
  const size_t nk = (size_t)cell->Nf * cell->k;
  for (int i = 0; i < 4 * cell->ns; ++i) {
    if (hipMemcpyAsync(cell->X0[i], X_dev + i * nk, nk * 8, hipMemcpyDeviceToDevice, cell->st) !=
            hipSuccess ||
        hipMemcpyAsync(cell->Y0[i], Yt_dev + i * nk, nk * 8, hipMemcpyDeviceToDevice, cell->st) !=
            hipSuccess)
      return (ctm_status)cfail(cell, CTM_E_DEVICE, "copy of the start blocks failed");
  }
  if (hipStreamSynchronize(cell->st) != hipSuccess)
    return (ctm_status)cfail(cell, CTM_E_DEVICE, "synchronisation failed");
  cell->blocks_set = true;
  cell->last_mode = -1;
  return CTM_OK;
}

ctm_status ctm_cell_iterate(ctm_cell* cell, int mode, double* delta) {
  if (!cell) return (ctm_status)cfail(nullptr, CTM_E_ARG, "null cell");
  if (mode != CTM_CELL_RSVD && mode != CTM_CELL_SI && mode != CTM_CELL_SVD)
    return (ctm_status)cfail(cell, CTM_E_ARG, "mode must be CTM_CELL_RSVD, _SI or _SVD");
  const bool si_from_state = mode == CTM_CELL_SI && cell->cur_set && cell->last_mode == CTM_CELL_SI;
  if (mode != CTM_CELL_SVD && !cell->blocks_set && !si_from_state)
    return (ctm_status)cfail(cell, CTM_E_STATE, "set the start blocks (or a state) first");
  cell->err.clear();
  const int r = iteration(cell, mode, delta);
  return (ctm_status)r;
}

ctm_status ctm_cell_run(ctm_cell* cell, int warmup, int warm_mode, double tol, int max_iter,
                        int* iters, double* deltas, int* kinds) {
  if (!cell || !iters) return (ctm_status)cfail(cell, CTM_E_ARG, "null argument");
  if (warm_mode != CTM_CELL_RSVD && warm_mode != CTM_CELL_SVD)
    return (ctm_status)cfail(cell, CTM_E_ARG, "warm_mode must be CTM_CELL_RSVD or CTM_CELL_SVD");
  if (!cell->blocks_set) return (ctm_status)cfail(cell, CTM_E_STATE, "set the start blocks first");
  cell->err.clear();
  int n = 0;
  double delta = 0.0;
  bool conv = false;
  while (n < max_iter) {
    bool full = true;
    for (const auto& e : cell->env) full = full && e.Cd[0][0] == cell->chi;
    const bool warm = n < warmup || !full;
    const int mode = warm ? warm_mode : CTM_CELL_SI;
    const int r = iteration(cell, mode, &delta);
    if (r) {
      *iters = n;
      return (ctm_status)r;
    }
    if (deltas) deltas[n] = delta;
    if (kinds) kinds[n] = mode;
    ++n;
    if (!warm && delta < tol) {
      conv = true;
      break;
    }
  }
  *iters = n;
  return conv ? CTM_OK : CTM_E_NOT_CONVERGED;
}

ctm_status ctm_cell_env_size(const ctm_cell* cell, size_t* n) {
  if (!cell || !n) return (ctm_status)cfail(nullptr, CTM_E_ARG, "null argument");
  *n = env_doubles(cell);
  return CTM_OK;
}

ctm_status ctm_cell_get_env(ctm_cell* cell, double* host, size_t n, int* dims) {
  if (!cell || !host || !dims) return (ctm_status)cfail(cell, CTM_E_ARG, "null argument");
  if (n != env_doubles(cell)) return (ctm_status)cfail(cell, CTM_E_SHAPE, "wrong environment size");
  const size_t chi = cell->chi, Dl = cell->Dl;
  double* p = host;
  std::fill(host, host + n, 0.0);
  for (int s = 0; s < cell->ns; ++s) {
    const SiteEnv& e = cell->env[s];
    for (int i = 0; i < 4; ++i) {
      if (hipMemcpyAsync(p, e.C[i], (size_t)e.Cd[i][0] * e.Cd[i][1] * 8, hipMemcpyDeviceToHost,
                         cell->st) != hipSuccess)
        return (ctm_status)cfail(cell, CTM_E_DEVICE, "copy of the environment failed");
      p += chi * chi;
      dims[s * 16 + 2 * i] = e.Cd[i][0];
      dims[s * 16 + 2 * i + 1] = e.Cd[i][1];
    }
    for (int i = 0; i < 4; ++i) {
      if (hipMemcpyAsync(p, e.T[i], (size_t)e.Td[i][0] * Dl * e.Td[i][1] * 8,
                         hipMemcpyDeviceToHost, cell->st) != hipSuccess)
        return (ctm_status)cfail(cell, CTM_E_DEVICE, "copy of the environment failed");
      p += chi * Dl * chi;
      dims[s * 16 + 8 + 2 * i] = e.Td[i][0];
      dims[s * 16 + 8 + 2 * i + 1] = e.Td[i][1];
    }
  }
  if (hipStreamSynchronize(cell->st) != hipSuccess)
    return (ctm_status)cfail(cell, CTM_E_DEVICE, "synchronisation failed");
  return CTM_OK;
}

ctm_status ctm_cell_set_env(ctm_cell* cell, const double* host, size_t n, const int* dims) {
  if (!cell || !host || !dims) return (ctm_status)cfail(cell, CTM_E_ARG, "null argument");
  if (n != env_doubles(cell)) return (ctm_status)cfail(cell, CTM_E_SHAPE, "wrong environment size");
  const int chi = cell->chi, Dl = cell->Dl;
  for (int i = 0; i < cell->ns * 16; ++i)
    if (dims[i] < 1 || dims[i] > chi)
      return (ctm_status)cfail(cell, CTM_E_SHAPE, "environment dimensions must be in 1..chi");
  const double* p = host;
  for (int s = 0; s < cell->ns; ++s) {
    SiteEnv& e = cell->env[s];
    for (int i = 0; i < 4; ++i) {
      e.Cd[i][0] = dims[s * 16 + 2 * i];
      e.Cd[i][1] = dims[s * 16 + 2 * i + 1];
      if (hipMemcpyAsync(e.C[i], p, (size_t)e.Cd[i][0] * e.Cd[i][1] * 8, hipMemcpyHostToDevice,
                         cell->st) != hipSuccess)
        return (ctm_status)cfail(cell, CTM_E_DEVICE, "copy of the environment failed");
      p += (size_t)chi * chi;
    }
    for (int i = 0; i < 4; ++i) {
      e.Td[i][0] = dims[s * 16 + 8 + 2 * i];
      e.Td[i][1] = dims[s * 16 + 8 + 2 * i + 1];
      if (hipMemcpyAsync(e.T[i], p, (size_t)e.Td[i][0] * Dl * e.Td[i][1] * 8,
                         hipMemcpyHostToDevice, cell->st) != hipSuccess)
        return (ctm_status)cfail(cell, CTM_E_DEVICE, "copy of the environment failed");
      p += (size_t)chi * Dl * chi;
    }
  }
  cell->last_mode = -1;
  const int r = spectra(cell, nullptr);
  return (ctm_status)r;
}

ctm_status ctm_cell_get_blocks(ctm_cell* cell, double* X_host, double* Yt_host) {
  if (!cell || !X_host || !Yt_host) return (ctm_status)cfail(cell, CTM_E_ARG, "null argument");
  const size_t nk = (size_t)cell->Nf * cell->k;
  for (int i = 0; i < 4 * cell->ns; ++i) {
    if (hipMemcpyAsync(X_host + i * nk, cell->X[i], nk * 8, hipMemcpyDeviceToHost, cell->st) !=
            hipSuccess ||
        hipMemcpyAsync(Yt_host + i * nk, cell->Y[i], nk * 8, hipMemcpyDeviceToHost, cell->st) !=
            hipSuccess)
      return (ctm_status)cfail(cell, CTM_E_DEVICE, "copy of the blocks failed");
  }
  if (hipStreamSynchronize(cell->st) != hipSuccess)
    return (ctm_status)cfail(cell, CTM_E_DEVICE, "synchronisation failed");
  return CTM_OK;
}

}  // extern "C"
