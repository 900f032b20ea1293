// Adjoint of the unit-cell move and the energy of the cell (the
// differentiation of the Differentiable fixed point passage, eq. implicit,
// through unrolled moves; the larger unit cell of the End Matter), and the
// state-vector entry points of include/ctm.h that it works on.
//
// Both are written against the reverse-mode tape (tape.h): the move of an
// environment of full dimension (every cut an SI cut with the state's own
// blocks, recycled) is recomputed from the caller's input state with every
// intermediate kept, the cotangents of the output state are seeded, and the
// tape's backward pass gives the cotangents of the input state and of the
// site tensors.  The forward contractions are those of the cell move
// (cell.hip) with the same descriptors; the energy contracts the two-site
// networks of every site's horizontal, vertical and diagonal bond with the
// open double layers of the two sites (iPEPS section, observables).
//
// State vector (device, float64): per site (index y*Lx + x) C1..C4
// (chi x chi each) then T1..T4 (chi x Dl x chi each); then X and then Y^T of
// every cut ([4 directions][Lx*Ly cuts][chi*Dl][k], the layout of
// ctm_cell_set_blocks).

#include "cell.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "elem.h"

using namespace sictm;

namespace {

int afail(ctm_cell* c, int code, const std::string& msg) {
  c->err = msg;
  set_thread_error(msg);
  return code;
}

#define ATRY(expr)                                                      \
  do {                                                                  \
    const int _r = (expr);                                              \
    if (_r != 0) {                                                      \
      if (c->err.empty()) c->err = thread_error();                      \
      return _r == 1 ? (int)CTM_E_ARG : _r;                             \
    }                                                                   \
  } while (0)

// ---------------------------------------------------------------------------
// state-vector layout
// ---------------------------------------------------------------------------
struct Layout {
  long chi, Dl, N, k, ns;
  long site_n() const { return 4 * chi * chi + 4 * chi * Dl * chi; }
  long C(int s, int i) const { return s * site_n() + i * chi * chi; }
  long T(int s, int i) const { return s * site_n() + 4 * chi * chi + i * chi * Dl * chi; }
  long X(int id) const { return ns * site_n() + (long)id * N * k; }
  long Y(int id) const { return ns * site_n() + 4 * ns * N * k + (long)id * N * k; }
  long total() const { return ns * site_n() + 8 * ns * N * k; }
};

Layout layout(const ctm_cell* c) { return Layout{c->chi, c->Dl, c->Nf, c->k, c->ns}; }

// ---------------------------------------------------------------------------
// two-operand contraction on the tape (labels: one character per leg; every
// output label belongs to exactly one operand, the others are summed)
// ---------------------------------------------------------------------------
struct TT {
  const double* p;
  std::vector<int> sh;
  std::string lab;
};

int permute_to(Tape& t, const TT& x, const std::string& order, const double** out) {
  if (order == x.lab) {
    *out = x.p;
    return 0;
  }
  const int nd = (int)order.size();
  std::vector<long> rs(x.lab.size());
  long st = 1;
  for (int j = (int)x.lab.size() - 1; j >= 0; --j) {
    rs[j] = st;
    st *= x.sh[j];
  }
  std::vector<int> dims(nd);
  std::vector<long> strides(nd);
  for (int j = 0; j < nd; ++j) {
    const size_t at = x.lab.find(order[j]);
    dims[j] = x.sh[at];
    strides[j] = rs[at];
  }
  double* d = t.alloc(st);
  if (!d) return CTM_E_NOMEM;
  const int rc = t.permute(x.p, d, nd, dims.data(), strides.data());
  *out = d;
  return rc;
}

int einsum2(Tape& t, const TT& A, const TT& B, const std::string& out, TT* res) {
  std::string freeA, freeB, con;
  auto dim = [&](char l) {
    size_t i = A.lab.find(l);
    if (i != std::string::npos) return A.sh[i];
    return B.sh[B.lab.find(l)];
  };
  for (char l : out) {
    const bool inA = A.lab.find(l) != std::string::npos, inB = B.lab.find(l) != std::string::npos;
    if (inA == inB) return CTM_E_ARG;
    (inA ? freeA : freeB) += l;
  }
  for (char l : A.lab)
    if (out.find(l) == std::string::npos) {
      if (B.lab.find(l) == std::string::npos) return CTM_E_ARG;
      if (A.sh[A.lab.find(l)] != B.sh[B.lab.find(l)]) return CTM_E_SHAPE;
      con += l;
    }
  long M = 1, N = 1, K = 1;
  for (char l : freeA) M *= dim(l);
  for (char l : freeB) N *= dim(l);
  for (char l : con) K *= dim(l);
  const double *pa = nullptr, *pb = nullptr;
  int rc = permute_to(t, A, freeA + con, &pa);
  if (!rc) rc = permute_to(t, B, con + freeB, &pb);
  if (rc) return rc;
  double* r = t.alloc(M * N);
  if (!r) return CTM_E_NOMEM;
  GemmBatch g = gemm_of((int)M, (int)N, (int)K, K, N, N);
  add(g, pa, pb, r);
  rc = t.gemm(g);
  if (rc) return rc;
  // res may alias A or B: the result is built completely before it is stored
  TT mid{r, {}, freeA + freeB};
  for (char l : mid.lab) mid.sh.push_back(dim(l));
  TT fin{nullptr, {}, out};
  for (char l : out) fin.sh.push_back(dim(l));
  if (mid.lab == out) {
    fin.p = r;
  } else {
    rc = permute_to(t, mid, out, &fin.p);
    if (rc) return rc;
  }
  *res = fin;
  return 0;
}

// ---------------------------------------------------------------------------
// network tensors on the tape
// ---------------------------------------------------------------------------
// a[(uU),(lL),(dD),(rR)] = sum_s A[s,u,l,d,r] A[s,U,L,D,R] (iPEPS section), or
// the given network tensor when d == 0.
int taped_network(ctm_cell* c, Tape& t, std::vector<const double*>& a) {
  const int d = c->cfg.d, D = c->cfg.D, Dl = c->Dl;
  const long D4 = (long)D * D * D * D;
  a.assign(c->ns, nullptr);
  for (int s = 0; s < c->ns; ++s) {
    if (d == 0) {
      t.external(c->a[s], (long)Dl * Dl * Dl * Dl, false);
      a[s] = c->a[s];
      continue;
    }
    t.external(c->A[s], (long)d * D4, false);
    double* kb = t.alloc(D4 * D4);
    double* out = t.alloc(D4 * D4);
    if (!kb || !out) return CTM_E_NOMEM;
    GemmBatch g = gemm_of((int)D4, (int)D4, d, D4, D4, D4);
    add(g, c->A[s], c->A[s], kb, 1);
    ATRY(t.gemm(g));
    // kb[(i,j,k,l),(I,J,K,L)] -> a[i,I,j,J,k,K,l,L]
    const long p[8] = {D4 * D * D * D, D * D * D, D4 * D * D, D * D, D4 * D, D, D4, 1};
    const int dims[8] = {D, D, D, D, D, D, D, D};
    ATRY(t.permute(kb, out, 8, dims, p));
    a[s] = out;
  }
  return 0;
}

// ao[s,t,(uU),(lL),(dD),(rR)] = A[s,u,l,d,r] A[t,U,L,D,R] (ket s, bra t).
int taped_open_layer(ctm_cell* c, Tape& t, int s, TT* ao) {
  const int d = c->cfg.d, D = c->cfg.D, Dl = c->Dl;
  const long D4 = (long)D * D * D * D, n1 = d * D4;
  double* outer = t.alloc(n1 * n1);
  double* out = t.alloc(n1 * n1);
  if (!outer || !out) return CTM_E_NOMEM;
  GemmBatch g = gemm_of((int)n1, (int)n1, 1, 1, n1, n1);
  add(g, c->A[s], c->A[s], outer);
  ATRY(t.gemm(g));
  // outer[(s,i,j,k,l),(t,I,J,K,L)] -> [s,t,i,I,j,J,k,K,l,L]
  const long D3 = (long)D * D * D;
  const long p[10] = {D4 * n1, D4, D3 * n1, D3, D * D * n1, D * D, D * n1, D, n1, 1};
  const int dims[10] = {d, d, D, D, D, D, D, D, D, D};
  ATRY(t.permute(outer, out, 10, dims, p));
  *ao = TT{out, {d, d, Dl, Dl, Dl, Dl}, ""};
  return 0;
}

// ---------------------------------------------------------------------------
// the move on the tape (every cut an SI cut)
// ---------------------------------------------------------------------------
struct TEnv {
  const double* C[4];
  const double* T[4];
};

int taped_move(ctm_cell* c, Tape& t, const std::vector<const double*>& a, std::vector<TEnv>& env,
               std::vector<const double*>& X, std::vector<const double*>& Y) {
  const int Dl = c->Dl, chi = c->chi, N = c->Nf, k = c->k;
  const long D2 = (long)Dl * Dl, Dl4 = D2 * D2, NN = (long)N * N, Nk = (long)N * k;
  const long envT = (long)chi * Dl * chi;
  // corner and edge permutations of every site's network tensor
  std::vector<std::array<const double*, 4>> ap(c->ns), apr(c->ns);
  {
    const long su = (long)Dl * Dl * Dl, sl = D2, sd = Dl, sr = 1;
    const long perm[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
    const int dims[4] = {Dl, Dl, Dl, Dl};
    for (int s = 0; s < c->ns; ++s)
      for (int i = 0; i < 4; ++i) {
        double* p1 = t.alloc(Dl4);
        double* p2 = t.alloc(Dl4);
        if (!p1 || !p2) return CTM_E_NOMEM;
        ATRY(t.permute(a[s], p1, 4, dims, perm[i]));
        const long pr[4] = {perm[i][1], perm[i][0], perm[i][2], perm[i][3]};
        ATRY(t.permute(a[s], p2, 4, dims, pr));
        ap[s][i] = p1;
        apr[s][i] = p2;
      }
  }
  for (int d = 0; d < 4; ++d) {
    const int W = width(c, d), H = height(c, d);
    for (int xt = 0; xt < W; ++xt) {
      std::vector<std::array<int, 4>> site(H);
      std::vector<std::array<const double*, 4>> Q(H);
      // enlarged corners, batched by 8
      {
        struct Job {
          int y, i;
        };
        std::vector<Job> jobs;
        for (int y = 0; y < H; ++y) {
          site[y] = {site_of(c, d, xt, y), site_of(c, d, xt + 1, y), site_of(c, d, xt + 1, y + 1),
                     site_of(c, d, xt, y + 1)};
          for (int i = 0; i < 4; ++i) jobs.push_back({y, i});
        }
        for (size_t b0 = 0; b0 < jobs.size(); b0 += 8) {
          GemmBatch g1 = gemm_of(chi, Dl * chi, chi, chi, (long)Dl * chi, 0);
          g1.cdiv_m = 1 << 30; g1.cs_m1 = 0; g1.cs_m0 = (long)Dl * chi;
          g1.cdiv_n = chi; g1.cs_n1 = 1; g1.cs_n0 = Dl;
          GemmBatch g2 = gemm_of(chi * Dl, Dl * chi, chi, chi, (long)Dl * chi, 0);
          g2.cdiv_m = Dl; g2.cs_m1 = (long)chi * D2; g2.cs_m0 = Dl;
          g2.cdiv_n = Dl; g2.cs_n1 = D2; g2.cs_n0 = 1;
          GemmBatch g3 = gemm_of(chi * chi, (int)D2, (int)D2, D2, D2, 0);
          g3.cdiv_m = chi; g3.cs_m1 = (long)Dl * chi * Dl; g3.cs_m0 = Dl;
          g3.cdiv_n = Dl; g3.cs_n1 = (long)chi * Dl; g3.cs_n0 = 1;
          for (size_t j = b0; j < std::min(jobs.size(), b0 + 8); ++j) {
            const int y = jobs[j].y, i = jobs[j].i, ci = (i + d) & 3, s = site[y][i];
            double* ct = t.alloc(envT);
            double* stem = t.alloc(NN);
            double* q = t.alloc(NN);
            if (!ct || !stem || !q) return CTM_E_NOMEM;
            add(g1, env[s].C[ci], env[s].T[ci], ct);
            add(g2, env[s].T[(ci + 3) & 3], ct, stem);
            add(g3, stem, ap[s][ci], q);
            Q[y][i] = q;
          }
          ATRY(t.gemm(g1));
          ATRY(t.gemm(g2));
          ATRY(t.gemm(g3));
        }
      }
      // SI projectors, up to 4 cuts per group
      std::vector<const double*> Pl(H), Prt(H);
      for (int y0 = 0; y0 < H; y0 += kCutsPerLaunch) {
        const int n = std::min(kCutsPerLaunch, H - y0);
        std::vector<const double*> xc(n), yc(n);
        std::vector<int> ids(n);
        for (int i = 0; i < n; ++i) {
          ids[i] = d * c->ns + (y0 + i) * W + xt;
          xc[i] = X[ids[i]];
          yc[i] = Y[ids[i]];
        }
        auto apply = [&](int qx, int tx, int qy, int tyy) -> int {
          GemmBatch g = gemm_of(N, k, N, N, k, k);
          std::vector<const double*> nx(n), ny(n);
          for (int i = 0; i < n; ++i) {
            double* o = t.alloc(Nk);
            if (!o) return CTM_E_NOMEM;
            add(g, Q[y0 + i][qx], xc[i], o, tx);
            nx[i] = o;
          }
          for (int i = 0; i < n; ++i) {
            double* o = t.alloc(Nk);
            if (!o) return CTM_E_NOMEM;
            add(g, Q[y0 + i][qy], yc[i], o, tyy);
            ny[i] = o;
          }
          ATRY(t.gemm(g));
          xc = nx;
          yc = ny;
          return 0;
        };
        auto qr_all = [&]() -> int {
          std::vector<const double*> h;
          std::vector<double*> q;
          for (int i = 0; i < n; ++i) {
            h.push_back(xc[i]);
            h.push_back(yc[i]);
          }
          for (size_t j = 0; j < h.size(); ++j) {
            double* o = t.alloc(Nk);
            if (!o) return CTM_E_NOMEM;
            q.push_back(o);
          }
          ATRY(t.qr((int)h.size(), h.data(), q.data(), N, k));
          for (int i = 0; i < n; ++i) {
            xc[i] = q[2 * i];
            yc[i] = q[2 * i + 1];
          }
          return 0;
        };
        // M W = Q3 Q4 Q1 Q2 W;  M^T W = Q2^T Q1^T Q4^T Q3^T W
        const int mq[4] = {1, 0, 3, 2}, tq[4] = {2, 3, 0, 1};
        for (int step = 0; step < c->cfg.n_si; ++step) {
          for (int half = 0; half < 2; ++half) {
            const bool x_with_M = half == 0;
            for (int a4 = 0; a4 < 4; ++a4)
              ATRY(apply(x_with_M ? mq[a4] : tq[a4], x_with_M ? 0 : 1, x_with_M ? tq[a4] : mq[a4],
                         x_with_M ? 1 : 0));
            if (c->cfg.stabilized || half == 1) ATRY(qr_all());
          }
        }
        const std::vector<const double*> xf = xc, yf = yc;
        ATRY(apply(1, 0, 2, 1));
        ATRY(apply(0, 0, 3, 1));
        const std::vector<const double*> Am = xc, Bt = yc;
        std::vector<const double*> rho(n);
        {
          GemmBatch g = gemm_of(k, k, N, k, k, k);
          for (int i = 0; i < n; ++i) {
            double* o = t.alloc((long)k * k);
            if (!o) return CTM_E_NOMEM;
            add(g, Bt[i], Am[i], o, 1);
            rho[i] = o;
          }
          ATRY(t.gemm(g));
        }
        std::vector<double*> us(n), vs(n), vsc(n), usc(n);
        for (int i = 0; i < n; ++i) {
          us[i] = t.alloc((long)k * k);
          vs[i] = t.alloc((long)k * k);
          vsc[i] = t.alloc((long)k * chi);
          usc[i] = t.alloc((long)k * chi);
          if (!us[i] || !vs[i] || !vsc[i] || !usc[i]) return CTM_E_NOMEM;
        }
        ATRY(t.svdproj(n, rho.data(), yf.data(), N, k, chi, c->cfg.pinv_rtol, us.data(), vs.data(),
                       vsc.data(), usc.data()));
        {
          GemmBatch g = gemm_of(N, chi, k, k, chi, chi);
          for (int i = 0; i < n; ++i) {
            double* pl = t.alloc((long)N * chi);
            double* pr = t.alloc((long)N * chi);
            if (!pl || !pr) return CTM_E_NOMEM;
            add(g, Am[i], vsc[i], pl);
            add(g, Bt[i], usc[i], pr);
            Pl[y0 + i] = pl;
            Prt[y0 + i] = pr;
          }
          ATRY(t.gemm(g));
        }
        {
          GemmBatch g = gemm_of(N, k, k, k, k, k);
          for (int i = 0; i < n; ++i) {
            double* xn = t.alloc(Nk);
            double* yn = t.alloc(Nk);
            if (!xn || !yn) return CTM_E_NOMEM;
            add(g, xf[i], vs[i], xn);
            add(g, yf[i], us[i], yn);
            X[ids[i]] = xn;
            Y[ids[i]] = yn;
          }
          ATRY(t.gemm(g));
        }
      }
      // the left environment of column xt moves to column xt + 1
      const int sC1 = d & 3, sT1 = d & 3, sT3 = (2 + d) & 3, sC4 = (3 + d) & 3, sT4 = (3 + d) & 3;
      std::vector<std::array<const double*, 3>> fresh(H);
      for (int y = 0; y < H; ++y) {
        const int yu = imod(y - 1, H);
        const TEnv& e = env[site[y][0]];
        double* t1 = t.alloc(envT);
        double* nC1 = t.alloc((long)chi * chi);
        double* t2 = t.alloc(envT);
        double* nC4 = t.alloc((long)chi * chi);
        double* z1 = t.alloc((long)chi * chi * D2);
        double* z2 = t.alloc((long)chi * chi * D2);
        double* nT4 = t.alloc(envT);
        if (!t1 || !nC1 || !t2 || !nC4 || !z1 || !z2 || !nT4) return CTM_E_NOMEM;
        GemmBatch g = gemm_of(chi, Dl * chi, chi, chi, (long)Dl * chi, (long)Dl * chi);
        add(g, e.C[sC1], e.T[sT1], t1);
        ATRY(t.gemm(g));
        GemmBatch g2 = gemm_of(chi, chi, chi * Dl, chi, chi, chi);
        add(g2, Prt[yu], t1, nC1, 1);
        ATRY(t.gemm(g2));
        GemmBatch g3 = gemm_of(chi * Dl, chi, chi, chi, chi, 0);
        g3.cdiv_m = Dl; g3.cs_m1 = (long)chi * Dl; g3.cs_m0 = 1;
        g3.cdiv_n = 1 << 30; g3.cs_n1 = 0; g3.cs_n0 = Dl;
        add(g3, e.T[sT3], e.C[sC4], t2);
        ATRY(t.gemm(g3));
        GemmBatch g4 = gemm_of(chi, chi, chi * Dl, (long)chi * Dl, chi, chi);
        add(g4, t2, Pl[y], nC4);
        ATRY(t.gemm(g4));
        GemmBatch g5 = gemm_of(chi * Dl, chi, chi, chi, (long)Dl * chi, 0);
        g5.cdiv_m = Dl; g5.cs_m1 = (long)chi * D2; g5.cs_m0 = 1;
        g5.cdiv_n = 1 << 30; g5.cs_n1 = 0; g5.cs_n0 = D2;
        g5.nbatch = Dl; g5.a_bs = 0; g5.b_bs = chi; g5.c_bs = Dl;
        add(g5, e.T[sT4], Pl[yu], z1);
        ATRY(t.gemm(g5));
        GemmBatch g6 = gemm_of(chi * chi, (int)D2, (int)D2, D2, D2, 0);
        g6.cdiv_m = chi; g6.cs_m1 = D2 * chi; g6.cs_m0 = 1;
        g6.cdiv_n = Dl; g6.cs_n1 = (long)Dl * chi; g6.cs_n0 = chi;
        add(g6, z1, apr[site[y][0]][(sT4 + 1) & 3], z2);
        ATRY(t.gemm(g6));
        GemmBatch g7 = gemm_of(Dl * chi, chi, chi * Dl, (long)Dl * chi, chi, 0);
        g7.cdiv_m = 1 << 30; g7.cs_m1 = 0; g7.cs_m0 = 1;
        g7.cdiv_n = 1 << 30; g7.cs_n1 = 0; g7.cs_n0 = (long)Dl * chi;
        add(g7, z2, Prt[y], nT4, 1);
        ATRY(t.gemm(g7));
        const double* xs[3] = {nC1, nT4, nC4};
        double* ys[3] = {t.alloc((long)chi * chi), t.alloc(envT), t.alloc((long)chi * chi)};
        if (!ys[0] || !ys[1] || !ys[2]) return CTM_E_NOMEM;
        const long ns3[3] = {(long)chi * chi, envT, (long)chi * chi};
        ATRY(t.normalize(3, xs, ys, ns3));
        fresh[y] = {ys[0], ys[1], ys[2]};
      }
      for (int y = 0; y < H; ++y) {
        TEnv& tg = env[site_of(c, d, xt + 1, y)];
        tg.C[sC1] = fresh[y][0];
        tg.T[sT4] = fresh[y][1];
        tg.C[sC4] = fresh[y][2];
      }
    }
  }
  return 0;
}

// Registers the input state and returns the per-site tensors and blocks it holds.
void bind_state(ctm_cell* c, Tape& t, const double* state, bool constant, std::vector<TEnv>& env,
                std::vector<const double*>& X, std::vector<const double*>& Y) {
  const Layout L = layout(c);
  t.external(state, L.total(), constant);
  env.assign(c->ns, TEnv{});
  for (int s = 0; s < c->ns; ++s)
    for (int i = 0; i < 4; ++i) {
      env[s].C[i] = state + L.C(s, i);
      env[s].T[i] = state + L.T(s, i);
    }
  X.assign(4 * c->ns, nullptr);
  Y.assign(4 * c->ns, nullptr);
  for (int id = 0; id < 4 * c->ns; ++id) {
    X[id] = state + L.X(id);
    Y[id] = state + L.Y(id);
  }
}

// ---------------------------------------------------------------------------
// the energy of the cell on the tape
// ---------------------------------------------------------------------------
TT ten(const double* p, std::vector<int> sh, const char* lab) { return TT{p, std::move(sh), lab}; }

int pair_h(Tape& t, const TEnv& L, const TEnv& R, const TT& x1, const TT& x2, int chi, int Dl,
           TT* E) {
  const std::vector<int> cc = {chi, chi}, tt = {chi, Dl, chi};
  TT t1, left, y1, y2, y3, t2, right, w1, w2, w3;
  int rc = einsum2(t, ten(L.C[0], cc, "ab"), ten(L.T[3], tt, "kla"), "bkl", &t1);
  if (!rc) rc = einsum2(t, t1, ten(L.C[3], cc, "jk"), "blj", &left);
  if (!rc) rc = einsum2(t, left, ten(L.T[0], tt, "bug"), "gulj", &y1);
  if (!rc) rc = einsum2(t, y1, TT{x1.p, x1.sh, "STuldm"}, "STgdmj", &y2);
  if (!rc) rc = einsum2(t, y2, ten(L.T[2], tt, "idj"), "STgmi", &y3);
  if (!rc) rc = einsum2(t, ten(R.C[1], cc, "hc"), ten(R.T[1], tt, "cwe"), "hwe", &t2);
  if (!rc) rc = einsum2(t, t2, ten(R.C[2], cc, "ef"), "hwf", &right);
  if (!rc) rc = einsum2(t, ten(R.T[0], tt, "gvh"), right, "gvwf", &w1);
  if (!rc) rc = einsum2(t, w1, TT{x2.p, x2.sh, "EFvmyw"}, "EFgmyf", &w2);
  if (!rc) rc = einsum2(t, w2, ten(R.T[2], tt, "fyi"), "EFgmi", &w3);
  if (!rc) rc = einsum2(t, y3, w3, "STEF", E);
  return rc;
}

int pair_v(Tape& t, const TEnv& U, const TEnv& B, const TT& x1, const TT& x2, int chi, int Dl,
           TT* E) {
  const std::vector<int> cc = {chi, chi}, tt = {chi, Dl, chi};
  TT a1, top, p1, p2, p3, b1, bot, q1, q2, q3;
  int rc = einsum2(t, ten(U.C[0], cc, "ab"), ten(U.T[0], tt, "bug"), "aug", &a1);
  if (!rc) rc = einsum2(t, a1, ten(U.C[1], cc, "gh"), "auh", &top);
  if (!rc) rc = einsum2(t, ten(U.T[3], tt, "nla"), top, "nluh", &p1);
  if (!rc) rc = einsum2(t, p1, TT{x1.p, x1.sh, "STulxr"}, "STnxrh", &p2);
  if (!rc) rc = einsum2(t, p2, ten(U.T[1], tt, "hrc"), "STnxc", &p3);
  if (!rc) rc = einsum2(t, ten(B.C[2], cc, "ij"), ten(B.T[2], tt, "jwk"), "iwk", &b1);
  if (!rc) rc = einsum2(t, b1, ten(B.C[3], cc, "km"), "iwm", &bot);
  if (!rc) rc = einsum2(t, ten(B.T[1], tt, "csi"), bot, "cswm", &q1);
  if (!rc) rc = einsum2(t, q1, TT{x2.p, x2.sh, "EFxpws"}, "EFcxpm", &q2);
  if (!rc) rc = einsum2(t, q2, ten(B.T[3], tt, "mpn"), "EFcxn", &q3);
  if (!rc) rc = einsum2(t, p3, q3, "STEF", E);
  return rc;
}

// Diagonal pair on the 2x2 plaquette: site 1 top-left with the open layer
// x1, site 3 bottom-right with x3, the closed layers a2 (top-right) and a4
// (bottom-left); E[S,T,E,F] = Ct1 Ct2 Ct3 Ct4 traced.
int pair_d(Tape& t, const TEnv& e1, const TEnv& e2, const TEnv& e3, const TEnv& e4, const TT& x1,
           const double* a2, const TT& x3, const double* a4, int chi, int Dl, TT* E) {
  const std::vector<int> cc = {chi, chi}, tt = {chi, Dl, chi}, aa = {Dl, Dl, Dl, Dl};
  TT c0, c1, c2, c3, m, P, Qm;
  int rc = einsum2(t, ten(e1.C[0], cc, "ab"), ten(e1.T[0], tt, "bug"), "aug", &m);
  if (!rc) rc = einsum2(t, ten(e1.T[3], tt, "tla"), m, "tlug", &m);
  if (!rc) rc = einsum2(t, m, TT{x1.p, x1.sh, "STuldr"}, "STtdgr", &c0);
  if (!rc) rc = einsum2(t, ten(e2.C[1], cc, "gh"), ten(e2.T[1], tt, "hre"), "gre", &m);
  if (!rc) rc = einsum2(t, ten(e2.T[0], tt, "bug"), m, "bure", &m);
  if (!rc) rc = einsum2(t, m, ten(a2, aa, "uldr"), "bled", &c1);
  if (!rc) rc = einsum2(t, ten(e3.C[2], cc, "ez"), ten(e3.T[2], tt, "zdn"), "edn", &m);
  if (!rc) rc = einsum2(t, ten(e3.T[1], tt, "hre"), m, "hrdn", &m);
  if (!rc) rc = einsum2(t, m, TT{x3.p, x3.sh, "EFuldr"}, "EFhunl", &c2);
  if (!rc) rc = einsum2(t, ten(e4.C[3], cc, "nt"), ten(e4.T[3], tt, "tla"), "nla", &m);
  if (!rc) rc = einsum2(t, ten(e4.T[2], tt, "zdn"), m, "zdla", &m);
  if (!rc) rc = einsum2(t, m, ten(a4, aa, "uldr"), "zrau", &c3);
  // rows and columns of the four corners: c0 [S,T,(t,d),(g,r)], c1 [(b,l),(e,d)],
  // c2 [E,F,(h,u),(n,l)], c3 [(z,r),(a,u)]
  if (!rc) rc = einsum2(t, TT{c0.p, c0.sh, "STabcd"}, TT{c1.p, c1.sh, "cdef"}, "STabef", &P);
  if (!rc) rc = einsum2(t, TT{c2.p, c2.sh, "EFefgh"}, TT{c3.p, c3.sh, "ghab"}, "EFefab", &Qm);
  if (!rc) rc = einsum2(t, P, Qm, "STEF", E);
  return rc;
}

// e = (1 / (Lx Ly)) sum over the sites and the bonds in `bonds` (1: h, 2: v,
// 4: d) of <op_b>; the per-(site, bond) values land in vals (device, one
// double each, in the order site-major, then h, v, d).
int taped_energy(ctm_cell* c, Tape& t, const std::vector<TEnv>& env,
                 const std::vector<const double*>& a, const double* ops, int bonds,
                 std::vector<double*>& vals) {
  const int d = c->cfg.d, chi = c->chi, Dl = c->Dl;
  const long dd = (long)d * d;
  std::vector<TT> ao(c->ns);
  for (int s = 0; s < c->ns; ++s) ATRY(taped_open_layer(c, t, s, &ao[s]));
  // weights of <op> = tr(op rho) / tr(rho) with rho[(s1 s2), (t1 t2)] = E[s1, t1, s2, t2]
  std::vector<double> w2h(dd * dd, 0.0);
  for (int A = 0; A < d; ++A)
    for (int E = 0; E < d; ++E) w2h[((A * d + A) * d + E) * d + E] = 1.0;
  const double* w2 = t.upload(w2h.data(), dd * dd);
  const double* w1[3] = {nullptr, nullptr, nullptr};
  std::vector<double> w1h[3];
  for (int b = 0; b < 3; ++b) {
    if (!(bonds & (1 << b))) continue;
    w1h[b].assign(dd * dd, 0.0);
    const double* op = ops + b * dd * dd;
    for (int A = 0; A < d; ++A)
      for (int B = 0; B < d; ++B)
        for (int E = 0; E < d; ++E)
          for (int F = 0; F < d; ++F)
            w1h[b][((A * d + B) * d + E) * d + F] = op[(B * d + F) * dd + (A * d + E)];
    w1[b] = t.upload(w1h[b].data(), dd * dd);
  }
  if (!w2) return CTM_E_NOMEM;
  vals.clear();
  for (int y = 0; y < c->Ly; ++y)
    for (int x = 0; x < c->Lx; ++x) {
      const int s = y * c->Lx + x;
      const int sr = y * c->Lx + imod(x + 1, c->Lx), sb = imod(y + 1, c->Ly) * c->Lx + x;
      const int sd = imod(y + 1, c->Ly) * c->Lx + imod(x + 1, c->Lx);
      for (int b = 0; b < 3; ++b) {
        if (!(bonds & (1 << b))) continue;
        TT E;
        int rc;
        if (b == 0)
          rc = pair_h(t, env[s], env[sr], ao[s], ao[sr], chi, Dl, &E);
        else if (b == 1)
          rc = pair_v(t, env[s], env[sb], ao[s], ao[sb], chi, Dl, &E);
        else
          rc = pair_d(t, env[s], env[sr], env[sd], env[sb], ao[s], a[sr], ao[sd], a[sb], chi, Dl, &E);
        ATRY(rc);
        double* v = t.alloc(1);
        if (!v) return CTM_E_NOMEM;
        ATRY(t.ratio(E.p, w1[b], w2, dd * dd, v));
        vals.push_back(v);
      }
    }
  return 0;
}

bool full_env(const ctm_cell* c) {
  for (const auto& e : c->env)
    for (int i = 0; i < 4; ++i)
      if (e.Cd[i][0] != c->chi || e.Cd[i][1] != c->chi || e.Td[i][0] != c->chi ||
          e.Td[i][1] != c->chi)
        return false;
  return true;
}

Tape& tape_of(ctm_cell* c) {
  if (!c->tape) c->tape.reset(new Tape(c->st));
  return *c->tape;
}

long site_doubles(const ctm_cell* c) {
  const long D4 = (long)c->cfg.D * c->cfg.D * c->cfg.D * c->cfg.D;
  return c->cfg.d > 0 ? c->cfg.d * D4 : (long)c->Dl * c->Dl * c->Dl * c->Dl;
}

}  // namespace

namespace {

int impl_get_state_device(ctm_cell* cell, double* dev, size_t n) {
  ctm_cell* c = cell;
  if (!c || !dev) return CTM_E_ARG;
  c->err.clear();
  const Layout L = layout(c);
  if (n != (size_t)L.total()) return afail(c, CTM_E_SHAPE, "wrong state size");
  if (!full_env(c)) return afail(c, CTM_E_STATE, "the environment has not reached chi");
  const bool cur = c->last_mode == CTM_CELL_SI;
  if (!cur && !c->blocks_set) return afail(c, CTM_E_STATE, "no blocks to export");
  const size_t cc = (size_t)c->chi * c->chi * 8, tt = (size_t)c->chi * c->Dl * c->chi * 8,
               nk = (size_t)c->Nf * c->k * 8;
  for (int s = 0; s < c->ns; ++s)
    for (int i = 0; i < 4; ++i) {
      CTM_HIP_TRY(hipMemcpyAsync(dev + L.C(s, i), c->env[s].C[i], cc, hipMemcpyDeviceToDevice, c->st));
      CTM_HIP_TRY(hipMemcpyAsync(dev + L.T(s, i), c->env[s].T[i], tt, hipMemcpyDeviceToDevice, c->st));
    }
  for (int id = 0; id < 4 * c->ns; ++id) {
    CTM_HIP_TRY(hipMemcpyAsync(dev + L.X(id), cur ? c->X[id] : c->X0[id], nk,
                               hipMemcpyDeviceToDevice, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(dev + L.Y(id), cur ? c->Y[id] : c->Y0[id], nk,
                               hipMemcpyDeviceToDevice, c->st));
  }
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  return CTM_OK;
}

int impl_set_state_device(ctm_cell* cell, const double* dev, size_t n) {
  ctm_cell* c = cell;
  if (!c || !dev) return CTM_E_ARG;
  c->err.clear();
  const Layout L = layout(c);
  if (n != (size_t)L.total()) return afail(c, CTM_E_SHAPE, "wrong state size");
  const size_t cc = (size_t)c->chi * c->chi * 8, tt = (size_t)c->chi * c->Dl * c->chi * 8,
               nk = (size_t)c->Nf * c->k * 8;
  for (int s = 0; s < c->ns; ++s)
    for (int i = 0; i < 4; ++i) {
      SiteEnv& e = c->env[s];
      CTM_HIP_TRY(hipMemcpyAsync(e.C[i], dev + L.C(s, i), cc, hipMemcpyDeviceToDevice, c->st));
      CTM_HIP_TRY(hipMemcpyAsync(e.T[i], dev + L.T(s, i), tt, hipMemcpyDeviceToDevice, c->st));
      e.Cd[i][0] = e.Cd[i][1] = e.Td[i][0] = e.Td[i][1] = c->chi;
    }
  for (int id = 0; id < 4 * c->ns; ++id) {
    CTM_HIP_TRY(hipMemcpyAsync(c->X[id], dev + L.X(id), nk, hipMemcpyDeviceToDevice, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(c->Y[id], dev + L.Y(id), nk, hipMemcpyDeviceToDevice, c->st));
  }
  c->cur_set = true;
  c->last_mode = CTM_CELL_SI;
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  return CTM_OK;
}

int impl_move_vjp(ctm_cell* cell, const double* state_in, const double* state_out_bar,
                             double* state_in_bar, double* site_bar, double* state_out) {
  ctm_cell* c = cell;
  if (!c || !state_in || (state_out_bar && !state_in_bar)) return CTM_E_ARG;
  c->err.clear();
  const Layout L = layout(c);
  Tape& t = tape_of(c);
  std::vector<TEnv> env;
  std::vector<const double*> a, X, Y;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) {
      t.begin_dry();
    } else {
      const int rc = t.reserve();
      if (rc) return afail(c, rc, t.error());
      t.begin();
    }
    bind_state(c, t, state_in, state_out_bar == nullptr, env, X, Y);
    if (state_out_bar && pass == 1) t.external_grad(state_in, state_in_bar);
    ATRY(taped_network(c, t, a));
    ATRY(taped_move(c, t, a, env, X, Y));
  }
  const long cc = (long)c->chi * c->chi, tt = (long)c->chi * c->Dl * c->chi, nk = (long)c->Nf * c->k;
  if (state_out) {
    for (int s = 0; s < c->ns; ++s)
      for (int i = 0; i < 4; ++i) {
        ATRY(t.copy_out(env[s].C[i], state_out + L.C(s, i), cc));
        ATRY(t.copy_out(env[s].T[i], state_out + L.T(s, i), tt));
      }
    for (int id = 0; id < 4 * c->ns; ++id) {
      ATRY(t.copy_out(X[id], state_out + L.X(id), nk));
      ATRY(t.copy_out(Y[id], state_out + L.Y(id), nk));
    }
  }
  if (state_out_bar) {
    for (int s = 0; s < c->ns; ++s)
      for (int i = 0; i < 4; ++i) {
        ATRY(t.seed(env[s].C[i], state_out_bar + L.C(s, i), cc));
        ATRY(t.seed(env[s].T[i], state_out_bar + L.T(s, i), tt));
      }
    for (int id = 0; id < 4 * c->ns; ++id) {
      ATRY(t.seed(X[id], state_out_bar + L.X(id), nk));
      ATRY(t.seed(Y[id], state_out_bar + L.Y(id), nk));
    }
    ATRY(t.backward());
    if (site_bar) {
      const long sn = site_doubles(c);
      for (int s = 0; s < c->ns; ++s)
        ATRY(t.accumulate_grad(c->cfg.d > 0 ? c->A[s] : c->a[s], site_bar + s * sn, sn));
    }
  }
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  if (!t.error().empty()) return afail(c, CTM_E_NOMEM, t.error());
  return CTM_OK;
}

int impl_energy_vjp(ctm_cell* cell, const double* state, const double* ops_host,
                               int bonds, double* e_out, double* state_bar, double* site_bar) {
  ctm_cell* c = cell;
  if (!c || !state || !ops_host || !e_out) return CTM_E_ARG;
  if (c->cfg.d < 1) return afail(c, CTM_E_STATE, "the energy needs physical legs (d > 0)");
  if (bonds <= 0 || bonds > 7) return afail(c, CTM_E_ARG, "bonds: a mask of 1 (h), 2 (v), 4 (d)");
  c->err.clear();
  Tape& t = tape_of(c);
  std::vector<TEnv> env;
  std::vector<const double*> a, X, Y;
  std::vector<double*> vals;
  const bool grads = state_bar || site_bar;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) {
      t.begin_dry();
    } else {
      const int rc = t.reserve();
      if (rc) return afail(c, rc, t.error());
      t.begin();
    }
    bind_state(c, t, state, !state_bar, env, X, Y);
    if (state_bar && pass == 1) t.external_grad(state, state_bar);
    ATRY(taped_network(c, t, a));
    ATRY(taped_energy(c, t, env, a, ops_host, bonds, vals));
  }
  std::vector<double> hv(vals.size());
  for (size_t i = 0; i < vals.size(); ++i)
    CTM_HIP_TRY(hipMemcpyAsync(&hv[i], vals[i], 8, hipMemcpyDeviceToHost, c->st));
  if (grads) {
    for (double* v : vals) ATRY(t.seed_scalar(v, 1.0 / c->ns));
    ATRY(t.backward());
    if (site_bar) {
      const long sn = site_doubles(c);
      for (int s = 0; s < c->ns; ++s) ATRY(t.accumulate_grad(c->A[s], site_bar + s * sn, sn));
    }
  }
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  if (!t.error().empty()) return afail(c, CTM_E_NOMEM, t.error());
  double e = 0.0;
  for (double v : hv) e += v;
  *e_out = e / c->ns;
  return CTM_OK;
}

}  // namespace

extern "C" {

ctm_status ctm_cell_state_size(const ctm_cell* cell, size_t* n) {
  if (!cell || !n) return CTM_E_ARG;
  *n = (size_t)layout(cell).total();
  return CTM_OK;
}

ctm_status ctm_cell_get_state_device(ctm_cell* cell, double* dev, size_t n) {
  return (ctm_status)impl_get_state_device(cell, dev, n);
}

ctm_status ctm_cell_set_state_device(ctm_cell* cell, const double* dev, size_t n) {
  return (ctm_status)impl_set_state_device(cell, dev, n);
}

ctm_status ctm_cell_move_vjp(ctm_cell* cell, const double* state_in, const double* state_out_bar,
                             double* state_in_bar, double* site_bar, double* state_out) {
  return (ctm_status)impl_move_vjp(cell, state_in, state_out_bar, state_in_bar, site_bar, state_out);
}

ctm_status ctm_cell_energy_vjp(ctm_cell* cell, const double* state, const double* ops_host,
                               int bonds, double* e_out, double* state_bar, double* site_bar) {
  return (ctm_status)impl_energy_vjp(cell, state, ops_host, bonds, e_out, state_bar, site_bar);
}

}  // extern "C"
