// Host orchestration of the SI-CTMRG move and the C ABI of include/ctm.h.
//
// A move (Fig. 1 of Zhang & Corboz) on one GPU, all of it stream-ordered on
// the context's stream:
//   1. enlarged corners Ct_i = T_(i-1) C_i T_i a, batched over the 4 corners
//      (three GEMMs each: C T, then T (C T), then the absorption of a);
//   2. projectors of the 4 bonds, batched:
//      - SI (QR-based projector section, steps 1-3): n_si subspace steps, each
//        8 applications of enlarged corners to the N x k blocks (X side and
//        Y side together, 8 problems per launch) and Householder QRs; then
//        A = R X, B^T = L^T Y^T, rho = B A, SVD of rho, the sign rule,
//        the pseudo-inverse scaling and the gauge recycle X <- X v,
//        Y <- u^T Y (eq. xy_recycle);
//      - full SVD (Standard CTMRG section): M_b = L_b R_b formed explicitly
//        and decomposed with rocSOLVER dgesvd; used for the comparator and
//        for growth moves that truncate;
//      - growth without truncation: identity projectors;
//   3. renormalisation C' = P_r Ct P_l and T' = P_r (T a) P_l;
//   4. unit Frobenius normalisation, NaN / zero guard, corner spectra and
//      the convergence measure.
// The environment is double-buffered: a move that fails the numeric guard
// leaves the committed corners and edges untouched.

#include "../../include/ctm.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "elem.h"
#include "vjp.h"

namespace sictm {

thread_local std::string g_err;

int hip_fail(hipError_t e, const char* what, int line) {
  g_err = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what + " (ctm.hip:" +
          std::to_string(line) + ")";
  return CTM_E_DEVICE;
}
const std::string& thread_error() { return g_err; }
void set_thread_error(const std::string& s) { g_err = s; }

}  // namespace sictm

using namespace sictm;

namespace {

size_t dt_size(DT t) { return t == DT::F64 ? 8 : (t == DT::F32 ? 4 : 2); }

struct Carver {
  char* base = nullptr;
  size_t off = 0;
  std::vector<std::pair<uintptr_t, uintptr_t>>* reg = nullptr;   // [begin, end) of each buffer
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    if (base && reg) reg->push_back({(uintptr_t)p, (uintptr_t)p + count * sizeof(T)});
    off += count * sizeof(T);
    return p;
  }
  void* take_bytes(size_t bytes) { return take<char>(bytes); }
};

// Recycling stops when delta grows by more than this factor between two
// successive SI moves (a stale subspace shows up in the corner spectra).
constexpr double kRecycleGuard = 10.0;

enum ProfClass { PC_CORNER = 0, PC_SI_APPLY, PC_QR, PC_SVD, PC_PROJ, PC_RENORM, PC_FULLSVD, PC_MISC, PC_N };
const char* kProfNames[PC_N] = {"corner_build", "si_apply", "householder_qr", "jacobi_svd",
                                "projector_gemm", "renormalise", "full_svd", "misc"};

// One operation of a recorded move (a batched move records the device work
// of each context's move, then launches the float64 GEMMs of the same step
// of every context as one grouped launch and the other operations in turn).
struct BatchOp {
  bool gemm;                              // a float64 GEMM that may be grouped
  GemmBatch g;
  std::function<int(hipStream_t)> fn;     // any other launch, on the given stream
};

}  // namespace

struct ctm_ctx {
  ctm_config cfg;
  int d, D, Dl, chi, k, N, xmax, Nmax;
  DT cp;
  bool split = false;        // contractions as split bfloat16 products (cp = F32 storage)
  hipStream_t st;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  // state
  int chi_env = 0, cur = 0, spec_cur = 0;
  bool si_ready = false, iso_pending = false;
  long si_moves = 0, moves = 0;
  // recycling of the SI blocks: `recycling` turns the subspace steps off;
  // si_upd counts SI moves with steps since recycling last stopped;
  // last_si_delta is the delta of the previous move if it was an SI move
  bool recycling = false;
  int si_upd = 0;
  double last_si_delta = -1.0;
  // buffers
  double* A_site = nullptr;
  double* a = nullptr;
  void* ap[4];
  void* apr[4];              // ap with its two leading legs swapped (renormalisation)
  double* imp[3];            // impurity scratch (Dl^4 each)
  double* imps[2];           // open-leg impurities of the two bond sites (d^2 Dl^4 each)
  double* e = nullptr;
  double* C[2][4];
  double* T[2][4];
  double* X[4];
  double* Yt[4];
  double* X0[4];
  double* Yt0[4];
  double* W[2][8];
  double* Xprev[8];          // recycling: blocks of the previous move (X then Y^T)
  double* ov[8];             // recycling: chi x chi overlaps of old and new blocks
  void* Ct[4];
  double* S1[4];
  double* S2[4];
  double* CT[4];
  double *rho[4], *u[4], *v[4], *vs[4], *s[4], *sg[4], *vsc[4], *usc[4];
  double *Pl[4], *Prt[4], *Zc[4];
  double* spec[2];
  double* csv[4];
  double* scal;              // [0..7] norms, [8] delta, [9..12] gap, [16..] observables
  int* bad;
  void* qr_ws;
  void* svd_ws;
  double *fs_s, *fs_E, *fs_sg, *fs_Us, *fs_Vs;
  int* fs_info;
  int* fs_perm;              // descending order of the dense SVD's singular values
  double* sk_part = nullptr;  // partial tiles of the balanced SI applications
  double* dot_part = nullptr; // partial sums of the plaquette dot products and of the norms
  // correlation length: block of kXiBlock vectors of the transfer matrix
  double *xi_V = nullptr, *xi_Vc = nullptr, *xi_W = nullptr, *xi_H = nullptr, *xi_out = nullptr;
  void* xi_qr = nullptr;
  int xi_m = 0;
  int sk_cus = kSplitMaxCus;  // CUs a balanced launch spreads over
  double* obs_y;             // [d^2][x Dl x]
  double* obs_w;             // [d^2][x Dl x]
  double* obs_op;            // [d^4] device copy of an operator
  rocblas_handle rb = nullptr;
  std::string err;
  // asynchronous moves: results land in pinned host memory, completion is
  // signalled by done_ev; the host-side state advances in finish_move
  double* hbuf = nullptr;    // [0..15] scal copy, [16] bad flag (as int)
  hipEvent_t done_ev = nullptr;
  // second stream of an eager move: the new corners' norms and spectra run
  // on it while the edges are renormalised (fork and join by events).
  // Created on the first eager move that uses it; contexts that replay
  // captured moves (ctm_use_graphs) keep the one-stream schedule.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool pending = false;
  int pend_mode = 0, pend_keep = 0, pend_nsi = 0;
  bool pend_measure = false;
  // captured SI moves: the device work of a move depends on the generation
  // `cur` and on the arrangement of the block pointers (the QR and the
  // recycling swap them), so a graph is kept per (cur, arrangement) with the
  // arrangement the move leaves behind
  bool use_graphs = false;
  struct GraphRec {
    int cur, spec_cur, nsi;
    bool measure;
    std::vector<void*> pre, post;
    hipGraphExec_t exec;
  };
  std::vector<GraphRec> graphs;
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  struct Rec { int cls; hipEvent_t a, b; double flops, bytes; };
  std::vector<Rec> recs;
  size_t ev_next = 0;
  // carved buffers, for the host-side bounds check of every GEMM launch
  std::vector<std::pair<uintptr_t, uintptr_t>> bufs;
  // while a batched move records this context's work: its operations
  std::vector<BatchOp>* rec = nullptr;
};

namespace {

int fail(ctm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return code;
}

// Propagates a non-zero launcher code (1 = bad argument) with its message.
#define TRY(expr)                                                    \
  do {                                                               \
    int _r = (expr);                                                 \
    if (_r != 0) {                                                   \
      c->err = g_err.empty() ? std::string(#expr) : g_err;           \
      return _r == 1 ? (int)CTM_E_ARG : _r;                          \
    }                                                                \
  } while (0)

// Device work of a move other than a float64 GEMM: launched on the
// context's stream, or, while a batched move records the context, kept as an
// operation (`st` names the stream inside the expression; its arguments are
// evaluated when it runs, so anything the recording changes afterwards -- the
// block pointers -- is copied into locals first).
#define ENQ(expr)                                                                 \
  do {                                                                            \
    if (c->rec) {                                                                 \
      c->rec->push_back(BatchOp{false, GemmBatch{}, [=](hipStream_t st) -> int {  \
                                  return (expr);                                  \
                                }});                                              \
    } else {                                                                      \
      hipStream_t st = c->st;                                                     \
      TRY(expr);                                                                  \
    }                                                                             \
  } while (0)

int hrc(hipError_t e) { return e == hipSuccess ? 0 : hip_fail(e, "stream operation", __LINE__); }

// Propagates a launcher code where no single context is concerned.
#define TRY_B(expr)                                  \
  do {                                               \
    int _r = (expr);                                 \
    if (_r != 0) return _r == 1 ? (int)CTM_E_ARG : _r; \
  } while (0)

int validate(const ctm_config* cfg) {
  if (!cfg) return fail(nullptr, CTM_E_ARG, "null config");
  if (cfg->d < 0 || cfg->D < 1 || cfg->chi < 1 || cfg->p < 0 || cfg->n_si < 0)
    return fail(nullptr, CTM_E_SHAPE, "need d >= 0, D >= 1, chi >= 1, p >= 0, n_si >= 0");
  if (cfg->proj != CTM_PROJ_FULLSVD && cfg->proj != CTM_PROJ_SI)
    return fail(nullptr, CTM_E_ARG, "unknown projector kind");
  if (cfg->prec < CTM_PREC_F64 || cfg->prec > CTM_PREC_BF16X3)
    return fail(nullptr, CTM_E_ARG, "unknown precision");
  if (!(cfg->pinv_rtol >= 0.0)) return fail(nullptr, CTM_E_ARG, "pinv_rtol must be >= 0");
  if (cfg->growth != 0 && cfg->growth != 1)
    return fail(nullptr, CTM_E_ARG, "growth must be 0 (full SVD) or 1 (randomized)");
  if (cfg->svd_driver < 0 || cfg->svd_driver > 2)
    return fail(nullptr, CTM_E_ARG, "svd_driver must be 0 (gesvd), 1 (gesdd) or 2 (gesvdx)");
  if (cfg->sym != CTM_SYM_NONE && cfg->sym != CTM_SYM_C4V)
    return fail(nullptr, CTM_E_ARG, "sym must be CTM_SYM_NONE or CTM_SYM_C4V");
  if (cfg->sym == CTM_SYM_C4V && cfg->prec != CTM_PREC_F64)
    return fail(nullptr, CTM_E_ARG, "the C4v mode runs in float64 only");
  if (!(cfg->recycle_sin2 == cfg->recycle_sin2))
    return fail(nullptr, CTM_E_ARG, "recycle_sin2 must be a number");
  if (cfg->recycle_sin2 > 0 && cfg->min_si_moves < 1)
    return fail(nullptr, CTM_E_ARG, "min_si_moves must be >= 1 when recycling");
  if (cfg->recycle_sin2 > 0 && cfg->sym == CTM_SYM_C4V)
    return fail(nullptr, CTM_E_ARG, "recycling is implemented for the four-direction move only");
  const int Dl = cfg->d > 0 ? cfg->D * cfg->D : cfg->D;
  const long N = (long)cfg->chi * Dl;
  const long k = std::min<long>(cfg->chi + cfg->p, N);
  if (k > 192) return fail(nullptr, CTM_E_SHAPE, "chi + p must be <= 192");
  if (cfg->proj == CTM_PROJ_SI && !qr_plan_ok((int)N, (int)k))
    return fail(nullptr, CTM_E_SHAPE,
                "no QR leaf partition for N = chi*Dl = " + std::to_string(N) + " rows and k = " +
                    std::to_string(k) + " columns: the rows must split into leaves of k to 192 "
                    "rows (reduce p, or choose chi so that such a split exists)");
  if (N > 65536) return fail(nullptr, CTM_E_SHAPE, "chi * Dl must be <= 65536");
  return CTM_OK;
}

void set_dims(ctm_ctx* c, const ctm_config* cfg) {
  c->cfg = *cfg;
  c->d = cfg->d;
  c->D = cfg->D;
  c->Dl = cfg->d > 0 ? cfg->D * cfg->D : cfg->D;
  c->chi = cfg->chi;
  c->N = c->chi * c->Dl;
  c->k = std::min(c->chi + cfg->p, c->N);
  c->xmax = std::max(c->chi, c->Dl);
  c->Nmax = c->xmax * c->Dl;
  // split bfloat16 keeps its contraction operands in float32 and splits them
  // into bfloat16 pairs inside the GEMM kernels
  c->cp = cfg->prec == CTM_PREC_F64 ? DT::F64
          : (cfg->prec == CTM_PREC_F32 || cfg->prec == CTM_PREC_BF16X3) ? DT::F32
                                                                       : DT::BF16;
  c->split = cfg->prec == CTM_PREC_BF16X3;
}

// Vectors of the block iteration for the correlation length.
constexpr int kXiBlock = 8;

// Assigns every buffer of the context from base (or only sizes it).
size_t carve(ctm_ctx* c, char* base) {
  Carver cv;
  cv.base = base;
  c->bufs.clear();
  cv.reg = &c->bufs;
  const size_t Dl4 = (size_t)c->Dl * c->Dl * c->Dl * c->Dl;
  const size_t xm = c->xmax, Dl = c->Dl, N = c->N, k = c->k, chi = c->chi, Nm = c->Nmax;
  const size_t es = dt_size(c->cp);
  const int dd = std::max(1, c->d * c->d);
  c->A_site = cv.take<double>(c->d > 0 ? (size_t)c->d * c->D * c->D * c->D * c->D : 1);
  c->a = cv.take<double>(Dl4);
  for (int i = 0; i < 4; ++i) c->ap[i] = cv.take_bytes(Dl4 * es);
  for (int i = 0; i < 4; ++i) c->apr[i] = cv.take_bytes(Dl4 * es);
  for (int i = 0; i < 3; ++i) c->imp[i] = cv.take<double>(Dl4);
  for (int i = 0; i < 2; ++i) c->imps[i] = cv.take<double>((size_t)dd * Dl4);
  c->e = cv.take<double>(Dl);
  for (int b = 0; b < 2; ++b)
    for (int i = 0; i < 4; ++i) {
      c->C[b][i] = cv.take<double>(xm * xm);
      c->T[b][i] = cv.take<double>(xm * Dl * xm);
    }
  for (int i = 0; i < 4; ++i) {
    c->X[i] = cv.take<double>(N * k);
    c->Yt[i] = cv.take<double>(N * k);
    c->X0[i] = cv.take<double>(N * k);
    c->Yt0[i] = cv.take<double>(N * k);
  }
  for (int s = 0; s < 2; ++s)
    for (int i = 0; i < 8; ++i) c->W[s][i] = cv.take<double>(N * k);
  const bool rec = c->cfg.recycle_sin2 > 0;
  for (int i = 0; i < 8; ++i) {
    c->Xprev[i] = rec ? cv.take<double>(N * k) : nullptr;
    c->ov[i] = rec ? cv.take<double>(chi * chi) : nullptr;
  }
  for (int i = 0; i < 4; ++i) c->Ct[i] = cv.take_bytes(Nm * Nm * es);
  for (int i = 0; i < 4; ++i) c->S1[i] = cv.take<double>(Nm * Nm);
  for (int i = 0; i < 4; ++i) c->S2[i] = cv.take<double>(Nm * Nm);
  for (int i = 0; i < 4; ++i) c->CT[i] = cv.take<double>(xm * Dl * xm);
  for (int i = 0; i < 4; ++i) {
    c->rho[i] = cv.take<double>(k * k);
    c->u[i] = cv.take<double>(k * k);
    c->v[i] = cv.take<double>(k * k);
    c->vs[i] = cv.take<double>(k * k);
    c->s[i] = cv.take<double>(std::max(k, xm));
    c->sg[i] = cv.take<double>(std::max(k, xm));
    c->vsc[i] = cv.take<double>(k * chi);
    c->usc[i] = cv.take<double>(k * chi);
    c->Pl[i] = cv.take<double>(Nm * std::max(Nm, chi));
    c->Prt[i] = cv.take<double>(Nm * std::max(Nm, chi));
    c->Zc[i] = cv.take<double>(Nm * std::max(Nm, chi));
    c->csv[i] = cv.take<double>(xm);
  }
  for (int i = 0; i < 2; ++i) c->spec[i] = cv.take<double>(4 * chi);
  c->scal = cv.take<double>(256);
  c->bad = cv.take<int>(64);
  c->qr_ws = cv.take_bytes(qr_workspace_bytes(8, (int)N, (int)k));
  c->svd_ws = cv.take_bytes(svd_workspace_bytes(8, (int)std::max(k, xm)));
  c->fs_s = cv.take<double>(Nm);
  c->fs_E = cv.take<double>(Nm);
  c->fs_sg = cv.take<double>(Nm);
  c->fs_Us = cv.take<double>(Nm * chi);
  c->fs_Vs = cv.take<double>(Nm * chi);
  c->fs_info = cv.take<int>(64);
  c->fs_perm = cv.take<int>(Nm);
  c->dot_part = cv.take<double>((size_t)kMaxDots * kDotBlocks);
  {
    const size_t nE = chi * Dl * chi;
    c->xi_m = (int)std::min<size_t>(kXiBlock, nE);
    const bool qr_ok = qr_plan_ok((int)nE, c->xi_m);
    c->xi_V = cv.take<double>(nE * c->xi_m);
    c->xi_Vc = cv.take<double>(nE * c->xi_m);
    c->xi_W = cv.take<double>(nE * c->xi_m);
    c->xi_H = cv.take<double>((size_t)kXiBlock * kXiBlock);
    c->xi_out = cv.take<double>(8);
    c->xi_qr = qr_ok ? cv.take_bytes(qr_workspace_bytes(1, (int)nE, c->xi_m)) : nullptr;
  }
  c->sk_part = (c->cp == DT::F64 || (c->cp == DT::F32 && !c->split)) &&
                       gemm_si_balanced_useful(8, (int)N, (int)k, (int)N, kSplitMaxCus)
                   ? (double*)cv.take_bytes(gemm_si_scratch_bytes())
                   : nullptr;
  c->obs_y = cv.take<double>((size_t)dd * xm * Dl * xm);
  c->obs_w = cv.take<double>((size_t)dd * xm * Dl * xm);
  c->obs_op = cv.take<double>(256);
  std::sort(c->bufs.begin(), c->bufs.end());
  return cv.off + 256;
}

// ---------------------------------------------------------------------------
// profiling: hipEvent pairs around launches of each class
// ---------------------------------------------------------------------------
struct ProfScope {
  ctm_ctx* c;
  int cls;
  double flops, bytes;
  hipEvent_t a{}, b{};
  ProfScope(ctm_ctx* ctx, int cl, double fl = 0, double by = 0) : c(ctx), cls(cl), flops(fl), bytes(by) {
    if (!c->prof) return;
    a = next();
    (void)hipEventRecord(a, c->st);
  }
  hipEvent_t next() {
    if (c->ev_next >= c->ev_pool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_next++];
  }
  ~ProfScope() {
    if (!c->prof) return;
    b = next();
    (void)hipEventRecord(b, c->st);
    c->recs.push_back({cls, a, b, flops, bytes});
  }
};

GemmBatch gemm_rowmajor(int count, int M, int N, int K, long lda, long ldb, long ldc) {
  GemmBatch g{};
  g.count = count;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  gemm_set_rowmajor_c(g, ldc);
  g.nbatch = 1;
  g.alpha = 1.0;
  return g;
}

void set_map(GemmBatch& g, int mdiv, long m1, long m0, int ndiv, long n1, long n0) {
  g.cdiv_m = mdiv; g.cs_m1 = m1; g.cs_m0 = m0;
  g.cdiv_n = ndiv; g.cs_n1 = n1; g.cs_n0 = n0;
}

double gemm_flops(const GemmBatch& g) { return 2.0 * g.M * g.N * (double)g.K * g.count * g.nbatch; }

// Largest element offset a 2-level map can address for indices < n.
long map_extent(int n, int div, long s1, long s0) {
  if (n <= 0) return 0;
  return (long)((n - 1) / div) * s1 + (long)std::min(div - 1, n - 1) * s0;
}

// True if [p, p + bytes) lies inside one carved buffer of the context.
bool inside(const ctm_ctx* c, const void* p, size_t bytes) {
  const uintptr_t a = (uintptr_t)p;
  auto it = std::upper_bound(c->bufs.begin(), c->bufs.end(),
                             std::make_pair(a, std::numeric_limits<uintptr_t>::max()));
  if (it == c->bufs.begin()) return false;
  --it;
  return a >= it->first && a + bytes <= it->second;
}

// Host-side bounds check of every operand of a GEMM launch against the
// buffer that holds its base pointer; refuses to launch on a violation.
int check_gemm(ctm_ctx* c, const GemmBatch& g, DT ta, DT tb, DT tc) {
  if (g.M <= 0 || g.N <= 0) return 0;
  for (int i = 0; i < g.count; ++i) {
    const long ea = g.K <= 0 ? 0
                    : (g.transA[i] ? (long)(g.K - 1) * g.lda + (g.M - 1)
                                   : (long)(g.M - 1) * g.lda + (g.K - 1)) +
                          (long)(g.nbatch - 1) * g.a_bs;
    const long eb = g.K <= 0 ? 0 : (long)(g.K - 1) * g.ldb + (g.N - 1) + (long)(g.nbatch - 1) * g.b_bs;
    const long ec = map_extent(g.M, g.cdiv_m, g.cs_m1, g.cs_m0) +
                    map_extent(g.N, g.cdiv_n, g.cs_n1, g.cs_n0) + (long)(g.nbatch - 1) * g.c_bs;
    const bool ok = (g.K <= 0 || inside(c, g.A[i], (size_t)(ea + 1) * dt_size(ta))) &&
                    (g.K <= 0 || inside(c, g.B[i], (size_t)(eb + 1) * dt_size(tb))) &&
                    inside(c, g.C[i], (size_t)(ec + 1) * dt_size(tc));
    if (!ok) {
      g_err = "GEMM operand out of its buffer (M=" + std::to_string(g.M) + " N=" +
              std::to_string(g.N) + " K=" + std::to_string(g.K) + " problem " +
              std::to_string(i) + "); launch refused";
      return CTM_E_SHAPE;
    }
  }
  return 0;
}

int run_gemm(ctm_ctx* c, int cls, const GemmBatch& g0, DT ta, DT tb, DT tc, double bytes = 0) {
  const int chk = check_gemm(c, g0, ta, tb, tc);
  if (chk) return chk;
  GemmBatch g = g0;
  // in the split bfloat16 mode every product with a float32-stored operand is
  // a contraction of the mode
  if (c->split && (ta == DT::F32 || tb == DT::F32)) g.split = 1;
  // thin float64 products with long K on the split kernel of the SI
  // applications (its own launch in a recorded batch: it sums cut tiles in
  // a fixed order of its own, so the product keeps the bits of a solo move)
  if (ta == DT::F64 && tb == DT::F64 && tc == DT::F64 && !g.split &&
      gemm_si_balanced_applies(g, c->sk_part, c->sk_cus)) {
    double* part = c->sk_part;
    const int cus = c->sk_cus;
    if (c->rec) {
      c->rec->push_back(BatchOp{false, GemmBatch{}, [=](hipStream_t st) {
                                  return launch_gemm_si_balanced(g, part, cus, st);
                                }});
      return 0;
    }
    ProfScope ps(c, cls, gemm_flops(g), bytes);
    return launch_gemm_si_balanced(g, part, cus, c->st);
  }
  // the float32 contractions of that shape on the float32 split kernel
  if (ta == DT::F32 && tb == DT::F64 && tc == DT::F64 && !g.split && !c->rec &&
      gemm_si_f32_balanced_applies(g, c->sk_part, c->sk_cus)) {
    ProfScope ps(c, cls, gemm_flops(g), bytes);
    return launch_gemm_si_f32_balanced(g, c->sk_part, c->sk_cus, c->st);
  }
  if (c->rec) {
    if (ta == DT::F64 && tb == DT::F64 && tc == DT::F64)
      c->rec->push_back(BatchOp{true, g, nullptr});
    else
      c->rec->push_back(BatchOp{false, GemmBatch{}, [=](hipStream_t st) {
                                  return launch_gemm(g, ta, tb, tc, st);
                                }});
    return 0;
  }
  ProfScope ps(c, cls, gemm_flops(g), bytes);
  return launch_gemm(g, ta, tb, tc, c->st);
}

// ---------------------------------------------------------------------------
// step 1: enlarged corners (batched over the four corners)
// ---------------------------------------------------------------------------
// The environment part of the four enlarged corners (float64):
// CT_i = C_i T_i into CT[i] and W_i = T_(i-1) CT_i into S1[i].  CT_i is
// stored with its last two legs swapped, (y, q) instead of T_i's (q, y), so
// that the columns of the second product, the large one (x^2 D^4 outputs per
// corner), run along q, the unit-stride leg of W_i; the scattered stores fall
// on the first product, whose output is D^2 times smaller.
int corner_stems(ctm_ctx* c, int phase) {
  const int x = c->chi_env, Dl = c->Dl;
  double* const* C = c->C[c->cur];
  double* const* T = c->T[c->cur];
  // CT_i[a, (y, q)] = C_i[a, b] T_i[b, q, y]
  GemmBatch g1 = gemm_rowmajor(4, x, Dl * x, x, x, (long)Dl * x, 0);
  set_map(g1, 1 << 30, 0, (long)Dl * x, x, 1, Dl);
  for (int i = 0; i < 4; ++i) {
    g1.A[i] = C[i];
    g1.B[i] = T[i];
    g1.C[i] = c->CT[i];
  }
  TRY(run_gemm(c, phase, g1, DT::F64, DT::F64, DT::F64));
  // W_i[(x_in, y), (p, q)] = T_(i-1)[(x_in, p), a] CT_i[a, (y, q)]
  GemmBatch g2 = gemm_rowmajor(4, x * Dl, Dl * x, x, x, (long)Dl * x, 0);
  set_map(g2, Dl, (long)x * Dl * Dl, Dl, Dl, (long)Dl * Dl, 1);
  for (int i = 0; i < 4; ++i) {
    g2.A[i] = T[(i + 3) % 4];
    g2.B[i] = c->CT[i];
    g2.C[i] = c->S1[i];
  }
  TRY(run_gemm(c, phase, g2, DT::F64, DT::F64, DT::F64));
  return 0;
}

// The site absorption of enlarged corners (after corner_stems):
// Ct_i[(x_in, o1), (y, o2)] = W_i[(x_in, y), (p, q)] site_i[(p, q), (o1, o2)]
// with site_i the corner-i permutation of the site tensor.
GemmBatch corner_site_gemm(ctm_ctx* c, int count) {
  const int x = c->chi_env, Dl = c->Dl, N1 = x * Dl;
  GemmBatch g3 = gemm_rowmajor(count, x * x, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
  g3.cdiv_m = x;
  g3.cs_m1 = (long)Dl * N1;
  g3.cs_m0 = Dl;
  g3.cdiv_n = Dl;
  g3.cs_n1 = N1;
  g3.cs_n0 = 1;
  return g3;
}

int build_corners(ctm_ctx* c) {
  TRY(corner_stems(c, PC_CORNER));
  if ((c->cp == DT::F64 || (c->cp == DT::F32 && !c->split)) && c->d > 0 &&
      absorb_corner_fits(c->D, c->d)) {
    // the single-layer absorption (ket layer, then bra layer with the
    // physical index): the same corners for a ninth of the flops at D = 6,
    // in float64 arithmetic (also in the float32 mode, where it is faster
    // than the float32 double-layer product; the corners are stored in the
    // mode's type)
    const bool f32 = c->cp == DT::F32;
    const long D = c->D, su = D * D * D, sl = D * D, sd = D, sr = 1;
    const long legs[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
    const double* W[4];
    void* Ct[4];
    for (int i = 0; i < 4; ++i) {
      W[i] = c->S1[i];
      Ct[i] = c->Ct[i];
    }
    const double* A = c->A_site;
    const int x = c->chi_env, Dd = c->D, d = c->d;
    if (c->rec) {
      struct Ptrs { const double* W[4]; void* Ct[4]; long legs[4][4]; } pp;
      std::memcpy(pp.W, W, sizeof(W));
      std::memcpy(pp.Ct, Ct, sizeof(Ct));
      std::memcpy(pp.legs, legs, sizeof(legs));
      c->rec->push_back(BatchOp{false, GemmBatch{}, [=](hipStream_t st) {
                                  return launch_absorb_corners(pp.W, pp.Ct, f32, A, pp.legs, x, Dd,
                                                               d, st);
                                }});
      return 0;
    }
    const double Dl = (double)c->Dl;
    ProfScope ps(c, PC_CORNER, 4.0 * 4.0 * x * x * Dl * Dl * Dl * d);
    const int r = launch_absorb_corners(W, Ct, f32, A, legs, x, Dd, d, c->st);
    if (r) return fail(c, CTM_E_DEVICE, thread_error());
    return 0;
  }
  GemmBatch g3 = corner_site_gemm(c, 4);
  for (int i = 0; i < 4; ++i) {
    g3.A[i] = c->S1[i];
    g3.B[i] = c->ap[i];
    g3.C[i] = c->Ct[i];
  }
  TRY(run_gemm(c, PC_CORNER, g3, DT::F64, c->cp, c->cp));
  return 0;
}

// One application step: dst_i = op(Ct[ci_i]) src_i for up to 8 problems.
int apply_step(ctm_ctx* c, int count, const int* ci, const int* trans, double* const* src,
               double* const* dst, int N1) {
  const int k = c->k;
  GemmBatch g = gemm_rowmajor(count, N1, k, N1, N1, k, k);
  for (int i = 0; i < count; ++i) {
    g.A[i] = c->Ct[ci[i]];
    g.transA[i] = trans[i];
    g.B[i] = src[i];
    g.C[i] = dst[i];
  }
  const double bytes = (double)count * ((double)N1 * N1 * dt_size(c->cp) + 2.0 * N1 * k * 8.0);
  if (c->rec && c->cp == DT::F64) {
    const int chk = check_gemm(c, g, DT::F64, DT::F64, DT::F64);
    if (chk) return chk;
    // the split kernel sums cut tiles in its own order: kept as its own launch
    // so that the product has the bits of a solo move; the tile kernels give
    // the same bits in any grid and are grouped
    if (gemm_si_balanced_applies(g, c->sk_part, c->sk_cus)) {
      double* part = c->sk_part;
      const int cus = c->sk_cus;
      c->rec->push_back(BatchOp{false, GemmBatch{}, [=](hipStream_t st) {
                                  return launch_gemm_si_balanced(g, part, cus, st);
                                }});
    } else {
      c->rec->push_back(BatchOp{true, g, nullptr});
    }
    return 0;
  }
  if (c->rec) return fail(c, CTM_E_STATE, "batched moves run float64 contractions only");
  if (c->cp == DT::F32) {
    const int chk = check_gemm(c, g, DT::F32, DT::F64, DT::F64);
    if (chk) return chk;
    ProfScope ps(c, PC_SI_APPLY, gemm_flops(g), bytes);
    if (c->split) return launch_gemm_si_bx3(g, c->st);
    return launch_gemm_si_f32_balanced(g, c->sk_part, c->sk_cus, c->st);
  }
  if (c->cp != DT::F64) return run_gemm(c, PC_SI_APPLY, g, c->cp, DT::F64, DT::F64, bytes);
  const int chk = check_gemm(c, g, DT::F64, DT::F64, DT::F64);
  if (chk) return chk;
  ProfScope ps(c, PC_SI_APPLY, gemm_flops(g), bytes);
  return launch_gemm_si_balanced(g, c->sk_part, c->sk_cus, c->st);
}

inline int md(int i) { return ((i % 4) + 4) % 4; }

// Applies M (or M^T) of every bond to the X side and the opposite operator
// to the Y side: the X block of bond b goes through Ct[b+2], Ct[b+1], Ct[b],
// Ct[b-1] (M) or their transposes in reverse order (M^T).
int half_step(ctm_ctx* c, bool x_with_M, int N1) {
  double* in[8];
  for (int b = 0; b < 4; ++b) {
    in[b] = c->X[b];
    in[4 + b] = c->Yt[b];
  }
  for (int t = 0; t < 4; ++t) {
    int ci[8], tr[8];
    double* out[8];
    for (int b = 0; b < 4; ++b) {
      const int mseq[4] = {md(b + 2), md(b + 1), md(b), md(b - 1)};
      const int tseq[4] = {md(b - 1), md(b), md(b + 1), md(b + 2)};
      ci[b] = x_with_M ? mseq[t] : tseq[t];
      tr[b] = x_with_M ? 0 : 1;
      ci[4 + b] = x_with_M ? tseq[t] : mseq[t];
      tr[4 + b] = x_with_M ? 1 : 0;
    }
    for (int i = 0; i < 8; ++i) out[i] = c->W[t & 1][i];
    TRY(apply_step(c, 8, ci, tr, in, out, N1));
    for (int i = 0; i < 8; ++i) in[i] = out[i];
  }
  return 0;
}

// The results of a half step live in W[1]; orthonormalise them in place and
// make them the current blocks (pointer swap, no copy).
int qr_and_swap(ctm_ctx* c, int N1) {
  {
    ProfScope ps(c, PC_QR, 8.0 * 4.0 * N1 * (double)c->k * c->k);
    double* w[8];
    for (int i = 0; i < 8; ++i) w[i] = c->W[1][i];
    const int k = c->k;
    void* ws = c->qr_ws;
    ENQ(launch_qr(8, w, N1, k, ws, st));
  }
  for (int b = 0; b < 4; ++b) {
    std::swap(c->X[b], c->W[1][b]);
    std::swap(c->Yt[b], c->W[1][4 + b]);
  }
  return 0;
}

int ensure_si_blocks(ctm_ctx* c) {
  const size_t nk = (size_t)c->N * c->k;
  if (c->iso_pending) {
    for (int b = 0; b < 4; ++b) {
      CTM_HIP_TRY(hipMemcpyAsync(c->X[b], c->X0[b], nk * 8, hipMemcpyDeviceToDevice, c->st));
      CTM_HIP_TRY(hipMemcpyAsync(c->Yt[b], c->Yt0[b], nk * 8, hipMemcpyDeviceToDevice, c->st));
    }
    c->iso_pending = false;
    c->si_ready = true;
  } else if (!c->si_ready) {
    for (int b = 0; b < 4; ++b) {
      TRY(elem_gauss(c->X[b], (long)nk, 1000 + b, c->st));
      TRY(elem_gauss(c->Yt[b], (long)nk, 2000 + b, c->st));
    }
    c->si_ready = true;
  }
  return 0;
}

// SI projectors of the four bonds (QR-based projector section, steps 1-3)
// with nsi subspace steps.  With `measure`, the recycling criterion (the
// largest over the 8 blocks of the mean sin^2 of the principal angles between
// the kept columns before and after the move) is written to scal[13].
int si_core(ctm_ctx* c, int keep, int nsi, bool measure, int N1);

int si_projectors(ctm_ctx* c, int keep, int nsi, bool measure) {
  TRY(ensure_si_blocks(c));
  return si_core(c, keep, nsi, measure, c->N);
}

// Randomized projectors of a truncating growth move (environment dimension
// chi_env < chi, N1 = chi_env Dl >= k rows): the SI steps run on the first
// N1 rows of the start blocks (or on Gaussian blocks when none were given),
// which stay pending for the first SI move.
int growth_si_projectors(ctm_ctx* c, int keep, int N1) {
  const size_t nk = (size_t)N1 * c->k;
  for (int b = 0; b < 4; ++b) {
    if (c->iso_pending) {
      CTM_HIP_TRY(hipMemcpyAsync(c->X[b], c->X0[b], nk * 8, hipMemcpyDeviceToDevice, c->st));
      CTM_HIP_TRY(hipMemcpyAsync(c->Yt[b], c->Yt0[b], nk * 8, hipMemcpyDeviceToDevice, c->st));
    } else {
      TRY(elem_gauss(c->X[b], (long)nk, 3000 + b, c->st));
      TRY(elem_gauss(c->Yt[b], (long)nk, 4000 + b, c->st));
    }
  }
  return si_core(c, keep, c->cfg.n_si, false, N1);
}

int si_core(ctm_ctx* c, int keep, int nsi, bool measure, int N1) {
  const int k = c->k;
  if (measure) {
    const size_t nk = (size_t)N1 * k * sizeof(double);
    for (int b = 0; b < 4; ++b) {
      double *dx = c->Xprev[b], *sx = c->X[b], *dy = c->Xprev[4 + b], *sy = c->Yt[b];
      ENQ(hrc(hipMemcpyAsync(dx, sx, nk, hipMemcpyDeviceToDevice, st)));
      ENQ(hrc(hipMemcpyAsync(dy, sy, nk, hipMemcpyDeviceToDevice, st)));
    }
  }
  for (int step = 0; step < nsi; ++step) {
    if (c->cfg.stabilized) {
      TRY(half_step(c, true, N1));   // X: M X      Y: M^T Y^T
      TRY(qr_and_swap(c, N1));
      TRY(half_step(c, false, N1));  // X: M^T (.)  Y: M (.)
      TRY(qr_and_swap(c, N1));
    } else {
      TRY(half_step(c, true, N1));
      for (int b = 0; b < 8; ++b) std::swap(b < 4 ? c->X[b] : c->Yt[b - 4], c->W[1][b]);
      TRY(half_step(c, false, N1));
      TRY(qr_and_swap(c, N1));
    }
  }
  // A_b = R_b X = Ct[b+1] (Ct[b+2] X);  B_b^T = L_b^T Y^T = Ct[b]^T (Ct[b-1]^T Y^T)
  {
    int ci[8], tr[8];
    double* in[8];
    double* out[8];
    for (int b = 0; b < 4; ++b) {
      ci[b] = md(b + 2); tr[b] = 0; in[b] = c->X[b]; out[b] = c->W[0][b];
      ci[4 + b] = md(b - 1); tr[4 + b] = 1; in[4 + b] = c->Yt[b]; out[4 + b] = c->W[0][4 + b];
    }
    TRY(apply_step(c, 8, ci, tr, in, out, N1));
    for (int b = 0; b < 4; ++b) {
      ci[b] = md(b + 1); in[b] = c->W[0][b]; out[b] = c->W[1][b];
      ci[4 + b] = md(b); in[4 + b] = c->W[0][4 + b]; out[4 + b] = c->W[1][4 + b];
    }
    TRY(apply_step(c, 8, ci, tr, in, out, N1));
  }
  double* const* A = c->W[1];        // A_b in W[1][b], B_b^T in W[1][4+b]
  // rho_b = B_b A_b = (B_b^T)^T A_b   (float64)
  {
    GemmBatch g = gemm_rowmajor(4, k, k, N1, k, k, k);
    for (int b = 0; b < 4; ++b) {
      g.A[b] = A[4 + b];
      g.transA[b] = 1;
      g.B[b] = A[b];
      g.C[b] = c->rho[b];
    }
    TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
  }
  {
    ProfScope ps(c, PC_SVD);
    ENQ(launch_svd(4, c->rho, c->u, c->s, c->v, k, c->svd_ws, st));
  }
  // Y^T u -> W[0][4+b]; signs from it
  {
    GemmBatch g = gemm_rowmajor(4, N1, k, k, k, k, k);
    for (int b = 0; b < 4; ++b) {
      g.A[b] = c->Yt[b];
      g.B[b] = c->u[b];
      g.C[b] = c->W[0][4 + b];
    }
    TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
  }
  SignArgs sa{};
  sa.N = N1;
  sa.k = k;
  sa.ld = k;
  for (int b = 0; b < 4; ++b) {
    sa.Y[b] = c->W[0][4 + b];
    sa.sg[b] = c->sg[b];
  }
  ENQ(elem_col_sign(sa, 4, st));
  ENQ(elem_scale_cols(sa, 4, st));
  ProjPrepArgs pa{};
  pa.k = k;
  pa.keep = keep;
  pa.rtol = c->cfg.pinv_rtol;
  pa.gap = c->scal + 9;
  for (int b = 0; b < 4; ++b) {
    pa.u[b] = c->u[b];
    pa.v[b] = c->v[b];
    pa.s[b] = c->s[b];
    pa.sg[b] = c->sg[b];
    pa.vs[b] = c->vs[b];
    pa.vsc[b] = c->vsc[b];
    pa.usc[b] = c->usc[b];
  }
  ENQ(elem_proj_prep(pa, 4, st));
  // X <- X v diag(sg) (into W[0][b]); P_l = A vsc; P_r^T = B^T usc
  {
    GemmBatch g = gemm_rowmajor(4, N1, k, k, k, k, k);
    for (int b = 0; b < 4; ++b) {
      g.A[b] = c->X[b];
      g.B[b] = c->vs[b];
      g.C[b] = c->W[0][b];
    }
    TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
  }
  {
    GemmBatch g = gemm_rowmajor(8, N1, keep, k, k, keep, keep);
    for (int b = 0; b < 4; ++b) {
      g.A[b] = A[b];
      g.B[b] = c->vsc[b];
      g.C[b] = c->Pl[b];
      g.A[4 + b] = A[4 + b];
      g.B[4 + b] = c->usc[b];
      g.C[4 + b] = c->Prt[b];
    }
    TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
  }
  for (int b = 0; b < 4; ++b) {
    std::swap(c->X[b], c->W[0][b]);
    std::swap(c->Yt[b], c->W[0][4 + b]);
  }
  if (measure) {
    // G_b = Q_old[:, :chi]^T Q_new[:, :chi] for the 8 blocks, then the criterion
    const int chi = c->chi;
    GemmBatch g = gemm_rowmajor(8, chi, chi, N1, k, k, chi);
    for (int b = 0; b < 8; ++b) {
      g.A[b] = c->Xprev[b];
      g.transA[b] = 1;
      g.B[b] = b < 4 ? c->X[b] : c->Yt[b - 4];
      g.C[b] = c->ov[b];
    }
    TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
    OverlapArgs oa{};
    for (int b = 0; b < 8; ++b) oa.G[b] = c->ov[b];
    oa.count = 8;
    oa.chi = chi;
    oa.out = c->scal + 13;
    ENQ(elem_sin2(oa, st));
  }
  return 0;
}

int ensure_rocblas(ctm_ctx* c) {
  if (c->rb) return 0;
  if (rocblas_create_handle(&c->rb) != rocblas_status_success)
    return fail(c, CTM_E_DEVICE, "rocblas_create_handle failed");
  rocblas_set_stream(c->rb, c->st);
  return 0;
}

// Full-SVD projectors (Standard CTMRG section) for environment dimension x.
int full_projectors(ctm_ctx* c, int keep) {
  const int N1 = c->chi_env * c->Dl;
  const DT cp = c->cp;
  TRY(ensure_rocblas(c));
  // P_i = Ct_i Ct_(i+1) in S1[i]
  {
    GemmBatch g = gemm_rowmajor(4, N1, N1, N1, N1, N1, N1);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = c->Ct[i];
      g.B[i] = c->Ct[(i + 1) % 4];
      g.C[i] = c->S1[i];
    }
    TRY(run_gemm(c, PC_FULLSVD, g, cp, cp, DT::F64));
  }
  for (int b = 0; b < 4; ++b) {
    const double* L = c->S1[md(b - 1)];
    const double* R = c->S1[md(b + 1)];
    double* M = c->S2[0];
    double* Ut = c->S2[1];   // receives V^T of M (row-major)
    double* Uv = c->S2[2];   // receives U of M (row-major)
    {
      GemmBatch g = gemm_rowmajor(1, N1, N1, N1, N1, N1, N1);
      g.A[0] = L;
      g.B[0] = R;
      g.C[0] = M;
      TRY(run_gemm(c, PC_FULLSVD, g, DT::F64, DT::F64, DT::F64));
    }
    {
      ProfScope ps(c, PC_FULLSVD);
      // rocSOLVER is column-major: it sees M^T = (V) S (U^T)
      // gesvdx computes only the leading min(N1, keep + 1) triples (bisection and
      // inverse iteration on the bidiagonal); its right vectors of M^T are
      // stored with leading dimension N1, the same layout as the others'
      rocblas_status st;
      if (c->cfg.svd_driver == 1)
        st = rocsolver_dgesdd(c->rb, rocblas_svect_singular, rocblas_svect_singular, N1, N1, M, N1,
                              c->fs_s, Ut, N1, Uv, N1, c->fs_info);
      else if (c->cfg.svd_driver == 2)
        st = rocsolver_dgesvdx(c->rb, rocblas_svect_singular, rocblas_svect_singular,
                               rocblas_srange_index, N1, N1, M, N1, 0.0, 0.0, 1,
                               std::min(N1, keep + 1), c->fs_info + 1, c->fs_s, Ut, N1, Uv, N1,
                               c->fs_perm, c->fs_info);
      else
        st = rocsolver_dgesvd(c->rb, rocblas_svect_singular, rocblas_svect_singular, N1, N1, M, N1,
                              c->fs_s, Ut, N1, Uv, N1, c->fs_E, rocblas_outofplace, c->fs_info);
      if (st != rocblas_status_success)
        return fail(c, CTM_E_DEVICE, "rocSOLVER SVD failed: " + std::to_string((int)st));
    }
    // keep the triples in descending order of the singular value: the
    // divide-and-conquer driver does not return them ordered at every size
    // (a no-op permutation for the QR-iteration driver); U into M's buffer,
    // V^T into S2[3], the values into fs_E
    {
      const int m = std::min(N1, keep + 1);
      TRY(elem_sort_triples(c->fs_s, Uv, Ut, N1, m, c->fs_perm, c->fs_E, M, c->S2[3], c->st));
      Uv = M;
      Ut = c->S2[3];
    }
    SignArgs sa{};
    sa.N = N1;
    sa.k = keep;
    sa.ld = N1;
    sa.Y[0] = Uv;
    sa.sg[0] = c->fs_sg;
    TRY(elem_col_sign(sa, 1, c->st));
    TRY(elem_proj_prep_full(Uv, Ut, c->fs_E, c->fs_sg, N1, keep, c->cfg.pinv_rtol, c->fs_Us,
                            c->fs_Vs, c->scal + 9 + b, c->st));
    // P_l = R Vs ; P_r^T = L^T Us
    GemmBatch g = gemm_rowmajor(2, N1, keep, N1, N1, keep, keep);
    g.A[0] = R;
    g.B[0] = c->fs_Vs;
    g.C[0] = c->Pl[b];
    g.A[1] = L;
    g.transA[1] = 1;
    g.B[1] = c->fs_Us;
    g.C[1] = c->Prt[b];
    TRY(run_gemm(c, PC_FULLSVD, g, DT::F64, DT::F64, DT::F64));
  }
  return 0;
}

// Step 3: C_i' = P_r^(i-1) Ct_i P_l^(i);  T_j' = P_r^(j) (T_j a) P_l^(j).
int renormalize_corners(ctm_ctx* c, int keep) {
  const int x = c->chi_env, Dl = c->Dl, N1 = x * Dl, xp = keep;
  const int nxt = 1 - c->cur;
  {
    GemmBatch g = gemm_rowmajor(4, N1, xp, N1, N1, xp, xp);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = c->Ct[i];
      g.B[i] = c->Pl[i];
      g.C[i] = c->Zc[i];
    }
    TRY(run_gemm(c, PC_RENORM, g, c->cp, DT::F64, DT::F64));
  }
  {
    GemmBatch g = gemm_rowmajor(4, xp, xp, N1, xp, xp, xp);
    for (int i = 0; i < 4; ++i) {
      g.A[i] = c->Prt[md(i - 1)];
      g.transA[i] = 1;
      g.B[i] = c->Zc[i];
      g.C[i] = c->C[nxt][i];
    }
    TRY(run_gemm(c, PC_RENORM, g, DT::F64, DT::F64, DT::F64));
  }
  return 0;
}

int renormalize_edges(ctm_ctx* c, int keep) {
  const int x = c->chi_env, Dl = c->Dl, xp = keep;
  const int nxt = 1 - c->cur;
  double* const* T = c->T[c->cur];
  // Z1[(b, g'), (r, u)] = sum_g T_j[(b, u), g] P_l[(g, r), g'], one product
  // per edge with columns (r, g') (P_l read as a x by Dl xp matrix), so that
  // it has the wide shape of the corner stems.  u, the row leg, is Z1's
  // unit-stride leg, so that the rows of a tile are stored contiguously; the
  // next product contracts (r, u) against the site tensor.
  {
    GemmBatch g = gemm_rowmajor(4, x * Dl, Dl * xp, x, x, (long)Dl * xp, 0);
    g.cdiv_m = Dl;
    g.cs_m1 = (long)xp * Dl * Dl;
    g.cs_m0 = 1;
    g.cdiv_n = xp;
    g.cs_n1 = Dl;
    g.cs_n0 = (long)Dl * Dl;
    for (int j = 0; j < 4; ++j) {
      g.A[j] = T[j];
      g.B[j] = c->Pl[j];
      g.C[j] = c->S1[j];
    }
    TRY(run_gemm(c, PC_RENORM, g, DT::F64, DT::F64, DT::F64));
  }
  // Z2[(b, l), g', d] = Z1[(b, g'), (r, u)] apr_(j+1)[(r, u), (l, d)], through
  // the single-layer tensor where it applies (as the corners' absorption); d
  // is Z2's unit-stride leg, so that each (b, g') row block is written in
  // runs of D^2
  if ((c->cp == DT::F64 || (c->cp == DT::F32 && !c->split)) && c->d > 0 &&
      absorb_corner_fits(c->D, c->d)) {
    const long Dd = c->D, su = Dd * Dd * Dd, sl = Dd * Dd, sd = Dd, sr = 1;
    const long cl[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
    struct Ptrs { const double* W[4]; void* out[4]; long legs[4][4]; long ostr[4]; } pp;
    for (int j = 0; j < 4; ++j) {
      const int i = (j + 1) % 4;
      pp.legs[j][0] = cl[i][1];
      pp.legs[j][1] = cl[i][0];
      pp.legs[j][2] = cl[i][2];
      pp.legs[j][3] = cl[i][3];
      pp.W[j] = c->S1[j];
      pp.out[j] = c->S2[j];
    }
    pp.ostr[0] = (long)Dl * Dl * xp;
    pp.ostr[1] = Dl;
    pp.ostr[2] = (long)Dl * xp;
    pp.ostr[3] = 1;
    const long nR = (long)x * xp;
    const double* A = c->A_site;
    const int Di = c->D, d = c->d;
    if (c->rec) {
      c->rec->push_back(BatchOp{false, GemmBatch{}, [=](hipStream_t st) {
                                  const double* As[4] = {A, A, A, A};
                                  return launch_absorb(4, pp.W, pp.out, false, As, pp.legs, nR, xp,
                                                       pp.ostr, Di, d, st);
                                }});
    } else {
      ProfScope ps(c, PC_RENORM, 4.0 * 4.0 * (double)nR * Dl * Dl * Dl * d);
      const double* As[4] = {A, A, A, A};
      if (launch_absorb(4, pp.W, pp.out, false, As, pp.legs, nR, xp, pp.ostr, Di, d, c->st))
        return fail(c, CTM_E_DEVICE, thread_error());
    }
  } else {
    GemmBatch g = gemm_rowmajor(4, x * xp, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
    g.cdiv_m = xp;
    g.cs_m1 = (long)Dl * Dl * xp;
    g.cs_m0 = Dl;
    g.cdiv_n = Dl;
    g.cs_n1 = (long)Dl * xp;
    g.cs_n0 = 1;
    for (int j = 0; j < 4; ++j) {
      g.A[j] = c->S1[j];
      g.B[j] = c->apr[(j + 1) % 4];
      g.C[j] = c->S2[j];
    }
    TRY(run_gemm(c, PC_RENORM, g, DT::F64, c->cp, DT::F64));
  }
  // T'[b', (d, g')] = sum_(b,l) P_r^T[(b, l), b'] Z2[(b, l), (g', d)]: one
  // GEMM per edge, computed as its transpose (rows (g', d), N = xp columns
  // b'), the tall-skinny shape of the split kernel; the output map writes it
  // back in T' order
  {
    GemmBatch g = gemm_rowmajor(4, Dl * xp, xp, x * Dl, (long)Dl * xp, xp, 0);
    set_map(g, Dl, 1, xp, 1 << 30, 0, (long)Dl * xp);
    for (int j = 0; j < 4; ++j) {
      g.A[j] = c->S2[j];
      g.transA[j] = 1;
      g.B[j] = c->Prt[j];
      g.C[j] = c->T[nxt][j];
    }
    TRY(run_gemm(c, PC_RENORM, g, DT::F64, DT::F64, DT::F64));
  }
  return 0;
}

// Normalises tensors first .. first+count-1 of buffer `buf` (0..3 the
// corners, 4..7 the edges; environment dimension x) and raises the device
// flag on a zero or non-finite norm.  Each tensor has its own partial sums
// and norm slot, so the corners and the edges can be normalised on two
// streams at once with the same results.
int normalize_env(ctm_ctx* c, int buf, int x, int first = 0, int count = 8) {
  NormArgs na{};
  for (int t = 0; t < count; ++t) {
    const int i = first + t;
    na.x[t] = i < 4 ? c->C[buf][i] : c->T[buf][i - 4];
    na.n[t] = i < 4 ? (long)x * x : (long)x * c->Dl * x;
  }
  na.out = c->scal + first;
  na.bad = c->bad;
  na.part = c->dot_part + (long)first * kNormBlocks;
  static_assert(8 * kNormBlocks <= kMaxDots * kDotBlocks, "norm partial sums exceed dot_part");
  ENQ(elem_normalize(na, count, st));
  return 0;
}

// Corner spectra of buffer `buf` and delta against the committed spectra.
int spectra(ctm_ctx* c, int buf, int x) {
  {
    ProfScope ps(c, PC_SVD);
    const double* A[4] = {c->C[buf][0], c->C[buf][1], c->C[buf][2], c->C[buf][3]};
    ENQ(launch_svd(4, A, nullptr, c->csv, nullptr, x, c->svd_ws, st));
  }
  SpecArgs sp{};
  for (int i = 0; i < 4; ++i) sp.s[i] = c->csv[i];
  sp.old_spec = c->spec[c->spec_cur];
  sp.new_spec = c->spec[1 - c->spec_cur];
  sp.delta = c->scal + 8;
  sp.x = std::min(x, c->chi);
  sp.chi = c->chi;
  ENQ(elem_spectra_delta(sp, st));
  return 0;
}

// ---------------------------------------------------------------------------
// C4v moves (a single symmetric corner C and edge T; the QR-based projector
// section specialised to the symmetric case, which the paper inherits from
// the C4v QR-CTMRG): the enlarged corner Ct is symmetric and the projector is
// an isometry P, the same for every bond.
//  - growth: P = I;  full: P = eigenvectors of the chi largest |lambda| of Ct
//    (rocSOLVER dsyevd), sign rule on the columns of P;
//  - SI: X <- QR(Ct X) n_si times, rho = X^T Ct X, its eigenvectors v (from the
//    Jacobi SVD of the symmetric rho: v_i with s_i = |lambda_i|), sign rule on
//    the columns of X v, X <- X v, P = X[:, :chi].
// The move then runs the four-direction renormalisation with P on every bond,
// symmetrises C' and T' of the first corner and edge and copies them to the
// other three.
// ---------------------------------------------------------------------------
int c4v_projectors(ctm_ctx* c, int mode, int keep) {
  const int N1 = c->chi_env * c->Dl, k = c->k;
  double* Ct0 = (double*)c->Ct[0];
  TRY(elem_symmetrize(Ct0, N1, c->st));
  double* P = c->Pl[0];
  if (mode == 0) {
    TRY(elem_identity(P, N1, N1, c->st));
  } else if (mode == 1) {
    TRY(ensure_rocblas(c));
    CTM_HIP_TRY(hipMemcpyAsync(c->S2[0], Ct0, (size_t)N1 * N1 * 8, hipMemcpyDeviceToDevice, c->st));
    {
      ProfScope ps(c, PC_FULLSVD);
      // column-major view of a symmetric matrix: the same matrix
      const rocblas_status st = rocsolver_dsyevd(c->rb, rocblas_evect_original, rocblas_fill_upper,
                                                 N1, c->S2[0], N1, c->fs_s, c->fs_E, c->fs_info);
      if (st != rocblas_status_success)
        return fail(c, CTM_E_DEVICE, "rocsolver_dsyevd failed: " + std::to_string((int)st));
    }
    TRY(elem_c4v_order(c->fs_s, c->S2[0], N1, keep, P, c->st));
    SignArgs sa{};
    sa.N = N1;
    sa.k = keep;
    sa.ld = keep;
    sa.Y[0] = P;
    sa.sg[0] = c->fs_sg;
    TRY(elem_col_sign(sa, 1, c->st));
    TRY(elem_scale_cols(sa, 1, c->st));
  } else {
    TRY(ensure_si_blocks(c));
    auto apply = [&](const double* in, double* out) {
      GemmBatch g = gemm_rowmajor(1, N1, k, N1, N1, k, k);
      g.A[0] = Ct0;
      g.B[0] = in;
      g.C[0] = out;
      const int chk = check_gemm(c, g, DT::F64, DT::F64, DT::F64);
      if (chk) return chk;
      ProfScope ps(c, PC_SI_APPLY, gemm_flops(g), (double)N1 * N1 * 8 + 2.0 * N1 * k * 8);
      return launch_gemm_si_balanced(g, c->sk_part, c->sk_cus, c->st);
    };
    for (int step = 0; step < c->cfg.n_si; ++step) {
      TRY(apply(c->X[0], c->W[0][0]));
      {
        ProfScope ps(c, PC_QR, 4.0 * N1 * (double)k * k);
        TRY(launch_qr(1, &c->W[0][0], N1, k, c->qr_ws, c->st));
      }
      std::swap(c->X[0], c->W[0][0]);
    }
    TRY(apply(c->X[0], c->W[0][0]));
    {
      GemmBatch g = gemm_rowmajor(1, k, k, N1, k, k, k);   // rho = X^T (Ct X)
      g.A[0] = c->X[0];
      g.transA[0] = 1;
      g.B[0] = c->W[0][0];
      g.C[0] = c->rho[0];
      TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
    }
    TRY(elem_symmetrize(c->rho[0], k, c->st));
    {
      ProfScope ps(c, PC_SVD);
      TRY(launch_svd(1, &c->rho[0], &c->u[0], &c->s[0], &c->v[0], k, c->svd_ws, c->st));
    }
    {
      GemmBatch g = gemm_rowmajor(1, N1, k, k, k, k, k);   // X v
      g.A[0] = c->X[0];
      g.B[0] = c->v[0];
      g.C[0] = c->W[0][0];
      TRY(run_gemm(c, PC_PROJ, g, DT::F64, DT::F64, DT::F64));
    }
    SignArgs sa{};
    sa.N = N1;
    sa.k = k;
    sa.ld = k;
    sa.Y[0] = c->W[0][0];
    sa.sg[0] = c->sg[0];
    TRY(elem_col_sign(sa, 1, c->st));
    TRY(elem_scale_cols(sa, 1, c->st));
    std::swap(c->X[0], c->W[0][0]);
    TRY(elem_copy_cols(c->X[0], N1, k, keep, P, c->st));
  }
  const size_t pb = (size_t)N1 * keep * 8;
  for (int b = 0; b < 4; ++b) {
    if (b) CTM_HIP_TRY(hipMemcpyAsync(c->Pl[b], P, pb, hipMemcpyDeviceToDevice, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(c->Prt[b], P, pb, hipMemcpyDeviceToDevice, c->st));
  }
  return 0;
}

// C' and T' of the first corner and edge, symmetrised, become all four.
int c4v_finish(ctm_ctx* c, int gen, int keep) {
  const int Dl = c->Dl;
  TRY(elem_symmetrize(c->C[gen][0], keep, c->st));
  TRY(elem_symmetrize_edge(c->T[gen][0], keep, Dl, c->st));
  for (int i = 1; i < 4; ++i) {
    CTM_HIP_TRY(hipMemcpyAsync(c->C[gen][i], c->C[gen][0], (size_t)keep * keep * 8,
                               hipMemcpyDeviceToDevice, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(c->T[gen][i], c->T[gen][0], (size_t)keep * Dl * keep * 8,
                               hipMemcpyDeviceToDevice, c->st));
  }
  return 0;
}

std::vector<void*> block_ptrs(const ctm_ctx* c) {
  std::vector<void*> v;
  for (int b = 0; b < 4; ++b) {
    v.push_back(c->X[b]);
    v.push_back(c->Yt[b]);
  }
  for (int s2 = 0; s2 < 2; ++s2)
    for (int i = 0; i < 8; ++i) v.push_back(c->W[s2][i]);
  return v;
}

void set_block_ptrs(ctm_ctx* c, const std::vector<void*>& v) {
  size_t o = 0;
  for (int b = 0; b < 4; ++b) {
    c->X[b] = (double*)v[o++];
    c->Yt[b] = (double*)v[o++];
  }
  for (int s2 = 0; s2 < 2; ++s2)
    for (int i = 0; i < 8; ++i) c->W[s2][i] = (double*)v[o++];
}

void drop_graphs(ctm_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

// Device work of a move (everything between the guard reset and the
// read-back of its scalars).
int move_work(ctm_ctx* c, int mode, int keep, int nsi, bool measure) {
  const int N1 = c->chi_env * c->Dl;
  ENQ(elem_zero_int(c->bad, st));
  TRY(build_corners(c));
  if (c->cfg.sym == CTM_SYM_C4V) {
    TRY(c4v_projectors(c, mode, keep));
  } else if (mode == 0) {
    for (int b = 0; b < 4; ++b) {
      TRY(elem_identity(c->Pl[b], N1, N1, c->st));
      TRY(elem_identity(c->Prt[b], N1, N1, c->st));
    }
  } else if (mode == 1) {
    TRY(full_projectors(c, keep));
  } else if (mode == 3) {
    TRY(growth_si_projectors(c, keep, N1));
  } else {
    TRY(si_projectors(c, keep, nsi, measure));
  }
  const int nxt = 1 - c->cur;
  if (c->cfg.sym == CTM_SYM_C4V || c->rec || c->use_graphs) {
    TRY(renormalize_corners(c, keep));
    TRY(renormalize_edges(c, keep));
    if (c->cfg.sym == CTM_SYM_C4V) TRY(c4v_finish(c, nxt, keep));
    TRY(normalize_env(c, nxt, keep));
    TRY(spectra(c, nxt, keep));
    return 0;
  }
  // the new corners' norms and spectra (the convergence measure) on the side
  // stream while the edges are renormalised: the same operations on the same
  // data, in a different schedule
  TRY(renormalize_corners(c, keep));
  if (!c->side) {
    if ((!c->ev_fork &&
         hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) ||
        (!c->ev_join &&
         hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
      c->side = nullptr;
      (void)hipGetLastError();
      return fail(c, CTM_E_DEVICE, "creation of the second stream or its events failed");
    }
  }
  CTM_HIP_TRY(hipEventRecord(c->ev_fork, c->st));
  CTM_HIP_TRY(hipStreamWaitEvent(c->side, c->ev_fork, 0));
  {
    hipStream_t main = c->st;
    c->st = c->side;
    int r = normalize_env(c, nxt, keep, 0, 4);
    if (!r) r = spectra(c, nxt, keep);
    c->st = main;
    if (r) return r;
  }
  TRY(renormalize_edges(c, keep));
  TRY(normalize_env(c, nxt, keep, 4, 4));
  CTM_HIP_TRY(hipEventRecord(c->ev_join, c->side));
  CTM_HIP_TRY(hipStreamWaitEvent(c->st, c->ev_join, 0));
  return 0;
}

// SI moves through a captured graph (one per (cur, pointer arrangement)).
int move_work_graph(ctm_ctx* c, int mode, int keep, int nsi, bool measure) {
  TRY(ensure_si_blocks(c));   // may copy the start blocks: outside the graph
  const std::vector<void*> pre = block_ptrs(c);
  for (auto& g : c->graphs) {
    if (g.cur == c->cur && g.spec_cur == c->spec_cur && g.nsi == nsi && g.measure == measure &&
        g.pre == pre) {
      set_block_ptrs(c, g.post);
      CTM_HIP_TRY(hipGraphLaunch(g.exec, c->st));
      return 0;
    }
  }
  CTM_HIP_TRY(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  const int rc = move_work(c, mode, keep, nsi, measure);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->st, &graph);
  if (rc || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_block_ptrs(c, pre);
    return rc ? rc : fail(c, CTM_E_DEVICE, "stream capture of the move failed");
  }
  ctm_ctx::GraphRec g;
  g.cur = c->cur;
  g.spec_cur = c->spec_cur;
  g.nsi = nsi;
  g.measure = measure;
  g.pre = pre;
  g.post = block_ptrs(c);
  const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    set_block_ptrs(c, pre);
    return fail(c, CTM_E_DEVICE, "graph instantiation failed");
  }
  c->graphs.push_back(g);
  CTM_HIP_TRY(hipGraphLaunch(g.exec, c->st));
  return 0;
}

// Enqueues one move on the context's stream; its scalar results (norms,
// delta, gaps, the numeric-guard flag) are copied to pinned host memory and
// done_ev is recorded behind them.  The environment buffers of the next
// generation are written; the context switches to them in finish_move.
int enqueue_move(ctm_ctx* c) {
  if (c->pending) return fail(c, CTM_E_STATE, "a move is already in flight");
  const int x = c->chi_env, N1 = x * c->Dl;
  int mode, keep;
  if (N1 <= c->chi) {
    mode = 0;
    keep = N1;
  } else if (x != c->chi || c->cfg.proj == CTM_PROJ_FULLSVD) {
    // truncating growth: randomized (SI) projectors on request, when the
    // N1 rows hold a k-column block with a QR leaf split; else full SVD
    const bool rnd = c->cfg.growth == 1 && c->cfg.proj == CTM_PROJ_SI &&
                     c->cfg.sym == CTM_SYM_NONE && x < c->chi && N1 >= c->k &&
                     qr_plan_ok(N1, c->k);
    mode = rnd ? 3 : 1;
    keep = c->chi;
  } else {
    mode = 2;
    keep = c->chi;
  }
  // growth and full-SVD moves call rocSOLVER and run eagerly; SI moves are
  // captured when graphs are enabled on a non-default stream
  // recycling: no subspace step while `recycling`; the criterion is measured
  // on moves with steps whose previous move was an SI move
  const bool rec = c->cfg.recycle_sin2 > 0;
  int nsi = 0;
  bool measure = false;
  if (mode == 2 && c->cfg.sym != CTM_SYM_C4V) {
    nsi = (rec && c->recycling) ? 0 : c->cfg.n_si;
    measure = rec && nsi > 0 && c->last_si_delta >= 0.0 && !c->iso_pending;
  } else if (mode == 2) {
    nsi = c->cfg.n_si;
  }
  if (mode == 2 && c->use_graphs && !c->prof && c->st != nullptr)
    TRY(move_work_graph(c, mode, keep, nsi, measure));
  else
    TRY(move_work(c, mode, keep, nsi, measure));
  CTM_HIP_TRY(hipMemcpyAsync(c->hbuf, c->scal, 16 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  CTM_HIP_TRY(hipMemcpyAsync(c->hbuf + 16, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->st));
  CTM_HIP_TRY(hipEventRecord(c->done_ev, c->st));
  c->pending = true;
  c->pend_mode = mode;
  c->pend_keep = keep;
  c->pend_nsi = nsi;
  c->pend_measure = measure;
  return CTM_OK;
}

// Completes the move in flight (done_ev has fired): checks the numeric guard
// and switches to the new environment generation.
int finish_move(ctm_ctx* c, ctm_move_info* info) {
  c->pending = false;
  const double* host = c->hbuf;
  int bad = 0;
  std::memcpy(&bad, c->hbuf + 16, sizeof(int));
  if (bad || !std::isfinite(host[8]))
    return fail(c, CTM_E_NUMERIC, "move produced a zero or non-finite norm; environment kept");
  const int mode = c->pend_mode, keep = c->pend_keep;
  if (mode == 2) ++c->si_moves;
  const double sin2 = c->pend_measure ? host[13] : -1.0;
  if (c->cfg.recycle_sin2 > 0 && mode == 2) {
    if (c->pend_nsi > 0) {
      ++c->si_upd;
      if (c->pend_measure && c->si_upd >= c->cfg.min_si_moves && sin2 < c->cfg.recycle_sin2)
        c->recycling = true;
    } else if (c->last_si_delta >= 0.0 && host[8] > kRecycleGuard * c->last_si_delta) {
      c->recycling = false;
      c->si_upd = 0;
    }
  }
  c->last_si_delta = mode == 2 ? host[8] : -1.0;
  c->cur = 1 - c->cur;
  c->chi_env = keep;
  c->spec_cur = 1 - c->spec_cur;
  ++c->moves;
  if (info) {
    info->delta = host[8];
    info->mode = mode;
    info->chi_env = keep;
    double gap = -1.0;
    if (mode != 0 && c->cfg.sym != CTM_SYM_C4V) {
      gap = 1e300;
      for (int b = 0; b < 4; ++b) gap = std::min(gap, host[9 + b]);
    }
    info->gap = gap;
    info->n_si = c->pend_nsi;
    info->sin2 = sin2;
  }
  return CTM_OK;
}

int wait_move(ctm_ctx* c, ctm_move_info* info) {
  CTM_HIP_TRY(hipEventSynchronize(c->done_ev));
  return finish_move(c, info);
}

int do_move(ctm_ctx* c, ctm_move_info* info) {
  TRY(enqueue_move(c));
  return wait_move(c, info);
}

// Completes a move still in flight before a call that reads or replaces the
// environment.
int drain(ctm_ctx* c) {
  if (!c->pending) return CTM_OK;
  return wait_move(c, nullptr);
}

// ---------------------------------------------------------------------------
// Batched moves (serving: environment solves of mixed (D, chi) moved
// together).  Each context's SI move is recorded as its sequence of
// operations; step i of every context is then launched together on one
// stream: the float64 GEMMs of the step as one persistent grouped launch
// over a device table of (descriptor, tile) work items, the other operations
// one after another.  Contexts are independent, so only each context's own
// order matters, and every product gets the bits of the solo move (the tile
// kernels do not depend on the grid; the split SI kernel, whose summation
// order does, keeps its own launch).
// ---------------------------------------------------------------------------
constexpr int kBatchMaxDevices = 64;

struct BatchTable {
  GroupItem* dev = nullptr;    // device copy of the descriptors
  GroupItem* host = nullptr;   // pinned staging of the descriptors
  size_t cap = 0;              // items both hold
  hipEvent_t done = nullptr;   // recorded after the last batch that read them
};
std::mutex g_batch_mu;
BatchTable g_batch[kBatchMaxDevices];

// True if the next move of c is an SI move that a batch records.
bool batchable(const ctm_ctx* c) {
  return !c->pending && c->chi_env == c->chi && c->chi * c->Dl > c->chi &&
         c->cfg.proj == CTM_PROJ_SI && c->cfg.sym == CTM_SYM_NONE && c->cp == DT::F64;
}

int enqueue_batch(ctm_ctx* const* ctxs, int n) {
  std::vector<ctm_ctx*> grp;
  for (int i = 0; i < n; ++i) {
    ctm_ctx* c = ctxs[i];
    if (!c) return fail(nullptr, CTM_E_ARG, "null context in the batch");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(c, CTM_E_ARG, "a context appears twice in the batch");
    if (c->pending) return fail(c, CTM_E_STATE, "a move is already in flight");
  }
  for (int i = 0; i < n; ++i) {
    ctm_ctx* c = ctxs[i];
    c->err.clear();
    if (batchable(c) && !c->prof) grp.push_back(c);
    else TRY(enqueue_move(c));                      // growth, full-SVD, C4v, reduced precision
  }
  if (grp.empty()) return CTM_OK;
  hipStream_t S = grp[0]->st;
  // work already queued on a context's own stream precedes its batched move
  for (ctm_ctx* c : grp)
    if (c->st != S) CTM_HIP_TRY(hipStreamSynchronize(c->st));
  // record every context's move; the recording swaps block pointers on the
  // host, so a failure before the launch restores every arrangement
  std::vector<std::vector<BatchOp>> ops(grp.size());
  std::vector<std::vector<void*>> arrangement(grp.size());
  for (size_t i = 0; i < grp.size(); ++i) arrangement[i] = block_ptrs(grp[i]);
  auto restore = [&](int code) {
    for (size_t i = 0; i < grp.size(); ++i) set_block_ptrs(grp[i], arrangement[i]);
    return code;
  };
  size_t steps = 0;
  for (size_t i = 0; i < grp.size(); ++i) {
    ctm_ctx* c = grp[i];
    hipStream_t own = c->st;
    c->st = S;                                      // eager parts below run on S
    const bool rec = c->cfg.recycle_sin2 > 0;
    const int nsi = (rec && c->recycling) ? 0 : c->cfg.n_si;
    const bool measure = rec && nsi > 0 && c->last_si_delta >= 0.0 && !c->iso_pending;
    int r = ensure_si_blocks(c);
    if (!r) {
      c->rec = &ops[i];
      r = move_work(c, 2, c->chi, nsi, measure);
      c->rec = nullptr;
    }
    c->st = own;
    if (r) return restore(r);
    c->pend_mode = 2;
    c->pend_keep = c->chi;
    c->pend_nsi = nsi;
    c->pend_measure = measure;
    steps = std::max(steps, ops[i].size());
  }
  // the grouped GEMMs of every step, in one table
  std::vector<GemmBatch> gs;
  std::vector<std::pair<size_t, int>> span(steps);   // (first item, items) per step
  std::vector<std::pair<long, int>> plan(steps);     // (work items, kind) per step
  for (size_t t = 0; t < steps; ++t) {
    span[t] = {gs.size(), 0};
    for (auto& v : ops)
      if (t < v.size() && v[t].gemm) gs.push_back(v[t].g);
    span[t].second = (int)(gs.size() - span[t].first);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kBatchMaxDevices)
    return restore(fail(nullptr, CTM_E_DEVICE, "no usable current device"));
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchTable& tb = g_batch[dev];
  if (!tb.done && hipEventCreateWithFlags(&tb.done, hipEventDisableTiming) != hipSuccess)
    return restore(fail(nullptr, CTM_E_DEVICE, "event creation failed"));
  // the previous batch has read the table before it is rewritten
  if (hipEventSynchronize(tb.done) != hipSuccess)
    return restore(fail(nullptr, CTM_E_DEVICE, "synchronisation failed"));
  if (gs.size() > tb.cap) {
    if (tb.dev) (void)hipFree(tb.dev);
    if (tb.host) (void)hipHostFree(tb.host);
    tb.dev = nullptr;
    tb.host = nullptr;
    tb.cap = 0;
    const size_t cap = std::max<size_t>(2 * gs.size(), 256);
    if (hipMalloc((void**)&tb.dev, cap * sizeof(GroupItem)) != hipSuccess ||
        hipHostMalloc((void**)&tb.host, cap * sizeof(GroupItem), hipHostMallocDefault) != hipSuccess)
      return restore(fail(nullptr, CTM_E_NOMEM, "descriptor table of the batched move"));
    tb.cap = cap;
  }
  for (size_t t = 0; t < steps; ++t) {
    const int cnt = span[t].second;
    if (!cnt) continue;
    const GemmBatch* g = gs.data() + span[t].first;
    const int kind = grouped_kind(g, cnt);
    plan[t] = {grouped_fill(g, cnt, kind, tb.host + span[t].first), kind};
  }
  if (!gs.empty())
    CTM_HIP_TRY(hipMemcpyAsync(tb.dev, tb.host, gs.size() * sizeof(GroupItem),
                               hipMemcpyHostToDevice, S));
  for (size_t t = 0; t < steps; ++t) {
    if (span[t].second)
      TRY_B(launch_gemm_grouped(tb.dev + span[t].first, span[t].second, plan[t].first,
                                plan[t].second, S));
    for (size_t i = 0; i < grp.size(); ++i)
      if (t < ops[i].size() && !ops[i][t].gemm) {
        const int r = ops[i][t].fn(S);
        if (r) return fail(grp[i], r == 1 ? CTM_E_ARG : r, g_err.empty() ? "batched launch" : g_err);
      }
  }
  CTM_HIP_TRY(hipEventRecord(tb.done, S));
  for (ctm_ctx* c : grp) {
    CTM_HIP_TRY(hipMemcpyAsync(c->hbuf, c->scal, 16 * sizeof(double), hipMemcpyDeviceToHost, S));
    CTM_HIP_TRY(hipMemcpyAsync(c->hbuf + 16, c->bad, sizeof(int), hipMemcpyDeviceToHost, S));
    CTM_HIP_TRY(hipEventRecord(c->done_ev, S));
    c->pending = true;
  }
  return CTM_OK;
}


// ---------------------------------------------------------------------------
// observables (iPEPS section: norm network and operator insertion)
// ---------------------------------------------------------------------------
GemmBatch gb1(int M, int N, int K, const void* A, long lda, int transA, const void* B, long ldb,
              void* C, long ldc) {
  GemmBatch g = gemm_rowmajor(1, M, N, K, lda, ldb, ldc);
  g.A[0] = A;
  g.transA[0] = transA;
  g.B[0] = B;
  g.C[0] = C;
  return g;
}

int g64(ctm_ctx* c, const GemmBatch& g) { return run_gemm(c, PC_MISC, g, DT::F64, DT::F64, DT::F64); }

// Permuted f64 copy of a rank-4 site tensor for absorption slot `slot`
// (0: K=(l,u) N=(d,r); 1: K=(u,r) N=(l,d); 2: K=(r,d) N=(u,l)).
int perm_site(ctm_ctx* c, const double* src, double* dst, int slot) {
  const long Dl = c->Dl;
  const long su = Dl * Dl * Dl, sl = Dl * Dl, sd = Dl, sr = 1;
  const long perm[3][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}};
  return elem_permute4(src, dst, DT::F64, (int)Dl, perm[slot][0], perm[slot][1], perm[slot][2],
                       perm[slot][3], c->st);
}

// Z11 with the site tensor xp (slot-0 permuted, f64) into *out.
int z11(ctm_ctx* c, const double* xp, double* out) {
  const int x = c->chi_env, Dl = c->Dl;
  double* const* C = c->C[c->cur];
  double* const* T = c->T[c->cur];
  TRY(g64(c, gb1(x, Dl * x, x, C[0], x, 0, T[0], (long)Dl * x, c->CT[0], (long)Dl * x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[0], x, 0, C[1], x, c->CT[1], x)));          // top[(a,u),h]
  GemmBatch g = gb1(x * Dl, Dl * x, x, T[3], x, 0, c->CT[1], (long)Dl * x, c->S1[0], 0);
  set_map(g, Dl, (long)x * Dl * Dl, Dl, x, 1, (long)Dl * Dl);                        // x1[(t,h),(l,u)]
  TRY(g64(c, g));
  g = gb1(x * x, Dl * Dl, Dl * Dl, c->S1[0], (long)Dl * Dl, 0, xp, (long)Dl * Dl, c->S2[0], 0);
  set_map(g, x, (long)Dl * Dl * x, Dl, Dl, (long)x * Dl, 1);                         // y[(t,d),(h,r)]
  TRY(g64(c, g));
  TRY(g64(c, gb1(x * Dl, x, x * Dl, c->S2[0], (long)x * Dl, 0, T[1], x, c->CT[2], x)));  // z[(t,d),e]
  TRY(g64(c, gb1(x, Dl * x, x, C[2], x, 0, T[2], (long)Dl * x, c->CT[3], (long)Dl * x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[3], x, 0, C[3], x, c->Zc[0], x)));              // bot[(e,d),t]
  return elem_dot_rev(c->CT[2], c->Zc[0], x, Dl, out, c->st);
}

// Z00, Z10, Z01 into out[0..2].
int z_rest(ctm_ctx* c, double* out) {
  const int x = c->chi_env, Dl = c->Dl;
  double* const* C = c->C[c->cur];
  double* const* T = c->T[c->cur];
  TRY(g64(c, gb1(x, x, x, C[0], x, 0, C[1], x, c->Zc[1], x)));
  TRY(g64(c, gb1(x, x, x, c->Zc[1], x, 0, C[2], x, c->Zc[2], x)));
  TRY(g64(c, gb1(x, x, x, c->Zc[2], x, 0, C[3], x, c->Zc[3], x)));
  TRY(elem_trace(c->Zc[3], x, out, c->st));
  // Z10: top[(a,u),h] C3[h,z] . T3[(z,u),n] C4[n,a]
  TRY(g64(c, gb1(x, Dl * x, x, C[0], x, 0, T[0], (long)Dl * x, c->CT[0], (long)Dl * x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[0], x, 0, C[1], x, c->CT[1], x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[1], x, 0, C[2], x, c->Zc[1], x)));
  TRY(g64(c, gb1(x * Dl, x, x, T[2], x, 0, C[3], x, c->Zc[2], x)));
  TRY(elem_dot_rev(c->Zc[1], c->Zc[2], x, Dl, out + 1, c->st));
  // Z01: C1[a,b] (C2 T2 C3)[b,(r,z)] . (C4 T4)[z,(r,a)]
  TRY(g64(c, gb1(x, Dl * x, x, C[1], x, 0, T[1], (long)Dl * x, c->CT[0], (long)Dl * x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[0], x, 0, C[2], x, c->CT[1], x)));
  TRY(g64(c, gb1(x, Dl * x, x, C[3], x, 0, T[3], (long)Dl * x, c->CT[2], (long)Dl * x)));
  TRY(g64(c, gb1(x, Dl * x, x, C[0], x, 0, c->CT[1], (long)Dl * x, c->CT[3], (long)Dl * x)));
  return elem_dot_rev(c->CT[3], c->CT[2], x, Dl, out + 2, c->st);
}

// Two-site network values E[i*n2 + j] for site-1 tensors s1[i] (slot 0 layout)
// and site-2 tensors s2[j] (slot 1 layout for horizontal, slot 2 for vertical).
int two_site(ctm_ctx* c, bool horizontal, const double* const* s1, int n1,
             const double* const* s2, int n2, double* E) {
  const int x = c->chi_env, Dl = c->Dl;
  const long L = (long)x * Dl * x;
  double* const* C = c->C[c->cur];
  double* const* T = c->T[c->cur];
  if (horizontal) {
    // left'[(j,l),b] = C4[j,k] T4[k,(l,a)] C1[a,b]
    TRY(g64(c, gb1(x, Dl * x, x, C[3], x, 0, T[3], (long)Dl * x, c->CT[0], (long)Dl * x)));
    TRY(g64(c, gb1(x * Dl, x, x, c->CT[0], x, 0, C[0], x, c->CT[1], x)));
    GemmBatch g = gb1(x * Dl, Dl * x, x, c->CT[1], x, 0, T[0], (long)Dl * x, c->S1[0], 0);
    set_map(g, Dl, (long)x * Dl * Dl, Dl, x, 1, (long)Dl * Dl);                    // y1'[(j,g),(l,u)]
    TRY(g64(c, g));
    for (int i = 0; i < n1; ++i) {
      g = gb1(x * x, Dl * Dl, Dl * Dl, c->S1[0], (long)Dl * Dl, 0, s1[i], (long)Dl * Dl, c->S2[0], 0);
      set_map(g, x, (long)x * Dl, Dl, Dl, (long)x * x * Dl, 1);                    // y2[(d,j),(g,m)]
      TRY(g64(c, g));
      g = gb1(x, x * Dl, x * Dl, T[2], (long)Dl * x, 0, c->S2[0], (long)x * Dl, c->obs_y + i * L, 0);
      set_map(g, 1 << 30, 0, 1, Dl, (long)Dl * x, x);                               // y3[g,m,i]
      TRY(g64(c, g));
    }
    // right[(h,w),f] = C2[h,c] T2[c,(w,e)] C3[e,f]
    TRY(g64(c, gb1(x, Dl * x, x, C[1], x, 0, T[1], (long)Dl * x, c->CT[2], (long)Dl * x)));
    TRY(g64(c, gb1(x * Dl, x, x, c->CT[2], x, 0, C[2], x, c->CT[3], x)));
    g = gb1(x * Dl, Dl * x, x, T[0], x, 0, c->CT[3], (long)Dl * x, c->S1[1], 0);
    set_map(g, Dl, (long)x * Dl * Dl, Dl, x, 1, (long)Dl * Dl);                    // w1'[(g,f),(v,w)]
    TRY(g64(c, g));
    for (int j = 0; j < n2; ++j) {
      g = gb1(x * x, Dl * Dl, Dl * Dl, c->S1[1], (long)Dl * Dl, 0, s2[j], (long)Dl * Dl, c->S2[1], 0);
      set_map(g, x, (long)Dl * Dl * x, Dl, Dl, (long)x * Dl, 1);                    // w2[(g,m),(f,y)]
      TRY(g64(c, g));
      TRY(g64(c, gb1(x * Dl, x, x * Dl, c->S2[1], (long)x * Dl, 0, T[2], x, c->obs_w + j * L, x)));
    }
    return elem_pair_dot(c->obs_y, c->obs_w, L, n1, n2, x, Dl, 0, E, c->st);
  }
  // vertical: top[(a,u),h]
  TRY(g64(c, gb1(x, Dl * x, x, C[0], x, 0, T[0], (long)Dl * x, c->CT[0], (long)Dl * x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[0], x, 0, C[1], x, c->CT[1], x)));
  GemmBatch g = gb1(x * Dl, Dl * x, x, T[3], x, 0, c->CT[1], (long)Dl * x, c->S1[0], 0);
  set_map(g, Dl, (long)x * Dl * Dl, Dl, x, 1, (long)Dl * Dl);                      // p1'[(n,h),(l,u)]
  TRY(g64(c, g));
  for (int i = 0; i < n1; ++i) {
    g = gb1(x * x, Dl * Dl, Dl * Dl, c->S1[0], (long)Dl * Dl, 0, s1[i], (long)Dl * Dl, c->S2[0], 0);
    set_map(g, x, (long)Dl * Dl * x, Dl, Dl, (long)x * Dl, 1);                      // p2[(n,x),(h,r)]
    TRY(g64(c, g));
    TRY(g64(c, gb1(x * Dl, x, x * Dl, c->S2[0], (long)x * Dl, 0, T[1], x, c->obs_y + i * L, x)));
  }
  // bot[(i,w),m] = C3[i,j] T3[j,(w,k)] C4[k,m]
  TRY(g64(c, gb1(x, Dl * x, x, C[2], x, 0, T[2], (long)Dl * x, c->CT[2], (long)Dl * x)));
  TRY(g64(c, gb1(x * Dl, x, x, c->CT[2], x, 0, C[3], x, c->CT[3], x)));
  g = gb1(x * Dl, Dl * x, x, T[1], x, 0, c->CT[3], (long)Dl * x, c->S1[1], 0);
  set_map(g, Dl, (long)x * Dl * Dl, Dl, x, 1, (long)Dl * Dl);                      // q1'[(c,m),(s,w)]
  TRY(g64(c, g));
  for (int j = 0; j < n2; ++j) {
    g = gb1(x * x, Dl * Dl, Dl * Dl, c->S1[1], (long)Dl * Dl, 0, s2[j], (long)Dl * Dl, c->S2[1], 0);
    set_map(g, x, (long)Dl * Dl * x, Dl, Dl, (long)x * Dl, 1);                      // q2[(c,x),(m,p)]
    TRY(g64(c, g));
    TRY(g64(c, gb1(x * Dl, x, x * Dl, c->S2[1], (long)x * Dl, 0, T[3], x, c->obs_w + j * L, x)));
  }
  return elem_pair_dot(c->obs_y, c->obs_w, L, n1, n2, x, Dl, 1, E, c->st);
}

// Enlarged corner i (float64, N x N, after corner_stems) with the rank-4
// site tensor xs (a-layout) in place of a; imp[1] holds its permutation.
int corner_with(ctm_ctx* c, int i, const double* xs, double* out) {
  const long Dl = c->Dl;
  const long su = Dl * Dl * Dl, sl = Dl * Dl, sd = Dl, sr = 1;
  const long perm[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
  TRY(elem_permute4(xs, c->imp[1], DT::F64, (int)Dl, perm[i][0], perm[i][1], perm[i][2], perm[i][3],
                    c->st));
  GemmBatch g = corner_site_gemm(c, 1);
  g.A[0] = c->S1[i];
  g.B[0] = c->imp[1];
  g.C[0] = out;
  return g64(c, g);
}

// Diagonal pair on the 2x2 plaquette Tr(Ct1 Ct2 Ct3 Ct4): site 1 in the
// corner o (0: top-left, 1: top-right for the anti-diagonal) and site 2 in
// corner o + 2, the plain double layer in the other two.
// E[i * n2 + j] = Tr(Ct_o(s1[i]) Ct_o+1 Ct_o+2(s2[j]) Ct_o+3), as
// <Ct_o(s1[i]), Z_j^T> with Z_j = Ct_o+1 Ct_o+2(s2[j]) Ct_o+3 stored
// transposed (n2 <= kMaxDots of them in Pl, Prt, Zc[0]).
int diag_pair(ctm_ctx* c, bool anti, const double* const* s1, int n1, const double* const* s2,
              int n2, double* E) {
  const int x = c->chi_env, Dl = c->Dl;
  const long N = (long)x * Dl;
  if (n1 < 1 || n2 < 1 || n2 > kMaxDots) return fail(c, CTM_E_SHAPE, "diagonal pair: bad count");
  const int o = anti ? 1 : 0, i1 = (o + 1) % 4, i2 = (o + 2) % 4, i3 = (o + 3) % 4;
  TRY(corner_stems(c, PC_MISC));
  TRY(corner_with(c, i1, c->a, c->S2[i1]));
  TRY(corner_with(c, i3, c->a, c->S2[i3]));
  double* Z[kMaxDots] = {c->Pl[0], c->Pl[1], c->Pl[2], c->Pl[3], c->Prt[0],
                         c->Prt[1], c->Prt[2], c->Prt[3], c->Zc[0]};
  for (int j = 0; j < n2; ++j) {
    TRY(corner_with(c, i2, s2[j], c->S2[o]));
    TRY(g64(c, gb1((int)N, (int)N, (int)N, c->S2[i1], N, 0, c->S2[o], N, c->S2[i2], N)));
    GemmBatch g = gb1((int)N, (int)N, (int)N, c->S2[i2], N, 0, c->S2[i3], N, Z[j], 0);
    set_map(g, 1 << 30, 0, 1, 1 << 30, 0, N);   // Z_j^T
    TRY(g64(c, g));
  }
  for (int i = 0; i < n1; ++i) {
    TRY(corner_with(c, o, s1[i], c->S2[o]));
    TRY(elem_dots(c->S2[o], Z, n2, N * N, c->dot_part, E + (long)i * n2, c->st));
  }
  return 0;
}

// w_i = E v_i for up to four vectors v_i (x, Dl, x) of the column transfer
// matrix E[(b, l, n), (g, r, z)] = T1[b,u,g] a[u,l,d,r] T3[z,d,n], as three
// batched GEMMs whose output maps leave each result in the layout the next
// one reads (intermediates of vector i in S1[i] and S2[i]):
// X[(g, n), (u, l)] = sum_b T1[b, (u, g)] v[b, (l, n)];
// Y[(d, n), (g, r)] = sum_(u,l) X[(g, n), (u, l)] a[(u, l), (d, r)];
// w[(g, r, z)]      = sum_(d,n) T3[z, (d, n)] Y[(d, n), (g, r)],
// written with stride ws (w_i = block + column, row-major block).
int transfer_apply(ctm_ctx* c, const double* T1, const double* T3, const double* a,
                   const double* const* v, double* const* w, int count, long ws) {
  const int x = c->chi_env, Dl = c->Dl;
  GemmBatch g = gemm_rowmajor(count, Dl * x, Dl * x, x, (long)Dl * x, (long)Dl * x, 0);
  for (int i = 0; i < count; ++i) {
    g.A[i] = T1;
    g.transA[i] = 1;
    g.B[i] = v[i];
    g.C[i] = c->S1[i];
  }
  set_map(g, x, Dl, (long)x * Dl * Dl, x, 1, (long)Dl * Dl);
  TRY(g64(c, g));
  g = gemm_rowmajor(count, x * x, Dl * Dl, Dl * Dl, (long)Dl * Dl, (long)Dl * Dl, 0);
  for (int i = 0; i < count; ++i) {
    g.A[i] = c->S1[i];
    g.B[i] = a;
    g.C[i] = c->S2[i];
  }
  set_map(g, x, Dl, (long)x * Dl, Dl, (long)x * x * Dl, 1);
  TRY(g64(c, g));
  g = gemm_rowmajor(count, x, x * Dl, Dl * x, (long)Dl * x, (long)x * Dl, 0);
  for (int i = 0; i < count; ++i) {
    g.A[i] = T3;
    g.B[i] = c->S2[i];
    g.C[i] = w[i];
  }
  set_map(g, 1 << 30, 0, ws, 1 << 30, 0, (long)x * ws);
  return g64(c, g);
}

// Correlation length along the rows (vertical: the turned network, edges
// T2 and T4 with the site legs rotated) by block iteration: W = E V, V =
// QR(W), `iters` times, then the Rayleigh-Ritz matrix H = V^T E V and its
// two leading eigenvalue moduli; out: xi, |l2/l1|, l1.
int correlation_length(ctm_ctx* c, bool vertical, int iters, double* out_host) {
  const int x = c->chi_env, Dl = c->Dl, m = c->xi_m;
  const long nE = (long)x * Dl * x;
  if (!c->xi_qr || (long)c->chi * Dl * c->chi < nE)
    return fail(c, CTM_E_SHAPE, "correlation length: no QR plan for the transfer-matrix block");
  const int mm = (int)std::min<long>(m, nE);
  if (!qr_plan_ok((int)nE, mm))
    return fail(c, CTM_E_SHAPE, "correlation length: no QR plan for the transfer-matrix block");
  double* const* T = c->T[c->cur];
  const double* a = c->a;
  const double *T1 = T[0], *T3 = T[2];
  if (vertical) {
    // turned network: a_r[u', l', d', r'] = a[u = l', l = d', d = r', r = u']
    const long D1 = Dl, D2 = D1 * Dl, D3 = D2 * Dl;
    TRY(elem_permute4(c->a, c->imp[2], DT::F64, Dl, 1, D3, D2, D1, c->st));
    a = c->imp[2];
    T1 = T[1];
    T3 = T[3];
  }
  // seeded start block (host generator; the same every call), row-major nE x mm
  std::vector<double> v0((size_t)nE * mm);
  uint64_t st = 0x9e3779b97f4a7c15ULL;
  for (double& e : v0) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    e = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  CTM_HIP_TRY(hipMemcpyAsync(c->xi_W, v0.data(), v0.size() * 8, hipMemcpyHostToDevice, c->st));
  double* Wp[1] = {c->xi_W};
  for (int it = 0; it <= iters; ++it) {
    TRY(launch_qr(1, Wp, (int)nE, mm, c->xi_qr, c->st) ? fail(c, CTM_E_DEVICE, thread_error()) : 0);
    CTM_HIP_TRY(hipMemcpyAsync(c->xi_V, c->xi_W, (size_t)nE * mm * 8, hipMemcpyDeviceToDevice, c->st));
    TRY(elem_transpose(c->xi_V, c->xi_Vc, nE, mm, c->st));
    for (int k0 = 0; k0 < mm; k0 += 4) {
      const int cnt = std::min(4, mm - k0);
      const double* vs[4];
      double* ws[4];
      for (int i = 0; i < cnt; ++i) {
        vs[i] = c->xi_Vc + (long)(k0 + i) * nE;
        ws[i] = c->xi_W + k0 + i;
      }
      TRY(transfer_apply(c, T1, T3, a, vs, ws, cnt, mm));
    }
  }
  // H = V^T (E V): mm^2 dot products over nE between the columns of V
  // (contiguous in Vc) and of W (transposed into V, no longer needed)
  TRY(elem_transpose(c->xi_W, c->xi_V, nE, mm, c->st));
  {
    const double* wc[kXiBlock];
    for (int j = 0; j < mm; ++j) wc[j] = c->xi_V + (long)j * nE;
    for (int i = 0; i < mm; ++i)
      TRY(elem_dots(c->xi_Vc + (long)i * nE, wc, mm, nE, c->dot_part, c->xi_H + (long)i * mm, c->st)
              ? fail(c, CTM_E_ARG, "dot products") : 0);
  }
  TRY(elem_xi_from_ritz(c->xi_H, mm, 60, c->xi_out, c->st) ? fail(c, CTM_E_ARG, "small eigenproblem") : 0);
  CTM_HIP_TRY(hipMemcpyAsync(out_host, c->xi_out, 3 * 8, hipMemcpyDeviceToHost, c->st));
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  return 0;
}

int observable(ctm_ctx* c, int kind, const double* op_host, double* out_host) {
  const int Dl = c->Dl, d = c->d;
  const size_t Dl4 = (size_t)Dl * Dl * Dl * Dl;
  double* sc = c->scal + 16;   // device scalars
  double host[32] = {0};
  if (kind == CTM_OBS_NORM) {
    TRY(perm_site(c, c->a, c->imp[2], 0));
    TRY(z11(c, c->imp[2], sc));
    TRY(z_rest(c, sc + 1));
    TRY(elem_kappa(sc, sc + 5, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(host, sc, 6 * 8, hipMemcpyDeviceToHost, c->st));
    CTM_HIP_TRY(hipStreamSynchronize(c->st));
    out_host[0] = host[5];
    for (int i = 0; i < 4; ++i) out_host[1 + i] = host[i];
    return 0;
  }
  if (kind == CTM_OBS_XI_H || kind == CTM_OBS_XI_V) {
    const int iters = op_host ? (int)op_host[0] : 100;
    if (iters < 1 || iters > 100000) return fail(c, CTM_E_ARG, "iterations outside [1, 100000]");
    return correlation_length(c, kind == CTM_OBS_XI_V, iters, out_host);
  }
  if (!op_host) return fail(c, CTM_E_ARG, "observable needs an operator");
  if (kind == CTM_OBS_ONESITE) {
    if (d > 0) {
      CTM_HIP_TRY(hipMemcpy(c->obs_op, op_host, (size_t)d * d * 8, hipMemcpyHostToDevice));
      TRY(elem_double_layer(c->A_site, c->obs_op, c->imp[0], d, c->D, c->st));
    } else {
      CTM_HIP_TRY(hipMemcpy(c->imp[0], op_host, Dl4 * 8, hipMemcpyHostToDevice));
    }
    TRY(perm_site(c, c->imp[0], c->imp[1], 0));
    TRY(perm_site(c, c->a, c->imp[2], 0));
    TRY(z11(c, c->imp[1], sc));
    TRY(z11(c, c->imp[2], sc + 1));
    TRY(elem_ratio(sc, sc + 1, sc + 2, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(host, sc, 3 * 8, hipMemcpyDeviceToHost, c->st));
    CTM_HIP_TRY(hipStreamSynchronize(c->st));
    out_host[0] = host[2];
    return 0;
  }
  if (kind == CTM_OBS_BOND_D || kind == CTM_OBS_BOND_AD) {
    const bool anti = kind == CTM_OBS_BOND_AD;
    if (d == 0) {
      // two impurities (site 1 then site 2) against the plain plaquette
      CTM_HIP_TRY(hipMemcpy(c->imps[0], op_host, Dl4 * 8, hipMemcpyHostToDevice));
      CTM_HIP_TRY(hipMemcpy(c->imps[1], op_host + Dl4, Dl4 * 8, hipMemcpyHostToDevice));
      const double* a1[1] = {c->imps[0]};
      const double* a2[1] = {c->imps[1]};
      TRY(diag_pair(c, anti, a1, 1, a2, 1, sc));
      const double* b1[1] = {c->a};
      TRY(diag_pair(c, anti, b1, 1, b1, 1, sc + 1));
      TRY(elem_ratio(sc, sc + 1, sc + 2, c->st));
      CTM_HIP_TRY(hipMemcpyAsync(host, sc, 3 * 8, hipMemcpyDeviceToHost, c->st));
      CTM_HIP_TRY(hipStreamSynchronize(c->st));
      out_host[0] = host[2];
      return 0;
    }
    const int d2 = d * d;
    if (d2 > kMaxDots) return fail(c, CTM_E_SHAPE, "diagonal bond observables support d <= 3");
    std::vector<const double*> so(d2);
    for (int st = 0; st < d2; ++st) {
      double* p = c->imps[0] + st * Dl4;
      TRY(elem_double_layer(c->A_site, nullptr, p, d, c->D, c->st, st / d, st % d));
      so[st] = p;
    }
    double* E = c->scal + 64;
    TRY(diag_pair(c, anti, so.data(), d2, so.data(), d2, E));
    CTM_HIP_TRY(hipMemcpy(c->obs_op, op_host, (size_t)d2 * d2 * 8, hipMemcpyHostToDevice));
    TRY(elem_bond_value(E, c->obs_op, d, sc, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(host, sc, 8, hipMemcpyDeviceToHost, c->st));
    CTM_HIP_TRY(hipStreamSynchronize(c->st));
    out_host[0] = host[0];
    return 0;
  }
  if (kind != CTM_OBS_BOND_H && kind != CTM_OBS_BOND_V)
    return fail(c, CTM_E_ARG, "unknown observable kind");
  const bool hor = kind == CTM_OBS_BOND_H;
  const int slot2 = hor ? 1 : 2;
  if (d == 0) {
    // two impurities (x1 then x2) against the plain network
    CTM_HIP_TRY(hipMemcpy(c->imp[0], op_host, Dl4 * 8, hipMemcpyHostToDevice));
    TRY(perm_site(c, c->imp[0], c->imp[1], 0));
    CTM_HIP_TRY(hipMemcpy(c->imp[0], op_host + Dl4, Dl4 * 8, hipMemcpyHostToDevice));
    TRY(perm_site(c, c->imp[0], c->imp[2], slot2));
    const double* a1[1] = {c->imp[1]};
    const double* a2[1] = {c->imp[2]};
    TRY(two_site(c, hor, a1, 1, a2, 1, sc));
    // plain network: permute a into both slots (imp[0], imp[1])
    TRY(perm_site(c, c->a, c->imp[0], 0));
    TRY(perm_site(c, c->a, c->imp[1], slot2));
    const double* b1[1] = {c->imp[0]};
    const double* b2[1] = {c->imp[1]};
    TRY(two_site(c, hor, b1, 1, b2, 1, sc + 1));
    TRY(elem_ratio(sc, sc + 1, sc + 2, c->st));
    CTM_HIP_TRY(hipMemcpyAsync(host, sc, 3 * 8, hipMemcpyDeviceToHost, c->st));
    CTM_HIP_TRY(hipStreamSynchronize(c->st));
    out_host[0] = host[2];
    return 0;
  }
  // open physical legs: one impurity per (ket s, bra t); d^2 x d^2 values E
  const int d2 = d * d;
  if (d2 > 9) return fail(c, CTM_E_SHAPE, "bond observables support d <= 3");
  std::vector<const double*> s1(d2), s2(d2);
  // site-1 tensors in imps[0], site-2 tensors in imps[1] (each Dl^4, d^2 of them)
  for (int st = 0; st < d2; ++st) {
    TRY(elem_double_layer(c->A_site, nullptr, c->imp[0], d, c->D, c->st, st / d, st % d));
    double* p1 = c->imps[0] + st * Dl4;
    double* p2 = c->imps[1] + st * Dl4;
    TRY(perm_site(c, c->imp[0], p1, 0));
    TRY(perm_site(c, c->imp[0], p2, slot2));
    s1[st] = p1;
    s2[st] = p2;
  }
  double* E = c->scal + 64;
  TRY(two_site(c, hor, s1.data(), d2, s2.data(), d2, E));
  CTM_HIP_TRY(hipMemcpy(c->obs_op, op_host, (size_t)d2 * d2 * 8, hipMemcpyHostToDevice));
  TRY(elem_bond_value(E, c->obs_op, d, sc, c->st));
  CTM_HIP_TRY(hipMemcpyAsync(host, sc, 8, hipMemcpyDeviceToHost, c->st));
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  out_host[0] = host[0];
  return 0;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ctm_status_str(ctm_status s) {
  switch (s) {
    case CTM_OK: return "ok";
    case CTM_E_ARG: return "invalid argument";
    case CTM_E_SHAPE: return "invalid shape";
    case CTM_E_NOMEM: return "out of memory";
    case CTM_E_DEVICE: return "device error";
    case CTM_E_NUMERIC: return "numerical failure";
    case CTM_E_NOT_CONVERGED: return "not converged";
    case CTM_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* ctm_last_error(const ctm_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_err.c_str();
}

ctm_status ctm_workspace_bytes(const ctm_config* cfg, size_t* bytes) {
  int r = validate(cfg);
  if (r) return (ctm_status)r;
  if (!bytes) return (ctm_status)fail(nullptr, CTM_E_ARG, "null bytes");
  ctm_ctx tmp;
  set_dims(&tmp, cfg);
  *bytes = carve(&tmp, nullptr);
  return CTM_OK;
}

ctm_status ctm_init(ctm_ctx** out, const ctm_config* cfg, const double* site_dev,
                    const double* boundary_dev, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return (ctm_status)fail(nullptr, CTM_E_ARG, "null out");
  *out = nullptr;
  int r = validate(cfg);
  if (r) return (ctm_status)r;
  if (!site_dev) return (ctm_status)fail(nullptr, CTM_E_ARG, "null site tensor");
  if (cfg->d == 0 && !boundary_dev)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "d == 0 needs a boundary vector");
  ctm_ctx* c = new ctm_ctx();
  set_dims(c, cfg);
  c->st = (hipStream_t)stream;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      c->sk_cus = std::min(cus, kSplitMaxCus);
  }
  const size_t need = carve(c, nullptr);
  if (workspace) {
    if (ws_bytes < need) {
      delete c;
      return (ctm_status)fail(nullptr, CTM_E_NOMEM, "workspace smaller than ctm_workspace_bytes");
    }
    c->ws = workspace;
  } else {
    if (hipMalloc(&c->ws, need) != hipSuccess) {
      delete c;
      return (ctm_status)fail(nullptr, CTM_E_NOMEM, "hipMalloc of the workspace failed");
    }
    c->own_ws = true;
  }
  c->ws_bytes = need;
  carve(c, (char*)c->ws);
  if (hipHostMalloc((void**)&c->hbuf, 32 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess) {
    std::string m = "pinned host buffer or event creation failed";
    ctm_destroy(c);
    return (ctm_status)fail(nullptr, CTM_E_NOMEM, m);
  }
  auto bail = [&](int code) {
    std::string m = c->err.empty() ? g_err : c->err;
    ctm_destroy(c);
    g_err = m;
    return (ctm_status)code;
  };
  const int Dl = c->Dl;
  const size_t Dl4 = (size_t)Dl * Dl * Dl * Dl;
  int rc = 0;
  if (c->d > 0) {
    const size_t nA = (size_t)c->d * c->D * c->D * c->D * c->D;
    if (hipMemcpyAsync(c->A_site, site_dev, nA * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
      return bail(fail(c, CTM_E_DEVICE, "copy of the site tensor failed"));
    rc = elem_double_layer(c->A_site, nullptr, c->a, c->d, c->D, c->st);
  } else {
    if (hipMemcpyAsync(c->a, site_dev, Dl4 * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
      return bail(fail(c, CTM_E_DEVICE, "copy of the site tensor failed"));
  }
  if (rc) return bail(rc);
  if (boundary_dev) {
    if (hipMemcpyAsync(c->e, boundary_dev, Dl * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
      return bail(fail(c, CTM_E_DEVICE, "copy of the boundary vector failed"));
  } else {
    std::vector<double> e(Dl, 0.0);
    for (int i = 0; i < c->D; ++i) e[i * c->D + i] = 1.0;
    if (hipMemcpy(c->e, e.data(), Dl * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(c, CTM_E_DEVICE, "copy of the boundary vector failed"));
  }
  // leg permutations of a for the four corner absorptions (a[u,l,d,r]):
  // corner 0: (l,u),(d,r); 1: (u,r),(l,d); 2: (r,d),(u,l); 3: (d,l),(r,u)
  const long su = (long)Dl * Dl * Dl, sl = (long)Dl * Dl, sd = Dl, sr = 1;
  const long perm[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
  for (int i = 0; i < 4 && !rc; ++i) {
    rc = elem_permute4(c->a, c->ap[i], c->cp, Dl, perm[i][0], perm[i][1], perm[i][2], perm[i][3],
                       c->st);
    if (!rc)
      rc = elem_permute4(c->a, c->apr[i], c->cp, Dl, perm[i][1], perm[i][0], perm[i][2],
                         perm[i][3], c->st);
  }
  if (rc) return bail(rc);
  rc = elem_init_env(c->a, c->e, Dl, c->C[0], c->T[0], c->st);
  if (!rc && c->cfg.sym == CTM_SYM_C4V) rc = c4v_finish(c, 0, Dl);
  if (rc) return bail(rc);
  c->cur = 0;
  c->chi_env = Dl;
  if (hipMemsetAsync(c->bad, 0, sizeof(int), c->st) != hipSuccess ||
      hipMemsetAsync(c->spec[0], 0, 4 * c->chi * 8, c->st) != hipSuccess ||
      hipMemsetAsync(c->spec[1], 0, 4 * c->chi * 8, c->st) != hipSuccess)
    return bail(fail(c, CTM_E_DEVICE, "memset failed"));
  rc = normalize_env(c, 0, Dl);
  if (!rc) rc = spectra(c, 0, Dl);
  if (rc) return bail(rc);
  c->spec_cur = 1;
  int bad = 0;
  if (hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return bail(fail(c, CTM_E_DEVICE, "synchronisation failed"));
  if (bad) return bail(fail(c, CTM_E_NUMERIC, "initial environment has a zero or non-finite norm"));
  *out = c;
  return CTM_OK;
}

void ctm_destroy(ctm_ctx* c) {
  if (!c) return;
  // a move in flight may run on another context's stream (a batched move)
  if (c->pending) (void)hipEventSynchronize(c->done_ev);
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  drop_graphs(c);
  if (c->done_ev) (void)hipEventDestroy(c->done_ev);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  if (c->rb) rocblas_destroy_handle(c->rb);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  delete c;
}

ctm_status ctm_set_isometries(ctm_ctx* c, const double* X_dev, const double* Yt_dev) {
  if (!c || !X_dev || !Yt_dev) return (ctm_status)fail(c, CTM_E_ARG, "null argument");
  if (c->pending) return (ctm_status)fail(c, CTM_E_STATE, "a move is in flight");
  const size_t nk = (size_t)c->N * c->k;
  for (int b = 0; b < 4; ++b) {
    if (hipMemcpyAsync(c->X0[b], X_dev + b * nk, nk * 8, hipMemcpyDeviceToDevice, c->st) !=
            hipSuccess ||
        hipMemcpyAsync(c->Yt0[b], Yt_dev + b * nk, nk * 8, hipMemcpyDeviceToDevice, c->st) !=
            hipSuccess)
      return (ctm_status)fail(c, CTM_E_DEVICE, "copy of the isometries failed");
  }
  c->iso_pending = true;
  c->si_ready = false;
  c->recycling = false;
  c->si_upd = 0;
  return CTM_OK;
}

ctm_status ctm_move(ctm_ctx* c, ctm_move_info* info) {
  if (!c) return (ctm_status)fail(nullptr, CTM_E_ARG, "null context");
  c->err.clear();
  g_err.clear();
  const int r = drain(c);
  if (r) return (ctm_status)r;
  return (ctm_status)do_move(c, info);
}

ctm_status ctm_use_graphs(ctm_ctx* c, int enable) {
  if (!c) return (ctm_status)fail(nullptr, CTM_E_ARG, "null context");
  const int rd = drain(c);
  if (rd) return (ctm_status)rd;
  if (enable && c->st == nullptr)
    return (ctm_status)fail(c, CTM_E_STATE, "graphs need a non-default stream");
  if (hipStreamSynchronize(c->st) != hipSuccess)
    return (ctm_status)fail(c, CTM_E_DEVICE, "synchronisation failed");
  if (!enable) drop_graphs(c);
  c->use_graphs = enable != 0;
  return CTM_OK;
}

ctm_status ctm_move_async(ctm_ctx* c) {
  if (!c) return (ctm_status)fail(nullptr, CTM_E_ARG, "null context");
  c->err.clear();
  return (ctm_status)enqueue_move(c);
}

ctm_status ctm_move_poll(ctm_ctx* c, int* done, ctm_move_info* info) {
  if (!c || !done) return (ctm_status)fail(c, CTM_E_ARG, "null argument");
  *done = 0;
  if (!c->pending) return (ctm_status)fail(c, CTM_E_STATE, "no move in flight");
  const hipError_t q = hipEventQuery(c->done_ev);
  if (q == hipErrorNotReady) return CTM_OK;
  if (q != hipSuccess) {
    c->pending = false;
    return (ctm_status)fail(c, CTM_E_DEVICE, std::string("move failed on the device: ") +
                                                 hipGetErrorString(q));
  }
  *done = 1;
  return (ctm_status)finish_move(c, info);
}

ctm_status ctm_move_batch_async(ctm_ctx* const* ctxs, int n) {
  if (!ctxs || n < 0) return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid batch");
  g_err.clear();
  return (ctm_status)enqueue_batch(ctxs, n);
}

ctm_status ctm_move_batch(ctm_ctx* const* ctxs, int n, ctm_move_info* infos) {
  if (!ctxs || n < 0) return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid batch");
  g_err.clear();
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return (ctm_status)fail(nullptr, CTM_E_ARG, "null context in the batch");
    const int rd = drain(ctxs[i]);
    if (rd) return (ctm_status)rd;
  }
  int first = enqueue_batch(ctxs, n);
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]->pending) continue;               // not enqueued (an earlier error)
    const int r = wait_move(ctxs[i], infos ? infos + i : nullptr);
    if (r && !first) first = r;
  }
  return (ctm_status)first;
}

ctm_status ctm_converge(ctm_ctx* c, double tol, int max_moves, int* moves_done,
                        double* last_delta) {
  if (!c || max_moves < 0) return (ctm_status)fail(c, CTM_E_ARG, "invalid argument");
  int n = 0;
  double delta = INFINITY;
  ctm_status st = CTM_E_NOT_CONVERGED;
  while (n < max_moves) {
    ctm_move_info info;
    ctm_status r = ctm_move(c, &info);
    if (r != CTM_OK) {
      st = r;
      break;
    }
    ++n;
    delta = info.delta;
    if (info.mode == 2 || info.mode == 1) {
      if (delta < tol && c->chi_env == c->chi) {
        st = CTM_OK;
        break;
      }
    }
  }
  if (moves_done) *moves_done = n;
  if (last_delta) *last_delta = delta;
  return st;
}

ctm_status ctm_state_size(const ctm_ctx* c, size_t* n) {
  if (!c || !n) return (ctm_status)fail(nullptr, CTM_E_ARG, "null argument");
  const size_t chi = c->chi, Dl = c->Dl, N = c->N, k = c->k;
  *n = 4 * chi * chi + 4 * chi * Dl * chi + 8 * N * k + 4;
  return CTM_OK;
}

}  // extern "C"

namespace {

// Copies the state vector (layout of ctm_state_size) to host or device memory.
int copy_state(ctm_ctx* c, double* dst, size_t n, bool device) {
  size_t need;
  if (c && c->pending) {
    const int rd = drain(c);
    if (rd) return rd;
  }
  if (ctm_state_size(c, &need) != CTM_OK || !dst || n < need)
    return fail(c, CTM_E_ARG, "state buffer too small");
  const size_t chi = c->chi, Dl = c->Dl, N = c->N, k = c->k;
  const size_t x = c->chi_env;
  const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (device) {
    CTM_HIP_TRY(hipMemsetAsync(dst, 0, need * sizeof(double), c->st));
  } else {
    std::fill(dst, dst + need, 0.0);
  }
  double* p = dst;
  for (int i = 0; i < 4; ++i, p += chi * chi)
    CTM_HIP_TRY(hipMemcpyAsync(p, c->C[c->cur][i], x * x * 8, kind, c->st));
  for (int i = 0; i < 4; ++i, p += chi * Dl * chi)
    CTM_HIP_TRY(hipMemcpyAsync(p, c->T[c->cur][i], x * Dl * x * 8, kind, c->st));
  // the blocks the next SI move starts from: the caller's start blocks while
  // they are pending, none (zeros) before any exist
  const bool blocks = c->iso_pending || c->si_ready;
  for (int i = 0; i < 4; ++i, p += N * k)
    if (blocks)
      CTM_HIP_TRY(hipMemcpyAsync(p, c->iso_pending ? c->X0[i] : c->X[i], N * k * 8, kind, c->st));
  for (int i = 0; i < 4; ++i, p += N * k)
    if (blocks)
      CTM_HIP_TRY(hipMemcpyAsync(p, c->iso_pending ? c->Yt0[i] : c->Yt[i], N * k * 8, kind, c->st));
  const double tail[4] = {(double)c->chi_env, (double)c->si_moves, c->recycling ? 1.0 : 0.0,
                          (double)c->si_upd};
  if (device) {
    CTM_HIP_TRY(hipMemcpyAsync(p, tail, sizeof(tail), hipMemcpyHostToDevice, c->st));
  } else {
    std::copy(tail, tail + 4, p);
  }
  CTM_HIP_TRY(hipStreamSynchronize(c->st));
  return CTM_OK;
}

}  // namespace

extern "C" {

ctm_status ctm_get_state(ctm_ctx* c, double* host, size_t n) {
  return (ctm_status)copy_state(c, host, n, false);
}

ctm_status ctm_get_state_device(ctm_ctx* c, double* dev, size_t n) {
  return (ctm_status)copy_state(c, dev, n, true);
}

ctm_status ctm_set_state(ctm_ctx* c, const double* host, size_t n) {
  size_t need;
  if (c && c->pending) {
    const int rd = drain(c);
    if (rd) return (ctm_status)rd;
  }
  if (ctm_state_size(c, &need) != CTM_OK || !host || n < need)
    return (ctm_status)fail(c, CTM_E_ARG, "state buffer too small");
  const size_t chi = c->chi, Dl = c->Dl, N = c->N, k = c->k;
  const double* p = host + 4 * chi * chi + 4 * chi * Dl * chi + 8 * N * k;
  const int x = (int)p[0];
  if (x < 1 || x > (int)chi) return (ctm_status)fail(c, CTM_E_SHAPE, "chi_env out of range");
  p = host;
  for (int i = 0; i < 4; ++i, p += chi * chi)
    if (hipMemcpy(c->C[c->cur][i], p, (size_t)x * x * 8, hipMemcpyHostToDevice) != hipSuccess)
      return (ctm_status)fail(c, CTM_E_DEVICE, "copy failed");
  for (int i = 0; i < 4; ++i, p += chi * Dl * chi)
    if (hipMemcpy(c->T[c->cur][i], p, (size_t)x * Dl * x * 8, hipMemcpyHostToDevice) != hipSuccess)
      return (ctm_status)fail(c, CTM_E_DEVICE, "copy failed");
  // blocks: the current ones at chi_env == chi; during growth, non-zero
  // blocks are the pending start blocks of the first SI move
  bool has_blocks = false;
  for (size_t i = 0; i < 8 * N * k && !has_blocks; ++i) has_blocks = p[i] != 0.0;
  const bool grow = x < (int)chi;
  for (int i = 0; i < 4; ++i, p += N * k)
    if (hipMemcpy(grow ? c->X0[i] : c->X[i], p, N * k * 8, hipMemcpyHostToDevice) != hipSuccess)
      return (ctm_status)fail(c, CTM_E_DEVICE, "copy failed");
  for (int i = 0; i < 4; ++i, p += N * k)
    if (hipMemcpy(grow ? c->Yt0[i] : c->Yt[i], p, N * k * 8, hipMemcpyHostToDevice) != hipSuccess)
      return (ctm_status)fail(c, CTM_E_DEVICE, "copy failed");
  c->chi_env = x;
  c->si_moves = (long)p[1];
  c->recycling = c->cfg.recycle_sin2 > 0 && p[2] != 0.0;
  c->si_upd = (int)p[3];
  c->last_si_delta = -1.0;
  c->si_ready = !grow;
  c->iso_pending = grow && has_blocks;
  // spectra of the restored corners become the reference of the next delta
  const int rs = spectra(c, c->cur, x);
  if (rs) return (ctm_status)(rs == 1 ? CTM_E_ARG : rs);
  c->spec_cur = 1 - c->spec_cur;
  if (hipStreamSynchronize(c->st) != hipSuccess)
    return (ctm_status)fail(c, CTM_E_DEVICE, "synchronisation failed");
  return CTM_OK;
}


}  // extern "C"

namespace sictm {

int vjp_view(ctm_ctx* c, VjpView* v) {
  const int rd = drain(c);
  if (rd) return rd;
  v->cfg = c->cfg;
  v->d = c->d;
  v->D = c->D;
  v->Dl = c->Dl;
  v->chi = c->chi;
  v->k = c->k;
  v->N = c->N;
  v->st = c->st;
  v->A_site = c->A_site;
  v->a = c->a;
  v->sk_part = c->sk_part;
  v->sk_cus = c->sk_cus;
  const long Dl = c->Dl;
  const long su = Dl * Dl * Dl, sl = Dl * Dl, sd = Dl, sr = 1;
  const long perm[4][4] = {{sl, su, sd, sr}, {su, sr, sl, sd}, {sr, sd, su, sl}, {sd, sl, sr, su}};
  for (int i = 0; i < 4; ++i) {
    v->ap[i] = (const double*)c->ap[i];
    for (int j = 0; j < 4; ++j) v->ap_strides[i][j] = perm[i][j];
  }
  return 0;
}

int vjp_fail(ctm_ctx* c, int code, const std::string& msg) { return fail(c, code, msg); }

int ctx_phys_dim(const ctm_ctx* c) { return c->d; }

}  // namespace sictm

extern "C" {

ctm_status ctm_observable(ctm_ctx* c, int kind, const double* op_host, double* out_host) {
  if (!c || !out_host) return (ctm_status)fail(c, CTM_E_ARG, "null argument");
  c->err.clear();
  const int rd = drain(c);
  if (rd) return (ctm_status)rd;
  const bool prof = c->prof;
  c->prof = false;
  const int r = observable(c, kind, op_host, out_host);
  c->prof = prof;
  return (ctm_status)r;
}

ctm_status ctm_profile(ctm_ctx* c, int enable) {
  if (!c) return (ctm_status)fail(nullptr, CTM_E_ARG, "null context");
  if (hipStreamSynchronize(c->st) != hipSuccess)
    return (ctm_status)fail(c, CTM_E_DEVICE, "synchronisation failed");
  c->recs.clear();
  c->ev_next = 0;
  c->prof = enable != 0;
  return CTM_OK;
}

ctm_status ctm_profile_read(ctm_ctx* c, ctm_prof_entry* out, int max_entries, int* n) {
  if (!c || !out || !n) return (ctm_status)fail(c, CTM_E_ARG, "null argument");
  if (hipStreamSynchronize(c->st) != hipSuccess)
    return (ctm_status)fail(c, CTM_E_DEVICE, "synchronisation failed");
  int cnt = 0;
  for (int cls = 0; cls < PC_N && cnt < max_entries; ++cls) {
    ctm_prof_entry e;
    std::memset(&e, 0, sizeof(e));
    std::strncpy(e.name, kProfNames[cls], sizeof(e.name) - 1);
    for (const auto& r : c->recs) {
      if (r.cls != cls) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
        return (ctm_status)fail(c, CTM_E_DEVICE, "hipEventElapsedTime failed");
      e.launches += 1;
      e.ms += ms;
      e.flops += r.flops;
      e.bytes += r.bytes;
    }
    if (e.launches) out[cnt++] = e;
  }
  *n = cnt;
  return CTM_OK;
}

ctm_status ctm_gemm_f64(int count, const double* const* A, const double* const* B,
                        double* const* C, int M, int N, int K, int trans_a, long lda, long ldb,
                        long ldc, double alpha, int accumulate, void* stream) {
  if (count < 0 || count > kMaxProb || M < 0 || N < 0 || K < 0 || !A || !B || !C)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid gemm arguments");
  GemmBatch g = gemm_rowmajor(count, M, N, K, lda, ldb, ldc);
  g.alpha = alpha;
  g.accumulate = accumulate;
  for (int i = 0; i < count; ++i) {
    g.A[i] = A[i];
    g.B[i] = B[i];
    g.C[i] = C[i];
    g.transA[i] = trans_a;
  }
  int r = launch_gemm_si(g, (hipStream_t)stream);   // skinny kernel when N <= 160
  return r ? CTM_E_DEVICE : CTM_OK;
}

size_t ctm_gemm_f64_split_scratch_bytes(void) { return gemm_si_scratch_bytes(); }

ctm_status ctm_gemm_f64_split(int count, const double* const* A, const double* const* B,
                              double* const* C, int M, int N, int K, const int* trans_a, long lda,
                              long ldb, long ldc, double alpha, int accumulate, void* scratch,
                              size_t scratch_bytes, int ncu, int* used_split, void* stream) {
  if (count < 0 || count > kMaxProb || M < 0 || N < 0 || K < 0 || !A || !B || !C || !trans_a)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid gemm arguments");
  if (scratch && scratch_bytes < gemm_si_scratch_bytes())
    return (ctm_status)fail(nullptr, CTM_E_ARG, "split scratch smaller than ctm_gemm_f64_split_scratch_bytes");
  if (ncu < 1 || ncu > kSplitMaxCus)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "ncu outside [1, 256]");
  GemmBatch g = gemm_rowmajor(count, M, N, K, lda, ldb, ldc);
  g.alpha = alpha;
  g.accumulate = accumulate;
  for (int i = 0; i < count; ++i) {
    if (trans_a[i] != 0 && trans_a[i] != 1)
      return (ctm_status)fail(nullptr, CTM_E_ARG, "trans_a entries must be 0 or 1");
    g.A[i] = A[i];
    g.B[i] = B[i];
    g.C[i] = C[i];
    g.transA[i] = trans_a[i];
  }
  if (used_split) *used_split = gemm_si_balanced_applies(g, scratch, ncu) ? 1 : 0;
  int r = launch_gemm_si_balanced(g, (double*)scratch, ncu, (hipStream_t)stream);
  return r ? CTM_E_DEVICE : CTM_OK;
}

ctm_status ctm_qr_f64(int count, double* const* W, int N, int k, void* stream) {
  if (count < 0 || count > kMaxProb || !W || k < 1 || N < k)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid qr arguments");
  void* ws = nullptr;
  if (hipMalloc(&ws, qr_workspace_bytes(count, N, k)) != hipSuccess)
    return (ctm_status)fail(nullptr, CTM_E_NOMEM, "hipMalloc failed");
  int r = launch_qr(count, W, N, k, ws, (hipStream_t)stream);
  (void)hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(ws);
  return r ? (ctm_status)(r == 1 ? CTM_E_ARG : r) : CTM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free thin QR: the workspace of launch_qr lives in a file-scope
// device array instead of a hipMalloc'd buffer.  Each device holds its own
// copy of the array at its own address; the host-side name is only a symbol,
// so the address used in kernel arguments is taken once per device with
// hipGetSymbolAddress (with that device current) and kept.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)96 << 20;   // 96 MiB per device
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of this device's scratch array (resolved on first use).
int scratch_address(void** out) {
  int dev = 0;
  CTM_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(nullptr, CTM_E_DEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, CTM_E_DEVICE,
                  std::string("hipGetSymbolAddress of the QR scratch failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

extern "C" {

size_t ctm_qr_f64_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

ctm_status ctm_qr_f64_noalloc(int count, double* const* W, int N, int k, void* stream) {
  if (count < 0 || count > kMaxProb || !W || k < 1 || N < k)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid qr arguments");
  if (count == 0) return CTM_OK;
  if (k > 192 || !qr_plan_ok(N, k))
    return (ctm_status)fail(nullptr, CTM_E_ARG,
                            "no QR leaf partition for these N, k (need k <= 192 and N/k not too large)");
  const size_t need = qr_workspace_bytes(count, N, k);
  if (need > kNoAllocScratchBytes)
    return (ctm_status)fail(nullptr, CTM_E_NOMEM,
                            "QR workspace of " + std::to_string(need) + " bytes exceeds the " +
                                std::to_string(kNoAllocScratchBytes) + "-byte static scratch");
  void* ws = nullptr;
  const int rs = scratch_address(&ws);
  if (rs) return (ctm_status)rs;
  const int r = launch_qr(count, W, N, k, ws, (hipStream_t)stream);
  return r ? (ctm_status)(r == 1 ? CTM_E_ARG : r) : CTM_OK;
}

ctm_status ctm_svd_f64(int count, const double* const* rho, double* const* u, double* const* s,
                       double* const* v, int n, void* stream) {
  if (count < 0 || count > kMaxProb || !rho || !s || n < 1)
    return (ctm_status)fail(nullptr, CTM_E_ARG, "invalid svd arguments");
  void* ws = nullptr;
  if (hipMalloc(&ws, svd_workspace_bytes(count, n)) != hipSuccess)
    return (ctm_status)fail(nullptr, CTM_E_NOMEM, "hipMalloc failed");
  int r = launch_svd(count, rho, u, s, v, n, ws, (hipStream_t)stream);
  (void)hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(ws);
  return r ? (ctm_status)(r == 1 ? CTM_E_ARG : r) : CTM_OK;
}

}  // extern "C"
