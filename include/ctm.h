/*
 * ctm.h -- C ABI of the MI355X SI-CTMRG library (libsictm.so).
 *
 * The library contracts an infinite square-lattice tensor network built from
 * one site tensor with the corner transfer matrix renormalisation group, using
 * the subspace-iteration projectors of Zhang & Corboz, "Fast two-dimensional
 * tensor-network contraction via subspace iteration" (QR-based projector
 * section, steps 1-4) or the standard full-SVD projectors (Standard CTMRG
 * section).  Every step of a move runs in this library's own HIP kernels on
 * the GPU; the full-SVD projectors additionally call rocSOLVER's dgesvd.
 *
 * Conventions shared by every entry point
 *  - All tensors are real float64, C-ordered (row-major).
 *  - Site tensor A[s,u,l,d,r] (physical, up, left, down, right) of shape
 *    (d, D, D, D, D) (iPEPS section, eq. ipeps_ansatz).  With d == 0 the
 *    caller passes the rank-4 network tensor a[u,l,d,r] itself (a classical
 *    model), of leg dimension D.  Dl denotes the leg dimension of the
 *    double layer a: Dl = D*D if d > 0, else D (eq. double_layer).
 *  - Environment (Fig. 1): corners C1..C4 (chi x chi) clockwise from the
 *    top-left, edges T1 (top), T2 (right), T3 (bottom), T4 (left) of shape
 *    (chi, Dl, chi), each ordered (in, inner, out) going clockwise:
 *    C1[a,b] T1[b,u,g] C2[g,h] T2[h,r,e] C3[e,z] T3[z,d,n] C4[n,t] T4[t,l,a].
 *  - N = chi * Dl, k = min(chi + p, N).  Bond b = 0,1,2,3 is the top, right,
 *    bottom, left cut between enlarged corners b and b+1.  Its isometries are
 *    X_b (N x k) and Y_b^T (N x k), both stored N x k row-major.
 *  - Device pointers are HIP device addresses; host pointers are ordinary
 *    process memory.  Unless stated otherwise the library never keeps a
 *    caller pointer beyond the call.
 *  - A stream argument is a hipStream_t passed as void* (NULL = the default
 *    stream).  All device work of a context is ordered on its stream.
 *  - Errors are returned as ctm_status; no entry point aborts the process.
 *    After an error, ctm_last_error() describes it.
 */
#ifndef SICTM_CTM_H
#define SICTM_CTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_ctx ctm_ctx;

typedef enum {
  CTM_OK = 0,
  CTM_E_ARG = 1,           /* null pointer or out-of-range argument            */
  CTM_E_SHAPE = 2,         /* inconsistent dimensions                          */
  CTM_E_NOMEM = 3,         /* workspace too small or device allocation failed  */
  CTM_E_DEVICE = 4,        /* a HIP / rocSOLVER call failed                    */
  CTM_E_NUMERIC = 5,       /* NaN/Inf or zero norm; the environment is kept    */
  CTM_E_NOT_CONVERGED = 6, /* move budget exhausted; the state stays valid     */
  CTM_E_STATE = 7          /* call not valid in the current state              */
} ctm_status;

typedef enum { CTM_PROJ_FULLSVD = 0, CTM_PROJ_SI = 1 } ctm_proj;

/* Lattice symmetry exploited by the move.  CTM_SYM_C4V: a single symmetric
 * corner C and edge T (stored in all four slots); the enlarged corner is
 * symmetric and the projector an isometry shared by all bonds (full mode:
 * eigenvectors of the chi largest |eigenvalues|; SI mode: QR iterations on
 * one block and the eigenvectors of X^T Ct X).  The caller's site tensor
 * must be invariant under the lattice rotations and reflections; float64
 * contractions only. */
typedef enum { CTM_SYM_NONE = 0, CTM_SYM_C4V = 1 } ctm_sym;

/* Precision of the contractions only; QR, small SVD, pseudo-inverse,
 * projector scaling and the stored environment are always float64.
 * CTM_PREC_BF16X3: split bfloat16 -- the contraction operands are kept in
 * float32 and each is written as hi + lo bfloat16 inside the GEMM, whose
 * product is the sum of the three bf16 matrix-core products hi*hi + hi*lo +
 * lo*hi with float32 accumulation (about 16 significant bits per operand). */
typedef enum {
  CTM_PREC_F64 = 0,
  CTM_PREC_F32 = 1,
  CTM_PREC_BF16 = 2,
  CTM_PREC_BF16X3 = 3
} ctm_prec;

typedef enum {
  CTM_OBS_NORM = 0,    /* out[0] = kappa = Z11 Z00 / (Z10 Z01), out[1..4] = Z11,Z00,Z10,Z01 */
  CTM_OBS_ONESITE = 1, /* d > 0: op is d x d (bra, ket); d == 0: op is an impurity a_O[u,l,d,r] */
  CTM_OBS_BOND_H = 2,  /* d > 0: op is d^2 x d^2 on (site1 site2); d == 0: two impurities     */
  CTM_OBS_BOND_V = 3,  /* as BOND_H for the vertical bond (site 1 above site 2)               */
  CTM_OBS_BOND_D = 4,  /* as BOND_H for the diagonal of a plaquette: site 1 top-left, site 2
                          bottom-right (the extra bond of the triangular lattice drawn on the
                          square one, triangular-lattice section)                             */
  CTM_OBS_BOND_AD = 5, /* the other diagonal: site 1 top-right, site 2 bottom-left            */
  CTM_OBS_XI_H = 6,    /* correlation length along a row from the column transfer matrix
                          E[(b,l,n),(g,r,z)] = T1[b,u,g] a[u,l,d,r] T3[z,d,n] (iPEPS benchmark
                          section): out[0] = -1/ln|l2/l1|, out[1] = |l2/l1|, out[2] = l1; op
                          may be NULL or point to the number of block iterations (default
                          100) of the 8 vectors whose Rayleigh-Ritz matrix gives l1, l2 */
  CTM_OBS_XI_V = 7     /* the same along a column (row transfer matrix, edges T4 and T2)     */
} ctm_obs;

typedef struct {
  int d;            /* physical dimension; 0 = the network tensor a is given directly    */
  int D;            /* virtual bond dimension of A, or leg dimension of a when d == 0    */
  int chi;          /* environment bond dimension (>= 1)                                 */
  int p;            /* oversampling of the subspace (>= 0); k = min(chi + p, N) <= 192,
                       and (SI) the N rows must split into QR leaves of k to 192 rows  */
  int n_si;         /* subspace-iteration steps per move (>= 0)                          */
  int proj;         /* ctm_proj                                                          */
  int prec;         /* ctm_prec                                                          */
  int stabilized;   /* 1: orthonormalise after M and after M^T; 0: only after M^T M      */
  double pinv_rtol; /* s_i <= pinv_rtol * s_1 gives s_i^-1/2 := 0 (e.g. 1e-12 in f64)   */
  int svd_driver;   /* dense SVD of M_b (full-SVD projectors and the growth moves):
                       0 = QR iteration (rocSOLVER gesvd; small singular values to
                       high relative accuracy), 1 = divide and conquer (rocSOLVER
                       gesdd via the eigenvectors of M^T M: fast, but its weak
                       directions are noise once s_chi / s_1 is below ~1e-8, which
                       the products of four enlarged corners reach), 2 = selected
                       triples (rocSOLVER gesvdx: bidiagonalisation, then
                       bisection and inverse iteration for the leading chi + 1) */
  int sym;          /* ctm_sym                                                           */
  double recycle_sin2; /* recycling of the SI blocks (QR-based projector section, step 4;
                       recycling criterion of the triangular Heisenberg benchmark):
                       > 0: after at least min_si_moves SI moves with subspace steps,
                       once the largest over the 8 blocks (X, Y of 4 bonds) of the
                       mean sin^2 of the principal angles between the kept chi
                       columns of two successive moves is below this value, later
                       moves take no subspace step (n_si = 0: rho and projectors
                       from the recycled blocks); the steps resume, and the count
                       restarts, when delta grows more than tenfold from one SI
                       move to the next.  The angles are measured only when the
                       previous move was an SI move.  <= 0: n_si steps every move */
  int min_si_moves;    /* SI moves with subspace steps before recycling may start (>= 1) */
  int growth;          /* truncating growth moves (chi_env < chi): 0 = full-SVD projectors
                          (svd_driver); 1 = randomized: SI projectors (n_si steps) from
                          the first chi_env*Dl rows of the start blocks, which stay
                          pending for the first SI move (the warm-up by a randomized
                          SVD that the paper allows); used when chi_env*Dl >= k with a
                          QR leaf split, else full SVD.  Mode 3 in ctm_move_info.   */
} ctm_config;

typedef struct {
  double delta;   /* max over corners of |s_new - s_old|_2 of unit-norm corner spectra */
  int mode;       /* 0: growth without truncation, 1: full-SVD projectors, 2: SI,
                     3: truncating growth with randomized (SI) projectors              */
  int chi_env;    /* environment dimension after the move                              */
  double gap;     /* min over bonds of s_chi / s_(chi+1) - 1 (-1 when not truncated)   */
  int n_si;       /* subspace steps this move took (0 when recycling or not an SI move) */
  double sin2;    /* recycling criterion measured this move, or -1 when not measured    */
} ctm_move_info;

/* Human-readable name of a status code (static string). */
const char* ctm_status_str(ctm_status s);

/* Last error message recorded on ctx (static per context), or "" if none. */
const char* ctm_last_error(const ctm_ctx* ctx);

/* Exact device bytes ctm_init needs for cfg (the admission size of a solve).
 * Returns CTM_E_ARG / CTM_E_SHAPE for invalid configurations. */
ctm_status ctm_workspace_bytes(const ctm_config* cfg, size_t* bytes);

/* Creates a context (iPEPS section: a = sum_s A A; Standard CTMRG section:
 * initial boundary).
 *  site_dev     device, A (d*D^4 doubles) or a (D^4) when d == 0; copied.
 *  boundary_dev device, Dl doubles closing every outer leg of the initial
 *               boundary site, or NULL for vec(I_D) (ket traced against bra;
 *               only valid when d > 0); copied.
 *  workspace    device memory of at least ctm_workspace_bytes(cfg) bytes owned
 *               by the caller and kept until ctm_destroy, or NULL to let the
 *               library allocate (and free) it.
 *  stream       hipStream_t as void*.
 * Builds a and the initial environment; returns once the stream has reached
 * that point.  On error *out is NULL. */
ctm_status ctm_init(ctm_ctx** out, const ctm_config* cfg, const double* site_dev,
                    const double* boundary_dev, void* workspace, size_t ws_bytes,
                    void* stream);

/* Frees the context (and its workspace if the library allocated it). */
void ctm_destroy(ctm_ctx* ctx);

/* Sets the start blocks of the subspace iteration (QR-based projector
 * section, step 1: random Gaussian matrices).  X_dev and Yt_dev are device
 * arrays of 4*N*k doubles ([bond][N][k]); copied.  They take effect at the
 * next SI move that starts from fresh blocks (the first move with
 * chi_env == chi), or immediately if the environment already has chi_env ==
 * chi.  Without this call the library draws its own standard normals. */
ctm_status ctm_set_isometries(ctm_ctx* ctx, const double* X_dev, const double* Yt_dev);

/* One simultaneous four-direction CTMRG move (Fig. 1).  Growth moves
 * (chi_env < chi) use no truncation when chi_env*Dl <= chi, else full-SVD
 * projectors; later moves use the configured projectors.  Stream-ordered;
 * info, if non-NULL, is filled after a stream synchronisation.  On
 * CTM_E_NUMERIC the previous environment is kept. */
ctm_status ctm_move(ctm_ctx* ctx, ctm_move_info* info);

/* Asynchronous move: enqueues one move on the context's stream and returns
 * without waiting (growth moves with full-SVD projectors may still block
 * inside rocSOLVER).  Only one move may be in flight per context
 * (CTM_E_STATE otherwise).  Every other call on the context first completes
 * the move in flight. */
ctm_status ctm_move_async(ctm_ctx* ctx);

/* Non-blocking completion check of the move in flight: *done = 0 while it
 * runs; *done = 1 once it has finished, with info (if non-NULL) filled as by
 * ctm_move and the context switched to the new environment.  CTM_E_STATE
 * when no move is in flight; CTM_E_NUMERIC as for ctm_move. */
ctm_status ctm_move_poll(ctm_ctx* ctx, int* done, ctm_move_info* info);

/* One move of each of n contexts (serving pattern: environment solves of
 * mixed (D, chi) moved together).  The SI moves of float64 contexts without
 * lattice symmetry are recorded and launched together on the stream of the
 * first such context: at every step of the move the float64 GEMMs of all of
 * them (the enlarged corners, the SI applications, rho, the projectors and
 * the renormalisation) run as one persistent grouped launch over a device
 * table of (problem, tile) work items, and the other operations (QR, SVD,
 * signs, norms, spectra) follow one after another.  Each context's results
 * are bit for bit those of ctm_move (the tile kernels' sums do not depend on
 * the grid; the split SI product keeps its own launch).  Other moves
 * (growth, full SVD, C4v, float32/bfloat16) run as ctm_move_async on their
 * own streams.  Work queued earlier on a batched context's own stream is
 * waited for first.  infos (n entries) or NULL; returns the first error
 * after every enqueued move has completed.  A context may appear once. */
ctm_status ctm_move_batch(ctm_ctx* const* ctxs, int n, ctm_move_info* infos);

/* As ctm_move_batch without waiting: every context then has a move in
 * flight, completed through ctm_move_poll (or any call that reads it). */
ctm_status ctm_move_batch_async(ctm_ctx* const* ctxs, int n);

/* Enables (1) or disables (0) graph replay of SI moves.  With graphs on, the
 * device work of an SI move is captured into a HIP graph the first time a
 * given buffer arrangement occurs (two arrangements alternate) and replayed
 * afterwards; growth and full-SVD moves, and moves while profiling, run
 * eagerly.  Results are identical to eager moves.  Needs a non-default
 * stream (CTM_E_STATE otherwise).  Off by default. */
ctm_status ctm_use_graphs(ctm_ctx* ctx, int enable);

/* Moves until the environment has converged (QR-based projector section,
 * step 4: the moves are repeated until C and T converge; Standard CTMRG
 * section: the environment is iterated to its fixed point): stops after the
 * first move at the full environment dimension chi whose delta -- the
 * largest over the four corners of the l2 distance between the unit-norm,
 * sorted, zero-padded singular values of the corner before and after the
 * move -- is below tol, or after max_moves moves.  Returns
 * CTM_E_NOT_CONVERGED when the budget ran out (the state stays valid, and
 * *moves_done, *last_delta report the moves made and the last delta; either
 * may be NULL); a failing move's status otherwise. */
ctm_status ctm_converge(ctm_ctx* ctx, double tol, int max_moves, int* moves_done,
                        double* last_delta);

/* Observable of the current environment (iPEPS section: operator insertion
 * into the norm network).  op_host and out_host are host arrays; see ctm_obs
 * for their meaning.  The diagonal bonds contract the 2x2 plaquette through
 * its four enlarged corners (2 d^2 products of N x N matrices, N = chi D^2;
 * d <= 3) and use the move's intermediate buffers, so they run between
 * moves.  Synchronises the stream. */
ctm_status ctm_observable(ctm_ctx* ctx, int kind, const double* op_host, double* out_host);

/* Number of doubles of the state vector: C1..C4, T1..T4, then X_0..X_3 and
 * Yt_0..Yt_3 (each N x k), then four doubles: chi_env, the number of SI
 * moves made, 1 if the SI blocks are being recycled without subspace steps
 * (else 0), and the SI moves with steps counted towards min_si_moves. */
ctm_status ctm_state_size(const ctm_ctx* ctx, size_t* n);

/* Copies the state vector to / from host memory (n doubles, see
 * ctm_state_size).  Corner and edge blocks are laid out for chi, with the
 * leading chi_env x ... sub-block meaningful during growth.  X, Yt are the
 * blocks the next SI move starts from: while the environment is still
 * growing, the start blocks given to ctm_set_isometries (zeros if none were
 * given; on set, non-zero blocks become the pending start blocks).
 * Synchronises. */
ctm_status ctm_get_state(ctm_ctx* ctx, double* host, size_t n);
/* As ctm_get_state, into device memory (n doubles); synchronises. */
ctm_status ctm_get_state_device(ctm_ctx* ctx, double* dev, size_t n);
ctm_status ctm_set_state(ctm_ctx* ctx, const double* host, size_t n);

/* Per-kernel-class timing of the context's launches, measured with HIP
 * event pairs recorded on the context's stream around every launch.
 * ctm_profile(ctx, 1) clears the records and starts recording; 0 stops.
 * ctm_profile_read synchronises and returns one entry per kernel class that
 * was launched: launches, summed device milliseconds between the event pairs,
 * and the algorithmic flops and bytes of those launches (flops = 2 M N K per
 * GEMM; bytes = one read of each operand and one write of the result). */
typedef struct {
  char name[32];
  int launches;
  double ms;
  double flops;
  double bytes;
} ctm_prof_entry;

ctm_status ctm_profile(ctm_ctx* ctx, int enable);
ctm_status ctm_profile_read(ctm_ctx* ctx, ctm_prof_entry* out, int max_entries, int* n);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of environment solves on one GPU.
 *
 * A server owns one device arena (allocated once, at creation) and
 * max_slots HIP streams.  Submitted requests wait in a queue and are
 * admitted, in submission order, while a slot is free and their footprint
 * (ctm_workspace_bytes of their configuration plus their staged inputs)
 * fits into the free part of the arena, first fit; a request that does not
 * fit does not hold back smaller ones behind it.  A running request is one
 * context on its slot's stream, with C, T, X and Y resident in its
 * workspace; every ctm_server_pump completes the moves that have finished,
 * launches the next move of each request still iterating (so the moves of
 * different requests overlap on the device), retires requests that reached
 * delta < tol at the full environment dimension or their move budget, and
 * admits queued ones.  A request runs exactly the kernels of a solo
 * ctm_converge with the same inputs, so its result does not depend on the
 * other requests.  The server is not thread safe; requests are numbered
 * from 0 in submission order.
 * ------------------------------------------------------------------------- */
typedef struct ctm_server ctm_server;

typedef struct {
  int state;             /* 0 queued, 1 running, 2 done, 3 failed                  */
  int moves;             /* moves made                                             */
  int converged;         /* 1 if delta < tol was reached                           */
  double delta;          /* delta of the last move                                 */
  double kappa;          /* norm per site of the final environment                 */
  double bond_h, bond_v; /* <op> on a horizontal / vertical bond (0 without op)    */
  double t_submit, t_admit, t_done; /* seconds on the server clock                 */
  size_t bytes;          /* arena bytes held while running                         */
} ctm_result;

/* Creates a server with an arena of arena_bytes device bytes and max_slots
 * (1..64) concurrent requests.  CTM_E_NOMEM if the arena cannot be allocated. */
ctm_status ctm_server_create(ctm_server** out, size_t arena_bytes, int max_slots);

/* Waits for and releases everything the server holds. */
void ctm_server_destroy(ctm_server* server);

/* Queues one environment solve.  All inputs are host arrays, copied before
 * the call returns: site_host as site_dev of ctm_init; boundary_host (Dl
 * doubles) or NULL as in ctm_init; X0_host and Yt0_host (4 N k doubles each,
 * as ctm_set_isometries) or both NULL; op_host a d^2 x d^2 bond operator
 * evaluated on both bond directions at the end, or NULL.  The solve stops at
 * delta < tol (full environment dimension) or after max_moves moves.
 * CTM_E_NOMEM if the request could never fit into the arena. */
ctm_status ctm_server_submit(ctm_server* server, const ctm_config* cfg, const double* site_host,
                             const double* boundary_host, const double* X0_host,
                             const double* Yt0_host, const double* op_host, double tol,
                             int max_moves, int* id);

/* Batched moves in the server: from now on, the SI moves of running float64
 * requests with chi * Dl <= max_n are made together through
 * ctm_move_batch_async (one grouped launch per GEMM step over all of them)
 * instead of each on its slot stream with graph replay; 0 (the default)
 * turns it off.  Results do not change (ctm_move_batch gives the bits of
 * ctm_move). */
ctm_status ctm_server_batching(ctm_server* server, int max_n);

/* Non-blocking progress (see above); n_running and n_queued may be NULL. */
ctm_status ctm_server_pump(ctm_server* server, int* n_running, int* n_queued);

/* Snapshot of request id's state and result. */
ctm_status ctm_server_result(const ctm_server* server, int id, ctm_result* out);

/* Error message of a failed request ("" otherwise). */
const char* ctm_server_error(const ctm_server* server, int id);

/* Seconds since the server was created (the clock of the result stamps). */
double ctm_server_clock(const ctm_server* server);

/* ---------------------------------------------------------------------------
 * Adjoint of one SI move (Differentiable fixed point passage, eq. implicit:
 * gradients of CTMRG observables are built from vector-Jacobian products
 * of the single move; unrolled over moves, or iterated at the fixed point).
 *
 * The move (C, T, X, Y^T, A) -> (C', T', X', Y^T') of the context's
 * configuration is recomputed from state_in, with its intermediates kept
 * in ws, and the cotangents are propagated back through every step (unit
 * norms, renormalisation, projectors with the pseudo-inverse, the SVD of
 * rho, the QRs of the subspace steps, every enlarged-corner application,
 * the enlarged corners and the double layer).  The discrete choices of
 * the forward move (QR diagonal signs, the sign rule, the pseudo-inverse
 * mask) are held constant.  Inverse singular-value gaps of rho carry a
 * Lorentzian broadening (1e-12 s_1^2)^2, relevant only for (near-)
 * degenerate pairs.
 *
 * Requirements: d >= 1, proj = SI, prec = F64, stabilized = 1, sym = NONE,
 * and chi_env == chi in state_in (an SI move); otherwise CTM_E_ARG /
 * CTM_E_STATE.  The context's own environment is not read or changed.
 * --------------------------------------------------------------------------- */

/* Device bytes of the adjoint workspace for cfg. */
ctm_status ctm_vjp_workspace_bytes(const ctm_config* cfg, size_t* bytes);

/* All pointers are device memory in the state-vector layout of
 * ctm_state_size (C1..C4, T1..T4, X_0..X_3, Yt_0..Yt_3, 4 counters):
 *  state_in       the move's input state (read);
 *  state_out_bar  cotangents of the move's outputs C', T', X', Y^T'
 *                 (counters ignored) (read);
 *  state_in_bar   cotangents of C, T, X, Y^T (written; counters set to 0);
 *  state_out      the move's output state, or NULL (written);
 *  site_bar       d*D^4 cotangent of the site tensor A, accumulated (+=),
 *                 or NULL;
 *  ws, ws_bytes   caller-owned workspace of ctm_vjp_workspace_bytes bytes.
 * Stream-ordered on the context's stream; returns after it has finished. */
ctm_status ctm_move_vjp(ctm_ctx* ctx, const double* state_in, const double* state_out_bar,
                        double* state_in_bar, double* state_out, double* site_bar, void* ws,
                        size_t ws_bytes);

/* Gradient at a fixed point (Differentiable fixed point passage, eq.
 * implicit): for a converged state x* = F(x*, A) and the cotangent g of an
 * objective's dependence on x*, sums the Neumann series
 *     x_bar    = sum_n (J_x^T)^n g,
 *     site_bar += sum_n J_A^T (J_x^T)^n g      (= J_A^T [I - J_x^T]^-1 g)
 * by repeated reverse passes of the move at x* (its forward move is
 * recomputed once), until |(J_x^T)^n g| <= tol |g| or max_iter passes.
 *  state_star  converged state (device, state layout);
 *  g_bar       cotangent g (device, state layout; counters ignored);
 *  x_bar       the summed cotangent (device, state layout), or NULL;
 *  site_bar    d*D^4, accumulated (+=);
 *  iters, rel_norm  passes made and the final |(J_x^T)^n g| / |g| (may be NULL).
 * Returns CTM_E_NOT_CONVERGED (with the partial sums written) when max_iter
 * passes do not reach tol; the series converges when the move is a
 * contraction at x*. */
ctm_status ctm_fixed_point_vjp(ctm_ctx* ctx, const double* state_star, const double* g_bar,
                               double tol, int max_iter, double* x_bar, double* site_bar,
                               void* ws, size_t ws_bytes, int* iters, double* rel_norm);

/* Bond energy and its gradient (iPEPS section, observables): for the
 * environment C, T of `state` (device, state layout, chi_env == chi) and
 * the site tensor of the context,
 *     e = <op>_H + <op>_V      (two-site reduced density matrices, trace 1),
 * op[(t1 t2), (s1 s2)] a d^2 x d^2 host operator (bra, ket).  Writes e to
 * *e_out (host, may be NULL), de/d(C, T) to state_bar (device, state layout;
 * X, Y^T and counters 0) and adds de/dA to site_bar (device, d*D^4).  The
 * vertical pair is evaluated as the horizontal pair of the network turned
 * by 90 degrees.  Together with ctm_fixed_point_vjp (g = state_bar) this
 * gives the gradient of the converged energy.  ws: ctm_vjp_workspace_bytes. */
ctm_status ctm_energy_vjp(ctm_ctx* ctx, const double* state, const double* op_host, double* e_out,
                          double* state_bar, double* site_bar, void* ws, size_t ws_bytes);

/* The same for any set of bonds, each with its own operator: e = sum over
 * the bonds in the mask `bonds` (CTM_BOND_H = 1, CTM_BOND_V = 2, CTM_BOND_D
 * = 4, CTM_BOND_AD = 8; the bonds of CTM_OBS_BOND_H/V/D/AD) of <op_bond>;
 * H + V + D is the energy of the triangular lattice drawn on the square one
 * (triangular-lattice section), and with one rotated operator per bond that
 * of its spiral ansatz.  ops_host holds one d^2 x d^2 operator (layout of
 * CTM_OBS_BOND_H) per bond of the mask, consecutively in the order H, V, D,
 * AD (popcount(bonds) * d^4 doubles, host).  The diagonal pair is the 2x2
 * plaquette through its four enlarged corners, differentiated by hand
 * (2 d^2 products of N x N matrices forward, 4 d^2 in reverse); the
 * anti-diagonal is the diagonal of the turned network.  ctm_energy_vjp is
 * this call with bonds = 3 and the same operator on both bonds.  CTM_E_ARG
 * for an empty or unknown mask. */
enum { CTM_BOND_H = 1, CTM_BOND_V = 2, CTM_BOND_D = 4, CTM_BOND_AD = 8 };
ctm_status ctm_bond_energy_vjp(ctm_ctx* ctx, const double* state, const double* ops_host, int bonds,
                               double* e_out, double* state_bar, double* site_bar, void* ws,
                               size_t ws_bytes);

/* ---------------------------------------------------------------------------
 * Building blocks of a move, exposed for testing and for callers composing
 * their own loops.  All operate on caller device memory on `stream`.
 * ------------------------------------------------------------------------- */

/* Batched C_i = alpha * op(A_i) * B_i (+ C_i if accumulate), float64 MFMA.
 * A_i is M x K row-major (lda) if trans_a == 0, else stored K x M row-major
 * (lda) and read transposed; B_i is K x N row-major (ldb); C_i is M x N
 * row-major (ldc).  Arrays of `count` device pointers are host arrays. */
ctm_status ctm_gemm_f64(int count, const double* const* A, const double* const* B,
                        double* const* C, int M, int N, int K, int trans_a, long lda,
                        long ldb, long ldc, double alpha, int accumulate, void* stream);

/* The product of ctm_gemm_f64 for the subspace-iteration applications
 * (QR-based projector section: M X and M^T Y^T with thin blocks, N <= 160)
 * and other thin products with long K, with the (192-row tile, 16-wide K
 * slice) space of all `count` problems split into R equal contiguous ranges,
 * R = min(ncu, pairs / 8) for `pairs` (tile, slice) pairs (every range holds
 * at least 8 slices), one per workgroup of 8 wavefronts (one workgroup per
 * CU: 256 on MI355X; 1 <= ncu <= 256), so that no CU idles while another
 * finishes a tile.  Tiles cut by range boundaries are summed from partial
 * tiles in `scratch` (device memory of ctm_gemm_f64_split_scratch_bytes()
 * bytes, owned by the caller, contents not preserved; calls sharing one
 * scratch must be ordered on one stream) by a second kernel in a fixed
 * order: the result is the same on every call.  trans_a is a host array of
 * `count` flags (0 or 1) as in ctm_gemm_f64; C is row-major with leading
 * dimension ldc.  Problems with N <= 128 take 192 x 128 tiles.  The split
 * applies when scratch is non-NULL and 16-byte aligned, N <= 160, K spans at
 * least 16 slices (K > 240), lda is even, the A bases are 16-byte aligned and
 * the B bases 16-byte aligned (even ldb) or 8-byte aligned (odd ldb);
 * otherwise the plain tile kernel runs.  If used_split is non-NULL it
 * receives 1 when the split ran, else 0. */
size_t ctm_gemm_f64_split_scratch_bytes(void);
ctm_status ctm_gemm_f64_split(int count, const double* const* A, const double* const* B,
                              double* const* C, int M, int N, int K, const int* trans_a, long lda,
                              long ldb, long ldc, double alpha, int accumulate, void* scratch,
                              size_t scratch_bytes, int ncu, int* used_split, void* stream);

/* Thin Householder QR of `count` N x k row-major matrices W_i (N >= k), in
 * place: on return W_i holds Q with R_ii >= 0 (QR-based projector section,
 * step 1).  Zero columns get tau = 0 and no division by zero. */
ctm_status ctm_qr_f64(int count, double* const* W, int N, int k, void* stream);

/* ctm_qr_f64 without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and result as ctm_qr_f64 (bit for
 * bit), with their workspace in a static device array of
 * ctm_qr_f64_noalloc_max_bytes() bytes (96 MiB) that each device holds
 * until the process ends; CTM_E_NOMEM when the workspace of (count, N, k)
 * exceeds it (8 blocks of 5184 x 160 need 71 MiB), CTM_E_ARG for shapes
 * without a QR leaf split.  Stream-ordered and asynchronous (no
 * synchronisation; ctm_qr_f64 synchronises).  Every call on a device
 * shares that device's array: calls that may overlap on one device (other
 * streams, other threads) race and must be ordered by the caller.  The
 * array needs no initial contents, so nothing is cleared between calls. */
size_t ctm_qr_f64_noalloc_max_bytes(void);
ctm_status ctm_qr_f64_noalloc(int count, double* const* W, int N, int k, void* stream);

/* Singular value decomposition of `count` n x n row-major matrices
 * (QR-based projector section, step 2): rho_i = u_i diag(s_i) v_i^T with
 * s descending.  u_i and v_i are n x n row-major (columns are the singular
 * vectors); any of them may be NULL for values only. */
ctm_status ctm_svd_f64(int count, const double* const* rho, double* const* u,
                       double* const* s, double* const* v, int n, void* stream);

/* ---------------------------------------------------------------------------
 * Unit cells (End Matter, larger unit-cell CTMRG): an Lx x Ly cell of
 * different site tensors, site (x, y) in column x and row y, periodic.
 * Every site has its own environment C1..C4, T1..T4 (the single-site index
 * conventions; the dimensions of each tensor are its own while the
 * environment grows, chi after it).  One iteration is a left, a top, a right
 * and a bottom move, the latter three being the left move of the cell turned
 * by 90, 180 and 270 degrees.  A left move renormalises column by column:
 * the left cut of every 2 x 2 cluster of a column gets its own projectors
 * from M = Ct3 Ct4 Ct1 Ct2 of the cluster's four enlarged corners (each
 * site's own), then the left environment (C1, T4, C4) of the column moves
 * one column to the right: C1' = P_r (C1 T1), T4' = P_r (T4 a) P_l,
 * C4' = (T3 C4) P_l, each normalised to unit Frobenius norm.
 * Projector kinds per cut: identities while the cut is not larger than chi
 * (CTM_CELL_GROW); randomized SVD: n_si subspace steps from the cut's fixed
 * start blocks (their first rows while the environment grows), which stay
 * unchanged (CTM_CELL_RSVD, the warm-up); subspace iteration on the cut's
 * own blocks, recycled as X v, Y^T u (CTM_CELL_SI, QR-based projector
 * section); the full SVD of M (CTM_CELL_SVD, Standard CTMRG section; also
 * taken when a randomized or SI step cannot run: fewer block rows than k, or
 * an environment still growing).  One stream per cell; every call is
 * synchronous.
 * ------------------------------------------------------------------------- */
typedef struct ctm_cell ctm_cell;

enum { CTM_CELL_RSVD = 0, CTM_CELL_SI = 1, CTM_CELL_SVD = 2, CTM_CELL_GROW = 3 };

typedef struct {
  int Lx, Ly;       /* columns and rows of the cell (1..16)                              */
  int d;            /* physical dimension; 0 = network tensors a given directly          */
  int D;            /* virtual bond dimension of A, or leg dimension of a when d == 0    */
  int chi;          /* environment bond dimension; chi >= Dl (= D^2, or D when d == 0)   */
  int p;            /* oversampling; k = min(chi + p, chi Dl) <= 192                     */
  int n_si;         /* subspace steps per cut and move (>= 0)                            */
  int stabilized;   /* 1: orthonormalise after M and after M^T; 0: only after M^T M      */
  double pinv_rtol; /* s_i <= pinv_rtol * s_1 gives s_i^-1/2 := 0                        */
} ctm_cell_config;

/* Device bytes ctm_cell_create allocates for cfg. */
ctm_status ctm_cell_workspace_bytes(const ctm_cell_config* cfg, size_t* bytes);

/* Creates a cell.  sites_dev: Lx*Ly site tensors in device memory, site
 * (x, y) at index y*Lx + x, each A[s, u, l, d, r] (d*D^4 doubles; the double
 * layer a = sum_s A A is formed on the device, iPEPS section) or, when
 * d == 0, the network tensor a[u, l, d, r] (D^4 doubles).  boundary_dev:
 * Lx*Ly*4*Dl doubles in device memory, the vectors that close leg u, l, d, r
 * (in that order) of each site when it forms part of a neighbour's initial
 * environment (every tensor of site (x, y) is the neighbour in its direction
 * with its outer legs closed), or NULL for the ket-bra delta vectors (d > 0)
 * or all-ones vectors (d == 0).  The initial environment is normalised and
 * its corner spectra recorded.  Inputs are copied; the caller keeps them.
 * CTM_E_SHAPE / CTM_E_ARG for invalid configurations, CTM_E_NOMEM when the
 * workspace (ctm_cell_workspace_bytes) cannot be allocated. */
ctm_status ctm_cell_create(ctm_cell** out, const ctm_cell_config* cfg, const double* sites_dev,
                           const double* boundary_dev);
void ctm_cell_destroy(ctm_cell* cell);
/* Last error message recorded on the cell, or "" if none. */
const char* ctm_cell_last_error(const ctm_cell* cell);

/* Start blocks of every cut (device memory, copied): X and Y^T, each
 * [4 directions][Lx*Ly cuts][chi*Dl][k] row-major; cut (x', y') of direction
 * d is the left cut of cluster (x', y') of the cell turned d times, at index
 * y'*Lx' + x' with Lx' = Lx for d = 0, 2 and Ly for d = 1, 3 (one turn puts
 * site (x, y) of a cell of width w at (y, w - 1 - x)). */
ctm_status ctm_cell_set_blocks(ctm_cell* cell, const double* X_dev, const double* Yt_dev);

/* One iteration (left, top, right, bottom moves) with projectors of the
 * given kind (CTM_CELL_RSVD, CTM_CELL_SI or CTM_CELL_SVD; see above; an SI
 * iteration after one of another kind starts from the start blocks).
 * *delta (may be NULL): the largest over sites and corners of
 * |s_new - s_old|_2 of the unit-norm corner spectra zero-padded to chi
 * (QR-based projector section, step 4).  CTM_E_STATE without start blocks
 * (RSVD, SI); CTM_E_NUMERIC on a zero or non-finite norm (the environment is
 * then undefined). */
ctm_status ctm_cell_iterate(ctm_cell* cell, int mode, double* delta);

/* Iterations until convergence: warm-up iterations of kind warm_mode
 * (CTM_CELL_RSVD or CTM_CELL_SVD) while fewer than `warmup` iterations were
 * made or some site's C1 has fewer than chi rows, then CTM_CELL_SI
 * iterations until delta < tol or max_iter iterations in all.  *iters: the
 * iterations made; deltas[i] and kinds[i] (may be NULL, else max_iter
 * entries): delta and kind of iteration i.  CTM_E_NOT_CONVERGED when the
 * budget ran out (the environment stays valid). */
ctm_status ctm_cell_run(ctm_cell* cell, int warmup, int warm_mode, double tol, int max_iter,
                        int* iters, double* deltas, int* kinds);

/* Doubles of the host environment layout: per site (index y*Lx + x) the
 * corners C1..C4, each in a chi x chi slot, then the edges T1..T4, each in a
 * chi x Dl x chi slot, every tensor row-major at the start of its slot with
 * its own dimensions (zeros after it). */
ctm_status ctm_cell_env_size(const ctm_cell* cell, size_t* n);
/* Copies the environment to host memory (n doubles) and its dimensions to
 * dims (16 ints per site: rows, cols of C1..C4, then in, out of T1..T4). */
ctm_status ctm_cell_get_env(ctm_cell* cell, double* host, size_t n, int* dims);
/* Replaces the environment (dimensions 1..chi and consistent around every
 * corner), records its corner spectra; the next SI iteration starts from
 * the start blocks. */
ctm_status ctm_cell_set_env(ctm_cell* cell, const double* host, size_t n, const int* dims);
/* Copies the current blocks of every cut (the recycled ones after SI
 * iterations; layout of ctm_cell_set_blocks) to host memory. */
ctm_status ctm_cell_get_blocks(ctm_cell* cell, double* X_host, double* Yt_host);

/* State vector of a cell whose environment has dimension chi (device
 * memory, float64): per site (index y*Lx + x) C1..C4 (chi x chi each) then
 * T1..T4 (chi x Dl x chi each), then X and then Y^T of every cut in the
 * layout of ctm_cell_set_blocks.  get: the environment and the blocks the
 * next SI iteration starts from (CTM_E_STATE while the environment is still
 * growing); set: replaces both, and the next SI iterations continue from
 * these blocks.  Both synchronise. */
ctm_status ctm_cell_state_size(const ctm_cell* cell, size_t* n);
ctm_status ctm_cell_get_state_device(ctm_cell* cell, double* dev, size_t n);
ctm_status ctm_cell_set_state_device(ctm_cell* cell, const double* dev, size_t n);

/* Vector-Jacobian product of one SI iteration of the cell (Differentiable
 * fixed point passage, eq. implicit: gradients are built from the VJPs of
 * single iterations; unrolling them gives the gradient of an energy after a
 * number of iterations).  The iteration is recomputed from state_in (device,
 * ctm_cell_state_size doubles, every cut an SI cut with the state's own
 * blocks), and state_out receives its result (may be NULL).  With
 * state_out_bar (the cotangent of the output state, device) the cotangent
 * of state_in is written to state_in_bar (device) and that of the site
 * tensors added to site_bar (device, Lx*Ly*d*D^4 doubles, or the network
 * tensors' Lx*Ly*D^4 when d == 0; may be NULL).  Discrete choices of the
 * iteration (QR diagonal signs, the sign rule, the pseudo-inverse mask) are
 * held fixed.  The intermediates live in device memory the cell allocates
 * on the first call and keeps (about 40 x 4 chi^2 Dl^4 bytes per cut of an
 * iteration for the corners and their cotangents); CTM_E_NOMEM if it cannot.
 * Synchronises; the cell's own environment is not changed. */
ctm_status ctm_cell_move_vjp(ctm_cell* cell, const double* state_in, const double* state_out_bar,
                             double* state_in_bar, double* site_bar, double* state_out);

/* Energy per site of the cell's state (device, as above; its blocks are not
 * read): e = (1 / (Lx Ly)) sum over the sites (x, y) and over the bonds in
 * the mask `bonds` (1: horizontal to (x+1, y), 2: vertical to (x, y+1),
 * 4: diagonal to (x+1, y+1)) of <op_b> from the two-site reduced density
 * matrix (iPEPS section, observables; the diagonal bond on the 2 x 2
 * plaquette of the four enlarged corners).  ops_host: three d^2 x d^2
 * operators op[(t1 t2), (s1 s2)] (bra, ket) for h, v, d in turn (host
 * memory; those outside the mask are not read).  With state_bar and/or
 * site_bar (device, may be NULL) the gradient: state_bar is written (the
 * blocks' part zero), site_bar accumulated.  Needs d > 0.  Synchronises. */
ctm_status ctm_cell_energy_vjp(ctm_cell* cell, const double* state, const double* ops_host,
                               int bonds, double* e_out, double* state_bar, double* site_bar);

/* ---------------------------------------------------------------------------
 * Self-checks of the adjoint's building blocks (test infrastructure for the
 * cell adjoint): each runs one operation of the reverse-mode tape on the
 * default stream, seeds the cotangent of its output and returns the output
 * and the input cotangents (device memory throughout, synchronous).
 *
 * GEMM with the library's descriptor: dims = {M, N, K, transA, cdiv_m,
 * cdiv_n, nbatch}, strides = {lda, ldb, cs_m1, cs_m0, cs_n1, cs_n0, a_bs,
 * b_bs, c_bs}; C (nC doubles, zero where the map writes nothing) = alpha
 * op(A) B; Abar, Bbar receive the cotangents for the output cotangent Cbar.
 * QR: Q_j = thin Householder QR of H_j (R_jj >= 0), count blocks n x k in a
 * row; Hbar for Qbar.  Projector factors: rho (k x k) and the sign source
 * Yt (nrows x k) give outs = [us, vs (k x k each), vsc, usc (k x keep
 * each)] (see the QR-based projector section), bars in the same layout give
 * rhobar.  Normalisation: count tensors of n[t] doubles in a row, y = x / |x|
 * each; xbar for ybar. */
ctm_status ctm_tape_check_gemm(const int* dims, const long* strides, double alpha, const double* A,
                               long nA, const double* B, long nB, double* C, long nC,
                               const double* Cbar, double* Abar, double* Bbar);
ctm_status ctm_tape_check_qr(int count, int n, int k, const double* H, double* Q, const double* Qbar,
                             double* Hbar);
ctm_status ctm_tape_check_svdproj(int k, int keep, int nrows, double rtol, const double* rho,
                                  const double* Yt, double* outs, const double* bars,
                                  double* rhobar);
ctm_status ctm_tape_check_normalize(int count, const long* n, const double* x, double* y,
                                    const double* ybar, double* xbar);

#ifdef __cplusplus
}
#endif

#endif /* SICTM_CTM_H */
