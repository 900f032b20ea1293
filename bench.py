"""Benchmark of one SI-CTMRG move on one MI355X (prints one JSON line).

Workload (the D=6, chi=144 precision configuration): single-site real iPEPS,
d=2, D=6 (double-layer bond 36), chi=144, p=16 (k=160), n_si=2 stabilised
subspace steps per move, enlarged corners of 5184 x 5184.  Site tensor:
product state (1,0) on every leg plus 0.1 * iid U[-1,1] noise (seed 3); start
blocks iid N(0,1) (seeds 40+b and 50+b).  A "step" is one full four-direction
SI move (enlarged corners, subspace iteration with Householder QRs, rho and
its SVD, projectors, renormalisation, normalisation and the convergence
measure), timed with inputs resident in HBM.

Also reported, in the same JSON line:
  * roofline of the dominant kernel (the enlarged-corner applications of the
    subspace iteration) from HIP events recorded around every launch of it on
    the library's stream during the timed region;
  * the full-SVD CTMRG move on the same GPU (the four 5184 x 5184 M_b formed
    with the library's GEMM and decomposed with rocSOLVER's QR-iteration
    dgesvd, the fastest of its dense SVDs that is accurate for these
    matrices: dgesdd is faster but returns wrong weak directions once
    s_chi / s_1 is far below 1e-8, as here), timed over --svd-moves moves
    from the same environment;
  * the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                                      # GB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(D=6, chi=144, p=16, seed=3):
    import synth as S
    A = S.product_plus_noise_site(2, D, seed)
    N, k = chi * D * D, min(chi + p, chi * D * D)
    X = np.stack([S.gaussian_block(N, k, 40 + b) for b in range(4)])
    Y = np.stack([S.gaussian_block(N, k, 50 + b) for b in range(4)])
    return A, X, Y


def measured_traffic(args):
    """HBM bytes per SI-application launch from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy), or None when the GEMM
    source or the workload differs from the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "si_apply_traffic.json")
    if not os.path.exists(path) or args.prec != "f64" or (args.D, args.chi, args.p) != (6, 144, 16):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2607_15158_amd", "csrc", "gemm.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["gemm_hip_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def measured_mfma_util(args):
    """MFMA busy fraction (%) of the SI-application kernel from the committed
    counter pass (MfmaUtil), or None when the GEMM source or the workload
    differs from the one it was taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "si_apply_mfma.json")
    if not os.path.exists(path) or args.prec != "f64" or (args.D, args.chi, args.p) != (6, 144, 16):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2607_15158_amd", "csrc", "gemm.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["gemm_hip_sha256"]:
        return None
    return rec["mfma_util_pct"]


def cpu_baseline(args, A, X, Y):
    """Times the FP64 oracle on one whole SI move of this workload.

    The sample is one full move (n_si stabilised subspace steps): the four
    enlarged corners, the SI projectors of the four bonds (QRs, rho, its
    SVD, the sign rule, the projectors and the recycled blocks), the
    renormalisation of the four corners and the four edges and the
    normalisation, from a seeded random environment of the move's shapes
    (the cost does not depend on the values), with the benchmark's site
    tensor and start blocks.
    """
    import oracle as O
    import synth as S
    threads = len(os.sched_getaffinity(0))
    chi, D = args.chi, args.D
    Dl = D * D
    a = O.double_layer(A)
    env = O.Env([S.gaussian_block(chi, chi, 60 + i) for i in range(4)],
                [S.gaussian_block(chi * Dl, chi, 70 + i).reshape(chi, Dl, chi) for i in range(4)])
    si = O.SIState(list(X), list(Y))
    t0 = time.perf_counter()
    _, info = O.ctm_move(env, a, chi, "si", si, n_si=args.n_si, eps=args.pinv_rtol)
    dt = time.perf_counter() - t0
    assert info["mode"] == "si"
    return {"value": round(1.0 / dt, 5), "unit": "moves/s", "cores": threads, "kind": "oracle",
            "sample": f"one whole SI move (n_si={args.n_si}, stabilised) of the same D={D}, "
                      f"chi={chi} workload from a seeded random environment: {dt:.1f} s, numpy "
                      f"float64 on {threads} threads"}


def serving(args, n_requests):
    """Serving workload: mixed (D, chi) environment solves, Poisson arrivals.

    Request i: D uniform in {3,4,5,6}, chi uniform in {D^2, 2D^2, 3D^2}
    (default_rng(4)), site tensor as in the main workload with seed 4000+i,
    p = max(4, ceil(0.15 chi)), n_si = 2, tol 1e-10, at most --serve-moves moves,
    Heisenberg bond energy evaluated at the end.  Phase 1 submits every request
    at t = 0 and measures the service rate mu; phase 2 replays them with
    Poisson arrivals at lambda = 0.7 mu (inter-arrival times from
    default_rng(44)) and reports latency p50/p99 and throughput.
    """
    import math
    import paper_2607_15158_amd as P
    import synth as S
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(n_requests):
        D = int(rng.choice([3, 4, 5, 6]))
        chi = int(rng.choice([D * D, 2 * D * D, 3 * D * D]))
        p = max(4, math.ceil(0.15 * chi))
        cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=2, svd_driver="gesvd", growth="si")
        reqs.append((cfg, S.product_plus_noise_site(2, D, 4000 + i)))
    h = S.heisenberg_bond()

    def run(arrivals, batch_n):
        srv = P.Server(arena_bytes=args.serve_arena_gb << 30, max_slots=args.serve_slots,
                       batch_max_n=batch_n)
        t0 = srv.clock()
        ids, nxt, done_log = [None] * len(reqs), 0, 0
        while True:
            now = srv.clock() - t0
            while nxt < len(reqs) and arrivals[nxt] <= now:
                cfg, A = reqs[nxt]
                ids[nxt] = srv.submit(cfg, A, op=h, tol=1e-10, max_moves=args.serve_moves)
                nxt += 1
            running, queued = srv.pump()
            if nxt == len(reqs) and running == 0 and queued == 0:
                break
            fin = sum(1 for r in ids if r is not None and srv.result(r)["state"] in ("done", "failed"))
            if fin >= done_log + max(1, len(reqs) // 8):
                done_log = fin
                log(f"  serving: {fin}/{len(reqs)} done, {running} running, {queued} queued, "
                    f"t = {srv.clock() - t0:.1f} s")
        res = [srv.result(r) for r in ids]
        span = max(r["t_done"] for r in res) - t0
        srv.close()
        return res, span

    out = {"metric": "serving latency p50/p99 of mixed (D, chi) environment solves",
           "unit": "requests/s", "n_gpus": 1, "requests": len(reqs), "slots": args.serve_slots,
           "arena_gb": args.serve_arena_gb, "max_moves": args.serve_moves, "dtype": "f64",
           "data": "synthetic", "higher_is_better": True}
    results = {}
    modes = (("per_stream", 0), ("batched", args.serve_batch_n))
    for name, batch_n in modes:
        log(f"serving ({name}) phase 1: {len(reqs)} requests at t = 0")
        res1, span1 = run([0.0] * len(reqs), batch_n)
        mu = len(reqs) / span1
        lam = 0.7 * mu
        gaps = np.random.default_rng(44).exponential(1.0 / lam, size=len(reqs))
        arrivals = np.cumsum(gaps) - gaps[0]
        log(f"serving ({name}) phase 2: Poisson arrivals at lambda = {lam:.3f} req/s "
            f"(mu = {mu:.3f})")
        res2, span2 = run(list(arrivals), batch_n)
        lat = np.array([r["t_done"] - r["t_submit"] for r in res2])
        same = all(a["kappa"] == b["kappa"] and a["bond_h"] == b["bond_h"] and
                   a["moves"] == b["moves"] for a, b in zip(res1, res2))
        results[name] = (res1, res2)
        out[name] = {"value": round(len(reqs) / span2, 4), "mu_req_per_s": round(mu, 4),
                     "lambda_req_per_s": round(lam, 4),
                     "p50_s": round(float(np.percentile(lat, 50)), 4),
                     "p99_s": round(float(np.percentile(lat, 99)), 4),
                     "mean_moves": round(float(np.mean([r["moves"] for r in res2])), 2),
                     "converged": int(sum(r["converged"] for r in res2)),
                     "failed": int(sum(r["state"] != "done" for r in res2)),
                     "results_identical_across_phases": bool(same),
                     "batch_max_n": batch_n}
        log(f"serving ({name}): mu {mu:.3f} req/s, p50 {out[name]['p50_s']} s, "
            f"p99 {out[name]['p99_s']} s")
    a, b = results["per_stream"][0], results["batched"][0]
    out["batched_results_identical_to_per_stream"] = bool(all(
        x["kappa"] == y["kappa"] and x["bond_h"] == y["bond_h"] and x["moves"] == y["moves"]
        for x, y in zip(a, b)))
    out["value"] = out["batched"]["value"]
    return out


def unit_cell(args):
    """The 3x3 unit cell of nine different site tensors at D=5, chi=100,
    p=5 (the paper's variational optimisation workload, larger unit-cell
    passage of the End Matter): randomized-SVD warm-up iterations, timed SI
    iterations (left, top, right and bottom moves, column by column), and one
    optimisation step: the triangular-lattice energy per site after
    ``args.cell_moves`` SI iterations and its gradient with respect to the
    nine site tensors through the unrolled iterations (checkpoints at every
    iteration boundary, the adjoint of every iteration recomputed from its
    checkpoint)."""
    import torch
    import paper_2607_15158_amd as P
    import synth as S

    dev = torch.device("cuda", 0)
    Lx, Ly, D = 3, 3, 5
    cfg = P.CellConfig(Lx, Ly, d=2, D=D, chi=100, p=5, n_si=2)
    sites = np.stack([S.product_plus_noise_site(2, D, 40 + 7 * (s % Lx) + 3 * (s // Lx), noise=0.05)
                      for s in range(cfg.ns)])
    X = np.zeros((4, cfg.ns, cfg.N, cfg.k))
    Y = np.zeros_like(X)
    for d in range(4):
        lx, ly = (Lx, Ly) if d % 2 == 0 else (Ly, Lx)
        for y in range(ly):
            for x in range(lx):
                X[d, y * lx + x] = S.gaussian_block(cfg.N, cfg.k, 31 + 100 * d + 10 * x + y)
                Y[d, y * lx + x] = S.gaussian_block(cfg.N, cfg.k, 1031 + 100 * d + 10 * x + y)
    st_sites = torch.from_numpy(sites).to(dev)
    c = P.Cell(cfg, st_sites)
    c.set_blocks(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
    del X, Y
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        c.iterate("rsvd")
    t_warm = (time.perf_counter() - t) / 3
    n_si = 10
    t = time.perf_counter()
    deltas = [c.iterate("si") for _ in range(n_si)]
    t_si = (time.perf_counter() - t) / n_si
    state = c.get_state_device()
    c.close()
    h = S.heisenberg_bond()
    ops = {"h": h, "v": h, "d": h}
    out = {"workload": f"{Lx}x{Ly} unit cell, nine d=2 D={D} site tensors, chi=100, p=5, n_si=2, "
                       f"N={cfg.N}; iteration = left, top, right, bottom moves",
           "warmup_iteration_s": round(t_warm, 4), "si_iteration_s": round(t_si, 4),
           "si_deltas": [float(f"{d:.3e}") for d in deltas]}
    if args.cell_moves > 0:
        x = st_sites.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        e = P.unrolled_cell_energy(x, cfg, ops, state, args.cell_moves)
        e.backward()
        torch.cuda.synchronize()
        t_opt = time.perf_counter() - t
        out.update({"optimisation_step_iterations": args.cell_moves,
                    "optimisation_step_s": round(t_opt, 3),
                    "energy_per_site": e.item(),
                    "gradient_norm": float(x.grad.norm())})
        log(f"unit cell: SI iteration {t_si:.3f} s; energy {e.item():.10f} and its gradient "
            f"through {args.cell_moves} iterations in {t_opt:.1f} s")
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=144)
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--n-si", type=int, default=2)
    ap.add_argument("--recycle-sin2", type=float, default=0.0,
                    help="> 0: stop the subspace steps once the kept subspaces of successive "
                         "moves align to this mean sin^2 (the paper's recycling); 0: n_si "
                         "steps every move")
    ap.add_argument("--min-si-moves", type=int, default=3)
    ap.add_argument("--converge-tol", type=float, default=1e-10,
                    help="> 0: time the SI environment from the initial one until delta < this "
                         "(with randomized growth, and from the shared full-SVD growth move) and "
                         "set it against the full-SVD moves run from the same growth move")
    ap.add_argument("--converge-max", type=int, default=200)
    ap.add_argument("--opt-moves", type=int, default=10,
                    help="> 0: time one optimisation step (the energy after this many SI moves "
                         "from the state after the timed moves, and its site-tensor gradient by "
                         "the unrolled adjoint with move-boundary checkpoints)")
    ap.add_argument("--vjp", type=int, default=3,
                    help="time this many adjoints of the move (ctm_move_vjp) at the state after "
                         "the timed moves (0: skip)")
    ap.add_argument("--opt-energy", default="triangular", choices=["triangular", "square"],
                    help="energy of the optimisation step: the triangular lattice (spiral "
                         "ansatz, h + v + diagonal; the paper's workload) or the square "
                         "lattice's h + v")
    ap.add_argument("--no-obs", action="store_true",
                    help="skip the observables (bond values, correlation lengths)")
    ap.add_argument("--xi-iters", type=int, default=30,
                    help="block iterations of the correlation-length observable")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16", "bf16x3"],
                    help="contraction precision (bf16x3: split bfloat16, three bf16 products "
                         "per contraction; its roofline counts the three products)")
    ap.add_argument("--pinv-rtol", type=float, default=1e-12)
    ap.add_argument("--svd-moves", type=int, default=1,
                    help="full-SVD comparator moves from the state after the growth move (0: skip)")
    ap.add_argument("--svd-driver", default="gesvd", choices=["gesvd", "gesdd", "gesvdx"],
                    help="dense SVD of the growth move and of the full-SVD comparator (gesvd: "
                         "accurate; gesdd: fast but its weak directions are noise at this "
                         "conditioning; gesvdx: accurate, slow)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="copy 1 GiB device to device once before the moves (the reference "
                         "dispatch for scaling hardware byte counters)")
    ap.add_argument("--graphs", action="store_true",
                    help="run the moves on a dedicated stream with SI moves replayed from "
                         "captured HIP graphs (the timed loop is then not profiled; the "
                         "roofline comes from a profiled pass of 5 eager moves after it)")
    ap.add_argument("--random-env", action="store_true",
                    help="start from a seeded random environment of full dimension instead of "
                         "the growth move (no rocSOLVER call; used for counter runs)")
    ap.add_argument("--serving", type=int, default=0,
                    help="run the serving workload with this many requests instead")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-arena-gb", type=int, default=96)
    ap.add_argument("--serve-moves", type=int, default=60)
    ap.add_argument("--serve-batch-n", type=int, default=1296,
                    help="requests with chi * D^2 up to this move together in grouped launches "
                         "(ctm_move_batch) in the batched serving mode")
    ap.add_argument("--cell-moves", type=int, default=30,
                    help="SI iterations of the unit-cell optimisation step (3x3 cell, D=5, "
                         "chi=100; -1: skip the unit-cell sub-measurement, 0: time the "
                         "iterations only)")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the serving sub-measurement of the default run (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_15158_amd as P

    torch.cuda.set_device(0)
    if args.serving:
        print(json.dumps(serving(args, args.serving)), flush=True)
        return
    dev = torch.device("cuda", 0)
    if args.copy_calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read, 1 GiB written")
        del src, dst
    A, X, Y = workload(args.D, args.chi, args.p)
    growth_s = None
    cfg = P.Config(d=2, D=args.D, chi=args.chi, p=args.p, n_si=args.n_si, proj="si",
                   prec=args.prec, stabilized=1, pinv_rtol=args.pinv_rtol,
                   svd_driver=args.svd_driver, recycle_sin2=args.recycle_sin2,
                   min_si_moves=args.min_si_moves)
    log(f"config d=2 D={args.D} chi={args.chi} k={cfg.k} N={cfg.N} prec={args.prec}; "
        f"workspace {P.workspace_bytes(cfg) / 2**30:.2f} GiB")
    stream = torch.cuda.Stream() if args.graphs else None
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(dev), stream=stream)
    ctx.set_isometries(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
    if args.random_env:
        import synth as S
        Dl = args.D * args.D
        C = [S.gaussian_block(args.chi, args.chi, 60 + i) for i in range(4)]
        T = [S.gaussian_block(args.chi * Dl, args.chi, 70 + i).reshape(args.chi, Dl, args.chi)
             for i in range(4)]
        ctx.set_state(ctx.pack_state(C, T, X, Y))
        log("seeded random environment of full dimension (no growth move)")
    else:
        t = time.perf_counter()
        info = ctx.move()                  # growth move (full SVD of the first M_b)
        growth_s = time.perf_counter() - t
        log(f"growth move mode={info['mode']} chi_env={info['chi_env']} {growth_s:.2f} s")
    state_after_growth = ctx.get_state()
    for i in range(args.warmup):
        t = time.perf_counter()
        info = ctx.move()
        log(f"warmup {i}: mode={info['mode']} n_si={info['n_si']} delta={info['delta']:.3e} "
            f"sin2={info['sin2']:.2e} {(time.perf_counter() - t) * 1e3:.1f} ms")

    if args.graphs:
        ctx.use_graphs(True)
    else:
        ctx.profile(True)
    torch.cuda.synchronize()
    lat, steps_used = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        info = ctx.move()                  # synchronises (reads delta)
        lat.append(time.perf_counter() - ts)
        steps_used.append(info["n_si"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if args.graphs:
        ctx.profile(True)                  # eager moves: events around every launch
        for i in range(5):
            ctx.move()
        prof = ctx.profile_read()
        ctx.profile(False)
        prof_steps = 5
    else:
        prof = ctx.profile_read()
        ctx.profile(False)
        prof_steps = args.steps
    ms_step = 1e3 * elapsed / args.steps
    log(f"timed {args.steps} moves: {ms_step:.2f} ms/move, last delta {info['delta']:.3e}")
    for e in prof:
        log(f"  {e['name']:16s} launches {e['launches']:5d}  {e['ms']:9.2f} ms  "
            f"{e['flops'] / max(e['ms'], 1e-9) / 1e9:8.2f} TFLOP/s")

    dom = next(e for e in prof if e["name"] == "si_apply")
    per_launch_ms = dom["ms"] / dom["launches"]
    flops_launch = dom["flops"] / dom["launches"]
    bytes_launch = dom["bytes"] / dom["launches"]
    achieved = flops_launch / (per_launch_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": "si_apply (8 enlarged-corner applications per launch)",
                "achieved": round(achieved, 2), "peak": PEAK[args.prec], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK[args.prec], 4), "traffic": measured_traffic(args),
                "launch_ms": round(per_launch_ms, 4), "flops_per_launch": flops_launch,
                "algorithmic_GBps": round(bytes_launch / (per_launch_ms * 1e-3) / 1e9, 1),
                "mfma_busy_pct_counters": measured_mfma_util(args)}
    total_flops = sum(e["flops"] for e in prof) / prof_steps
    breakdown = {e["name"]: round(e["ms"] / prof_steps, 3) for e in prof}

    vjp = None
    if args.vjp > 0 and args.prec == "f64":
        st = torch.from_numpy(ctx.get_state()).to(dev)
        bar = torch.randn(st.numel(), dtype=torch.float64, device=dev,
                          generator=torch.Generator(device=dev).manual_seed(7))
        ctx.move_vjp(st, bar, want_out=False)               # workspace and warm-up
        torch.cuda.synchronize()
        tv = []
        for _ in range(args.vjp):
            t1 = time.perf_counter()
            ctx.move_vjp(st, bar, want_out=False)           # returns after the stream finished
            tv.append(time.perf_counter() - t1)
        vjp = {"ms_per_vjp": round(1e3 * float(np.median(tv)), 2), "count": args.vjp,
               "ratio_to_move": round(1e3 * float(np.median(tv)) / ms_step, 2),
               "what": "reverse pass of one SI move incl. its recomputed forward (tape)"}
        log(f"adjoint: {vjp['ms_per_vjp']} ms per move VJP ({vjp['ratio_to_move']}x the move)")
        import synth as S
        h = S.heisenberg_bond()
        vjp["energy_vjp_ms"] = {}
        for bonds in ("hv", "hvd"):
            ctx.energy_vjp(st, h, bonds=bonds)                  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.energy_vjp(st, h, bonds=bonds)
            vjp["energy_vjp_ms"][bonds] = round(1e3 * (time.perf_counter() - t1), 2)
        log(f"energy gradient: {vjp['energy_vjp_ms']} ms (nearest-neighbour bonds; with the "
            f"diagonal, the triangular lattice)")

    obs = None
    if args.prec == "f64" and not args.no_obs:
        import synth as S
        h = S.heisenberg_bond()
        kinds = (("bond_h", P.OBS_BOND_H), ("bond_v", P.OBS_BOND_V), ("bond_d", P.OBS_BOND_D))
        ctx.observable(P.OBS_BOND_D, h)                      # first call: code paths warm
        obs = {"what": "Heisenberg bond values of the final environment and the time of one "
                       "call each (the diagonal contracts the 2x2 plaquette through its four "
                       "enlarged corners, 2 d^2 products of N x N matrices)"}
        for name, kind in kinds:
            t1 = time.perf_counter()
            val = ctx.observable(kind, h)[0]
            obs[name] = {"value": val, "ms": round(1e3 * (time.perf_counter() - t1), 2)}
        for direction in "hv":
            t1 = time.perf_counter()
            xi, r2 = ctx.correlation_length(direction, iters=args.xi_iters)
            obs[f"xi_{direction}"] = {"value": xi, "l2_over_l1": r2, "iterations": args.xi_iters,
                                      "ms": round(1e3 * (time.perf_counter() - t1), 2)}
        kinds = kinds + (("xi_h", None), ("xi_v", None))
        log("observables: " + ", ".join(f"{k} {obs[k]['value']:.8f} ({obs[k]['ms']} ms)"
                                        for k, _ in kinds))

    opt = None
    if args.opt_moves > 0 and args.prec == "f64":
        import synth as S
        st0 = ctx.get_state_device()
        At = torch.from_numpy(A).to(dev).requires_grad_(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if args.opt_energy == "triangular":
            th = 2 * np.pi / 3
            op_opt = P.spiral_bond_operators(S.heisenberg_bond(), {"h": th, "v": th, "d": 2 * th})
        else:
            op_opt = S.heisenberg_bond()
        e_opt = P.unrolled_energy(At, cfg, op_opt, st0, args.opt_moves)
        e_opt.backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        opt = {"moves": args.opt_moves, "seconds": round(dt, 3),
               "energy": ("triangular lattice, spiral ansatz: h + v + d with rotated bond operators"
                          if args.opt_energy == "triangular" else "square lattice: h + v"),
               "what": "energy after the moves and its gradient wrt the site tensor (unrolled "
                       "adjoint, checkpoints at move boundaries, moves recomputed in reverse)"}
        log(f"optimisation step ({args.opt_moves} unrolled moves, forward + backward): {dt:.2f} s")
        del At, e_opt

    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    svd = None
    if args.svd_moves > 0 and not args.random_env:
        # full-SVD CTMRG moves from the state after the (shared) growth move
        cfg_s = P.Config(d=2, D=args.D, chi=args.chi, p=args.p, n_si=args.n_si, proj="svd",
                         prec="f64", stabilized=1, pinv_rtol=args.pinv_rtol,
                         svd_driver=args.svd_driver)
        cs = P.Ctm(cfg_s, torch.from_numpy(A).to(dev))
        cs.set_state(state_after_growth)
        tt, deltas = [], []
        for i in range(args.svd_moves):
            t = time.perf_counter()
            inf = cs.move()
            tt.append(time.perf_counter() - t)
            deltas.append(inf["delta"])
            log(f"full-SVD move {i}: {tt[-1]:.2f} s, delta {inf['delta']:.3e}")
        svd = {"moves_per_s": round(1.0 / float(np.mean(tt)), 4),
               "ms_per_move": round(1e3 * float(np.mean(tt)), 1), "moves": args.svd_moves,
               "deltas": deltas, "start": "the state after the growth move",
               "solver": f"rocsolver_d{args.svd_driver} on 4 x ({cfg.N} x {cfg.N})"}
        cs.close()
        del cs
        torch.cuda.empty_cache()

    conv = None
    if args.converge_tol > 0 and not args.random_env and args.prec == "f64":
        # time per converged environment (delta < tol at chi_env = chi) from the
        # same initial environment: SI-CTMRG with its own randomized (SI)
        # growth, and SI from the full-SVD growth move the comparator shares
        tol = args.converge_tol
        conv = {"tol": tol, "max_moves": args.converge_max}
        runs = (("si_randomized_growth", "si", None), ("si_after_svd_growth", "svd", state_after_growth))
        for name, growth, start in runs:
            cfg_c = P.Config(d=2, D=args.D, chi=args.chi, p=args.p, n_si=args.n_si, proj="si",
                             prec="f64", stabilized=1, pinv_rtol=args.pinv_rtol,
                             svd_driver=args.svd_driver, growth=growth)
            cc = P.Ctm(cfg_c, torch.from_numpy(A).to(dev))
            cc.set_isometries(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
            if start is not None:
                cc.set_state(start)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = cc.converge(tol, args.converge_max)
            dt = time.perf_counter() - t
            if start is not None:
                dt += growth_s
            import synth as S
            h = S.heisenberg_bond()
            e = cc.observable(P.OBS_BOND_H, h)[0] + cc.observable(P.OBS_BOND_V, h)[0]
            conv[name] = {"moves": r["moves"] + (1 if start is not None else 0),
                          "seconds": round(dt, 3), "converged": r["converged"],
                          "last_delta": r["delta"], "energy": e, "kappa": cc.kappa()}
            log(f"converged environment ({name}): {conv[name]['moves']} moves, {dt:.2f} s, "
                f"delta {r['delta']:.2e}, energy {e:.12f}")
            cc.close()
            del cc
            torch.cuda.empty_cache()
        if svd is not None:
            done = any(d < tol for d in svd["deltas"])
            t_svd = growth_s + sum(1e-3 * svd["ms_per_move"] for _ in svd["deltas"])
            conv["full_svd"] = {"moves_run": 1 + len(svd["deltas"]), "seconds_run": round(t_svd, 2),
                                "deltas_after_growth": svd["deltas"], "converged": done}
            if not done:
                # not converged after the moves run: its time per converged
                # environment exceeds the time already spent
                conv["ratio_lower_bound_full_svd_over_si"] = {
                    k: round(t_svd / conv[k]["seconds"], 2) for k, _, _ in runs}
                conv["ratio_if_full_svd_needed_as_many_moves_as_si"] = round(
                    (growth_s + (conv["si_after_svd_growth"]["moves"] - 1) * 1e-3 * svd["ms_per_move"])
                    / conv["si_after_svd_growth"]["seconds"], 1)
            log(f"full-SVD CTMRG: {conv['full_svd']}; ratio lower bound "
                f"{conv.get('ratio_lower_bound_full_svd_over_si')}")

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (one SI move) ...")
        cpu = cpu_baseline(args, A, X, Y)
        log(f"CPU oracle: {1.0 / cpu['value']:.1f} s per move on {cpu['cores']} threads")

    serve = None
    if args.serve_requests > 0 and args.prec == "f64":
        serve = serving(args, args.serve_requests)

    cell = None
    if args.cell_moves >= 0 and args.prec == "f64":
        cell = unit_cell(args)


    value = args.steps / elapsed
    out = {
        "metric": "SI-CTMRG iters/s at D=6 chi=144 vs full-SVD on same GPU; MFMA util; p50/p99",
        "value": round(value, 4), "unit": "moves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": f"SI-CTMRG move, single-site iPEPS d=2 D={args.D} chi={args.chi} "
                               f"p={args.p} n_si={args.n_si}, enlarged corner {cfg.N}x{cfg.N}",
                   "D": args.D, "chi": args.chi, "k": cfg.k, "n_si": args.n_si,
                   "contraction_precision": args.prec, "parallelism": "1 GPU",
                   "recycle_sin2": args.recycle_sin2},
        "timed_moves_without_subspace_steps": int(sum(1 for n in steps_used if n == 0)),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "tflops_per_move": round(total_flops / 1e12, 4),
        "tflops_per_s": round(total_flops / (ms_step * 1e-3) / 1e12, 2),
        "phase_ms_per_move": breakdown,
        "roofline": roofline,
        "full_svd_same_gpu": svd,
        "adjoint": vjp,
        "observables": obs,
        "optimisation_step": opt,
        "converged_environment": conv,
        "speedup_vs_full_svd": None if svd is None else round(value / svd["moves_per_s"], 2),
        "serving": serve,
        "unit_cell": cell,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
