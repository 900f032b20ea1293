"""Serving: continuous batching of environment solves through the C ABI.

* asynchronous moves reproduce synchronous ones exactly;
* every request served in a mix (staggered arrivals, several running at
  once, mixed D and chi) gives bit-for-bit the result of its solo run;
* admission never exceeds the arena: with an arena holding two requests at
  most two run at once, and every request still finishes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2607_15158_amd as P  # noqa: E402
import synth as S  # noqa: E402


def request(D, chi, seed, p=4):
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=2, svd_driver="gesvd", growth="si")
    A = S.product_plus_noise_site(2, D, seed, noise=0.3)
    X = np.stack([S.gaussian_block(cfg.N, cfg.k, 100 * seed + b) for b in range(4)])
    Y = np.stack([S.gaussian_block(cfg.N, cfg.k, 100 * seed + 10 + b) for b in range(4)])
    return cfg, A, X, Y


def solo(cfg, A, X, Y, tol, max_moves):
    dev = torch.device("cuda", 0)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    ctx.set_isometries(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
    r = ctx.converge(tol, max_moves)
    h = S.heisenberg_bond()
    return {"moves": r["moves"], "delta": r["delta"], "kappa": ctx.kappa(),
            "bond_h": ctx.observable(P.OBS_BOND_H, h)[0],
            "bond_v": ctx.observable(P.OBS_BOND_V, h)[0]}


def test_async_moves_equal_sync_moves():
    cfg, A, X, Y = request(2, 6, 1)
    dev = torch.device("cuda", 0)
    a = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    b = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    for c in (a, b):
        c.set_isometries(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
    for _ in range(5):
        ia = a.move()
        b.move_async()
        ib = None
        while ib is None:
            ib = b.move_poll()
        assert ia == ib
    assert np.array_equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("recycle", [0.0, 1e-3])
def test_graph_replay_matches_eager_moves(recycle):
    """SI moves replayed from captured graphs equal eager moves bit for bit,
    on every replay, with unrelated eager work and synchronisations between
    the replays; with recycling, the moves with and without subspace steps
    (and with the criterion measured) are captured separately."""
    cfg, A, X, Y = request(2, 6, 7)
    cfg.recycle_sin2 = recycle
    dev = torch.device("cuda", 0)
    eager = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    side = torch.cuda.Stream()
    graphed = P.Ctm(cfg, torch.from_numpy(A).to(dev), stream=side)
    for c in (eager, graphed):
        c.set_isometries(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
    graphed.use_graphs(True)
    noise = torch.randn(512, 512, device=dev)
    steps = []
    for n in range(14):
        ie = eager.move()
        ig = graphed.move()
        assert ie == ig, n
        assert np.array_equal(eager.get_state(), graphed.get_state()), n
        if ig["mode"] == 2:
            steps.append(ig["n_si"])
        noise = noise @ noise.T / 512.0            # eager work between replays
        torch.cuda.synchronize()
    assert ig["mode"] == 2
    assert (0 in steps) == (recycle > 0)


def test_mix_equals_solo_runs():
    tol, max_moves = 1e-10, 40
    specs = [(2, 4, 1), (3, 9, 2), (2, 8, 3), (3, 12, 4), (2, 6, 5), (3, 18, 6)]
    reqs = [request(*sp) for sp in specs]
    srv = P.Server(arena_bytes=1 << 30, max_slots=3)
    h = S.heisenberg_bond()
    ids, peak = [], 0
    for i, (cfg, A, X, Y) in enumerate(reqs):
        ids.append(srv.submit(cfg, A, X0=X, Yt0=Y, op=h, tol=tol, max_moves=max_moves))
        for _ in range(3 * i):          # staggered arrivals: others are mid-solve
            run, _ = srv.pump()
            peak = max(peak, run)
    while True:
        run, queued = srv.pump()
        peak = max(peak, run)
        if run == 0 and queued == 0:
            break
    assert peak > 1, "requests never overlapped"
    for rid, (cfg, A, X, Y), sp in zip(ids, reqs, specs):
        got = srv.result(rid)
        assert got["state"] == "done", got
        ref = solo(cfg, A, X, Y, tol, max_moves)
        print(sp, got["moves"], got["kappa"], ref["kappa"])
        for key in ("moves", "delta", "kappa", "bond_h", "bond_v"):
            assert got[key] == ref[key], (sp, key, got[key], ref[key])
    srv.close()


def test_admission_by_arena_footprint():
    specs = [(3, 9, 11), (3, 9, 12), (3, 9, 13), (3, 9, 14)]
    reqs = [request(*sp) for sp in specs]
    ws = P.workspace_bytes(reqs[0][0])
    # room for two requests (workspace + staged inputs), not three
    srv = P.Server(arena_bytes=int(2.6 * ws), max_slots=4)
    ids = [srv.submit(cfg, A, X0=X, Yt0=Y, tol=1e-9, max_moves=15) for cfg, A, X, Y in reqs]
    peak = 0
    while True:
        run, queued = srv.pump()
        peak = max(peak, run)
        if run == 0 and queued == 0:
            break
    assert peak == 2
    for rid in ids:
        r = srv.result(rid)
        assert r["state"] == "done" and r["t_admit"] >= r["t_submit"] and r["t_done"] > r["t_admit"]
    srv.close()


def test_move_batch_equals_solo_moves():
    """ctm_move_batch over contexts of mixed (D, chi): the SI moves of all of
    them run as grouped launches (one per GEMM step) on one stream, the
    growth moves on their own; after every move each batched context holds
    bit for bit the state and move info of a twin moved alone.  The D=6,
    chi=108 context (N = 3888) takes the split SI product, which keeps its
    own launch inside the batch."""
    specs = [(2, 4, 1, 4), (3, 9, 2, 4), (2, 8, 3, 4), (3, 18, 6, 4), (6, 108, 7, 16)]
    dev = torch.device("cuda", 0)
    solo, batched = [], []
    for D, chi, seed, p in specs:
        cfg, A, X, Y = request(D, chi, seed, p)
        for group in (solo, batched):
            c = P.Ctm(cfg, torch.from_numpy(A).to(dev), stream=torch.cuda.Stream())
            c.set_isometries(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev))
            group.append(c)
    modes = []
    for n in range(6):
        want = [c.move() for c in solo]
        got = P.move_batch(batched)
        modes.append([g["mode"] for g in got])
        for i, (a, b) in enumerate(zip(want, got)):
            assert a == b, (n, specs[i], a, b)
        for i, (a, b) in enumerate(zip(solo, batched)):
            assert np.array_equal(a.get_state(), b.get_state()), (n, specs[i])
    assert all(m == 2 for m in modes[-1]), modes
    for c in solo + batched:
        c.close()


def test_server_with_batched_moves_equals_solo_runs():
    """The server with batched moves for every request (ctm_server_batching):
    results bit for bit those of solo ctm_converge runs, as without it."""
    tol, max_moves = 1e-10, 40
    specs = [(2, 4, 1), (3, 9, 2), (2, 8, 3), (3, 12, 4), (2, 6, 5), (3, 18, 6)]
    reqs = [request(*sp) for sp in specs]
    srv = P.Server(arena_bytes=1 << 30, max_slots=4, batch_max_n=1 << 20)
    h = S.heisenberg_bond()
    ids = []
    for i, (cfg, A, X, Y) in enumerate(reqs):
        ids.append(srv.submit(cfg, A, X0=X, Yt0=Y, op=h, tol=tol, max_moves=max_moves))
        for _ in range(2 * i):
            srv.pump()
    while True:
        run, queued = srv.pump()
        if run == 0 and queued == 0:
            break
    for rid, (cfg, A, X, Y), sp in zip(ids, reqs, specs):
        got = srv.result(rid)
        assert got["state"] == "done", got
        ref = solo(cfg, A, X, Y, tol, max_moves)
        for key in ("moves", "delta", "kappa", "bond_h", "bond_v"):
            assert got[key] == ref[key], (sp, key, got[key], ref[key])
    srv.close()
