"""Unit-cell CTMRG on the GPU (ctm_cell_*) against the unit-cell oracle.

The oracle (oracle.multisite) renormalises an Lx x Ly cell direction by
direction and column by column with per-cut projectors; the GPU runs the
same iterations through the C ABI from the same seeded site tensors and
start blocks.  Compared iteration by iteration: every environment tensor of
every site (shapes and elements, through the growth of the environment, the
randomized-SVD warm-up, the full-SVD projectors and the recycled SI
iterations), the recycled blocks and the convergence measure.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import oracle.multisite as M  # noqa: E402
import paper_2607_15158_amd as P  # noqa: E402
import synth as S  # noqa: E402

DEV = torch.device("cuda", 0)


def turned_size(Lx, Ly, d):
    return (Lx, Ly) if d % 2 == 0 else (Ly, Lx)


def start_blocks(Lx, Ly, N, k, seed):
    """Blocks per direction and cut: the oracle's dict and the GPU's
    [4, Lx*Ly, N, k] stack (cut (x', y') at y' * Lx' + x')."""
    iso = {}
    X = np.zeros((4, Lx * Ly, N, k))
    Y = np.zeros_like(X)
    for d in range(4):
        lx, ly = turned_size(Lx, Ly, d)
        iso[d] = {}
        for y in range(ly):
            for x in range(lx):
                xb = S.gaussian_block(N, k, seed + 100 * d + 10 * x + y)
                yb = S.gaussian_block(N, k, seed + 100 * d + 10 * x + y + 1000)
                iso[d][(x, y)] = (xb, yb)
                X[d, y * lx + x], Y[d, y * lx + x] = xb, yb
    return iso, X, Y


def peps_sites(Lx, Ly, D, seed, noise=0.5):
    return {(x, y): S.product_plus_noise_site(2, D, seed + 7 * x + 3 * y, noise=noise)
            for x in range(Lx) for y in range(Ly)}


def stack_sites(sites, Lx, Ly):
    return torch.from_numpy(np.stack([sites[(s % Lx, s // Lx)] for s in range(Lx * Ly)])).to(DEV)


def env_error(gpu_env, cell):
    """Largest relative element error over all tensors (shapes must agree)."""
    worst = 0.0
    for s, (C, T) in gpu_env.items():
        e = cell.env[s]
        for g, o in list(zip(C, e.C)) + list(zip(T, e.T)):
            assert g.shape == o.shape, (s, g.shape, o.shape)
            worst = max(worst, np.abs(g - o).max() / np.abs(o).max())
    return worst


def spectra_of(env, Lx, Ly, chi):
    return np.stack([O.corner_spectra(O.Env(*env[(x, y)]), chi)
                     for x in range(Lx) for y in range(Ly)])


def make_cell(cfg, sites, boundary=None):
    return P.Cell(cfg, stack_sites(sites, cfg.Lx, cfg.Ly),
                  None if boundary is None else torch.from_numpy(boundary).to(DEV))


@pytest.mark.parametrize("L", [(2, 2), (3, 2), (1, 2)])
def test_cell_iterations_match_oracle_step_by_step(L):
    """Random PEPS cell (D=2, chi=8, p=4): two randomized-SVD warm-up
    iterations (the environment grows from Dl=4 to chi in the first, every
    cut taking the randomized SVD of its start blocks' first rows), then
    three SI iterations with recycled blocks; every tensor and the recycled
    blocks after every iteration.  Lx != Ly checks the turned cells'
    coordinates; Lx = 1 a column whose new environment overwrites the one it
    is made from."""
    Lx, Ly = L
    D, chi, p = 2, 8, 4
    cfg = P.CellConfig(Lx, Ly, d=2, D=D, chi=chi, p=p, n_si=2)
    sites = peps_sites(Lx, Ly, D, 5)
    iso, X, Y = start_blocks(Lx, Ly, cfg.N, cfg.k, 31)
    g = make_cell(cfg, sites)
    g.set_blocks(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV))
    a = {s: O.double_layer(A) for s, A in sites.items()}
    cell = M.cell_initial_env(a, Lx, Ly, S.trace_boundary(D))
    err0 = env_error(g.get_env(), cell)
    print(f"initial environment: max rel err {err0:.2e}")
    assert err0 <= 1e-13
    spec = M.cell_corner_spectra(cell, chi)
    cur = None
    for it, mode in enumerate(["rsvd", "rsvd", "si", "si", "si"]):
        delta = g.iterate(mode)
        if mode == "si" and cur is None:
            cur = {d: dict(iso[d]) for d in range(4)}
        cell, blocks, modes = M.ctm_iteration(cell, chi, mode, cur if mode == "si" else iso, 2,
                                              1e-12, True)
        if mode == "si":
            cur = blocks
        new = M.cell_corner_spectra(cell, chi)
        d_or = float(np.max(np.linalg.norm(new - spec, axis=2)))
        spec = new
        err = env_error(g.get_env(), cell)
        print(f"iteration {it} ({mode}, oracle modes {sorted(set(modes))}): env err {err:.2e}, "
              f"delta {delta:.3e} vs {d_or:.3e}")
        assert err <= 1e-9, (it, err)
        assert abs(delta - d_or) <= 1e-10 + 1e-8 * d_or, (it, delta, d_or)
        if mode == "si":
            Xg, Yg = g.get_blocks()
            for d in range(4):
                lx, ly = turned_size(Lx, Ly, d)
                for (x, y), (xb, yb) in cur[d].items():
                    i = y * lx + x
                    ex = np.abs(Xg[d, i][:, :chi] - xb[:, :chi]).max()
                    ey = np.abs(Yg[d, i][:, :chi] - yb[:, :chi]).max()
                    assert ex <= 1e-8 and ey <= 1e-8, (it, d, x, y, ex, ey)
    g.close()


def test_cell_full_svd_iterations_match_oracle():
    """Full-SVD projectors for every cut (3x2 PEPS cell, D=2, chi=8) for
    three iterations, the first of them growing the environment."""
    Lx, Ly, D, chi = 3, 2, 2, 8
    cfg = P.CellConfig(Lx, Ly, d=2, D=D, chi=chi, p=4, n_si=2)
    sites = peps_sites(Lx, Ly, D, 17)
    g = make_cell(cfg, sites)
    a = {s: O.double_layer(A) for s, A in sites.items()}
    cell = M.cell_initial_env(a, Lx, Ly, S.trace_boundary(D))
    for it in range(3):
        g.iterate("svd")
        cell, _, modes = M.ctm_iteration(cell, chi, "svd", None)
        err = env_error(g.get_env(), cell)
        print(f"svd iteration {it} ({sorted(set(modes))}): env err {err:.2e}")
        assert err <= 1e-8, (it, err)
    g.close()


def bond_gauged_ising(beta, Lx, Ly, seed):
    """The Ising ferromagnet with each bond's weight split by its own random
    gauge (every site tensor differs; the network is the ferromagnet), with
    the boundary vectors per (site, leg) as a [Lx*Ly, 4, 2] array (legs
    u, l, d, r of site y*Lx + x)."""
    rng = np.random.default_rng(seed)
    W = S.ising_weights(beta)
    Gh = {(x, y): np.eye(2) + 0.4 * rng.uniform(-1, 1, (2, 2)) for x in range(Lx) for y in range(Ly)}
    Gv = {(x, y): np.eye(2) + 0.4 * rng.uniform(-1, 1, (2, 2)) for x in range(Lx) for y in range(Ly)}
    inv_t = lambda G: np.linalg.inv(G).T  # noqa: E731
    a, legs = {}, np.zeros((Lx * Ly, 4, 2))
    for x in range(Lx):
        for y in range(Ly):
            up = W @ inv_t(Gv[(x, (y - 1) % Ly)])
            left = W @ inv_t(Gh[((x - 1) % Lx, y)])
            down = W @ Gv[(x, y)]
            right = W @ Gh[(x, y)]
            a[(x, y)] = np.einsum("su,sl,sd,sr->uldr", up, left, down, right)
            s = y * Lx + x
            legs[s, 0] = (W @ Gv[(x, (y - 1) % Ly)])[0]
            legs[s, 1] = (W @ Gh[((x - 1) % Lx, y)])[0]
            legs[s, 2] = (W @ inv_t(Gv[(x, y)]))[0]
            legs[s, 3] = (W @ inv_t(Gh[(x, y)]))[0]
    return a, legs


def test_cell_run_on_a_bond_gauged_ising_cell_matches_oracle():
    """3x3 cell of nine different classical tensors (d = 0, Dl = 2, chi =
    16): identity projectors while the cuts grow (2 -> 4 -> 8 -> 16), two
    randomized-SVD warm-up iterations, then SI iterations to delta < 1e-11:
    the same iteration count and kinds as the oracle's run, deltas and the
    converged environment."""
    Lx, Ly, chi = 3, 3, 16
    beta = 0.5
    a, legs = bond_gauged_ising(beta, Lx, Ly, 21)
    cfg = P.CellConfig(Lx, Ly, d=0, D=2, chi=chi, p=8, n_si=2)
    iso, X, Y = start_blocks(Lx, Ly, cfg.N, cfg.k, 11)
    g = make_cell(cfg, a, legs)
    g.set_blocks(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV))
    r = g.run(warmup=2, tol=1e-11, max_iter=80)
    cell = M.cell_initial_env(a, Lx, Ly, lambda s, leg: legs[s[1] * Lx + s[0], "uldr".index(leg)])
    cell, hist = M.run_cell(cell, chi, iso, warmup=2, tol=1e-11, max_iter=80)
    print("gpu", r["iters"], r["kinds"][:4], r["deltas"][-3:])
    print("oracle", len(hist), [h["kind"] for h in hist][:4], [h["delta"] for h in hist][-3:])
    assert r["converged"] and r["iters"] == len(hist)
    kinds = ["rsvd" if h["kind"] == "warmup" else "si" for h in hist]
    assert r["kinds"] == kinds
    for dg, h in zip(r["deltas"], hist):
        assert abs(dg - h["delta"]) <= 1e-9 + 1e-6 * h["delta"], (dg, h["delta"])
    env = g.get_env()
    err = env_error(env, cell)
    print(f"converged environment: max rel err {err:.2e}")
    assert err <= 1e-8
    sg = spectra_of(env, Lx, Ly, chi)
    so = M.cell_corner_spectra(cell, chi)
    # both runs stop once the corner spectra change by less than 1e-11 per
    # iteration (the convergence measure), which is what fixes them
    assert np.abs(sg - so).max() <= 1e-11
    g.close()


def test_cell_rejects_bad_configurations():
    with pytest.raises(P.CtmError):
        P.Cell(P.CellConfig(2, 2, d=2, D=3, chi=4, p=4), torch.zeros(4, 2 * 3 ** 4,
                                                                       dtype=torch.float64,
                                                                       device=DEV))
    cfg = P.CellConfig(2, 2, d=2, D=2, chi=8, p=4)
    g = P.Cell(cfg, stack_sites(peps_sites(2, 2, 2, 3), 2, 2))
    with pytest.raises(P.CtmError):
        g.iterate("si")          # no start blocks
    g.close()
