"""Adjoint of the unit-cell iteration and the cell energy on the GPU
(ctm_cell_move_vjp, ctm_cell_energy_vjp) against the reverse-mode
reference of the unit-cell oracle (oracle.multisite_adjoint, torch autograd
on the CPU), and the gradient of the energy after unrolled iterations
against central differences of GPU runs.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle.multisite as M  # noqa: E402
import oracle.multisite_adjoint as MA  # noqa: E402
import paper_2607_15158_amd as P  # noqa: E402
import synth as S  # noqa: E402

DEV = torch.device("cuda", 0)
HEIS = S.heisenberg_bond()


def turned_size(Lx, Ly, d):
    return (Lx, Ly) if d % 2 == 0 else (Ly, Lx)


def unpack(cfg, v):
    """State vector -> ({site: (C list, T list)}, {d: {cut: (X, Yt)}})."""
    chi, Dl, N, k, ns = cfg.chi, cfg.Dl, cfg.N, cfg.k, cfg.ns
    env, off = {}, 0
    for s in range(ns):
        C = [v[off + i * chi * chi: off + (i + 1) * chi * chi].reshape(chi, chi) for i in range(4)]
        off += 4 * chi * chi
        T = [v[off + i * chi * Dl * chi: off + (i + 1) * chi * Dl * chi].reshape(chi, Dl, chi)
             for i in range(4)]
        off += 4 * chi * Dl * chi
        env[(s % cfg.Lx, s // cfg.Lx)] = (C, T)
    X = v[off: off + 4 * ns * N * k].reshape(4, ns, N, k)
    Y = v[off + 4 * ns * N * k:].reshape(4, ns, N, k)
    iso = {}
    for d in range(4):
        lx, ly = turned_size(cfg.Lx, cfg.Ly, d)
        iso[d] = {(x, y): (X[d, y * lx + x], Y[d, y * lx + x]) for x in range(lx) for y in range(ly)}
    return env, iso


def pack(cfg, env, iso):
    parts = []
    for s in range(cfg.ns):
        C, T = env[(s % cfg.Lx, s // cfg.Lx)]
        parts += [np.ravel(c) for c in C] + [np.ravel(t) for t in T]
    X = np.zeros((4, cfg.ns, cfg.N, cfg.k))
    Y = np.zeros_like(X)
    for d in range(4):
        lx, _ = turned_size(cfg.Lx, cfg.Ly, d)
        for (x, y), (a, b) in iso[d].items():
            X[d, y * lx + x], Y[d, y * lx + x] = a, b
    return np.concatenate(parts + [X.ravel(), Y.ravel()])


def start_blocks(cfg, seed):
    X = np.zeros((4, cfg.ns, cfg.N, cfg.k))
    Y = np.zeros_like(X)
    for d in range(4):
        lx, ly = turned_size(cfg.Lx, cfg.Ly, d)
        for y in range(ly):
            for x in range(lx):
                X[d, y * lx + x] = S.gaussian_block(cfg.N, cfg.k, seed + 100 * d + 10 * x + y)
                Y[d, y * lx + x] = S.gaussian_block(cfg.N, cfg.k, seed + 100 * d + 10 * x + y + 1000)
    return X, Y


def sites_of(cfg, seed, noise=0.5):
    return {(x, y): S.product_plus_noise_site(cfg.d, cfg.D, seed + 7 * x + 3 * y, noise=noise)
            for x in range(cfg.Lx) for y in range(cfg.Ly)}


def stacked(cfg, A):
    return torch.from_numpy(np.stack([A[(s % cfg.Lx, s // cfg.Lx)] for s in range(cfg.ns)])).to(DEV)


def full_state(cfg, A, warm=2, si=1, seed=31):
    """A state of full dimension: randomized warm-up, then SI iterations."""
    c = P.Cell(cfg, stacked(cfg, A))
    X, Y = start_blocks(cfg, seed)
    c.set_blocks(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV))
    for _ in range(warm):
        c.iterate("rsvd")
    for _ in range(si):
        c.iterate("si")
    return c, c.get_state_device()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CFG = P.CellConfig(2, 2, d=2, D=2, chi=8, p=4, n_si=2)


def test_taped_iteration_reproduces_the_cell_iteration():
    """The adjoint's recomputed iteration (fresh buffers, taped) gives the
    state of the cell's own SI iteration."""
    A = sites_of(CFG, 5)
    c, st = full_state(CFG, A)
    out, _, _ = c.move_vjp(st)
    c.iterate("si")
    ref = c.get_state_device().cpu().numpy()
    e1, i1 = unpack(CFG, out.cpu().numpy())
    e2, i2 = unpack(CFG, ref)
    worst = max(rel(a, b) for s in e1 for a, b in zip(e1[s][0] + e1[s][1], e2[s][0] + e2[s][1]))
    print(f"taped iteration vs cell iteration: env rel err {worst:.2e}")
    assert worst <= 1e-12
    for d in range(4):
        for kk in i1[d]:
            assert rel(i1[d][kk][0][:, :CFG.chi], i2[d][kk][0][:, :CFG.chi]) <= 1e-11
    c.close()


@pytest.mark.parametrize("L", [(2, 2), (3, 2)])
def test_cell_move_vjp_matches_oracle_autograd(L):
    cfg = P.CellConfig(L[0], L[1], d=2, D=2, chi=8, p=4, n_si=2)
    A = sites_of(cfg, 9)
    c, st = full_state(cfg, A)
    env, iso = unpack(cfg, st.cpu().numpy())
    rng = np.random.default_rng(2)
    env_b = {s: ([rng.standard_normal(x.shape) for x in C], [rng.standard_normal(x.shape) for x in T])
             for s, (C, T) in env.items()}
    # cotangents on the kept columns of the blocks (the oversampled columns are
    # weak directions whose derivatives are set by rounding)
    def kept(shape):
        b = rng.standard_normal(shape)
        b[:, cfg.chi:] = 0.0
        return b

    iso_b = {d: {kk: (kept(X.shape), kept(Y.shape)) for kk, (X, Y) in iso[d].items()} for d in range(4)}
    bar = torch.from_numpy(pack(cfg, env_b, iso_b)).to(DEV)
    _, sbar, site_bar = c.move_vjp(st, bar)
    env_g, iso_g, A_g = MA.cell_move_vjp(env, iso, A, cfg.Lx, cfg.Ly, cfg.chi, (env_b, iso_b))
    ge, gi = unpack(cfg, sbar.cpu().numpy())
    ref_env = np.concatenate([np.ravel(x) for s in env_g for x in env_g[s][0] + env_g[s][1]])
    got_env = np.concatenate([np.ravel(x) for s in env_g for x in ge[s][0] + ge[s][1]])
    e_env = rel(got_env, ref_env)
    ref_iso = np.concatenate([np.ravel(iso_g[d][kk][j]) for d in range(4) for kk in iso_g[d] for j in (0, 1)])
    got_iso = np.concatenate([np.ravel(gi[d][kk][j]) for d in range(4) for kk in iso_g[d] for j in (0, 1)])
    e_iso = rel(got_iso, ref_iso)
    sb = site_bar.cpu().numpy().reshape(cfg.ns, -1)
    e_site = max(rel(sb[s], A_g[(s % cfg.Lx, s // cfg.Lx)].ravel()) for s in range(cfg.ns))
    print(f"cell move VJP vs oracle autograd: env {e_env:.2e}, blocks {e_iso:.2e}, sites {e_site:.2e}")
    assert e_env <= 1e-7 and e_iso <= 1e-7 and e_site <= 1e-7
    c.close()


def test_cell_energy_and_its_gradient_match_oracle_autograd():
    cfg = P.CellConfig(2, 2, d=2, D=2, chi=8, p=4, n_si=2)
    A = sites_of(cfg, 13)
    c, st = full_state(cfg, A)
    env, _ = unpack(cfg, st.cpu().numpy())
    ops = {"h": HEIS, "v": 0.7 * HEIS, "d": 0.4 * HEIS}
    e, sbar, site_bar = c.energy_vjp(st, ops)
    e_o, env_g, A_g = MA.cell_energy_vjp(env, A, cfg.Lx, cfg.Ly, ops)
    print(f"cell energy {e:.15f} oracle {e_o:.15f}")
    assert abs(e - e_o) <= 1e-12 * abs(e_o)
    ge, gi = unpack(cfg, sbar.cpu().numpy())
    ref = np.concatenate([np.ravel(x) for s in env_g for x in env_g[s][0] + env_g[s][1]])
    got = np.concatenate([np.ravel(x) for s in env_g for x in ge[s][0] + ge[s][1]])
    assert rel(got, ref) <= 1e-10
    assert all(np.abs(gi[d][kk][j]).max() == 0.0 for d in range(4) for kk in gi[d] for j in (0, 1))
    sb = site_bar.cpu().numpy().reshape(cfg.ns, -1)
    for s in range(cfg.ns):
        assert rel(sb[s], A_g[(s % cfg.Lx, s // cfg.Lx)].ravel()) <= 1e-10
    c.close()


def test_unrolled_cell_energy_gradient_matches_central_differences():
    """Energy after 4 SI iterations from a fixed state, differentiated with
    respect to the four site tensors by the unrolled adjoint, against central
    differences of GPU runs along a random direction (step 1e-4: the
    iterations carry rounding noise of ~1e-11)."""
    cfg = CFG
    A = sites_of(cfg, 21)
    c, st = full_state(cfg, A)
    c.close()
    ops = {"h": HEIS, "v": HEIS, "d": HEIS}
    sites = stacked(cfg, A).requires_grad_(True)
    e = P.unrolled_cell_energy(sites, cfg, ops, st, 4)
    e.backward()
    g = sites.grad.cpu().numpy()
    rng = np.random.default_rng(7)
    dA = rng.standard_normal(g.shape)

    def energy_at(t):
        cc = P.Cell(cfg, (stacked(cfg, A) + t * torch.from_numpy(dA).to(DEV)).contiguous())
        cc.set_state_device(st)
        for _ in range(4):
            cc.iterate("si")
        v = cc.energy_vjp(cc.get_state_device(), ops, grad=False)
        cc.close()
        return v

    h = 1e-4
    fd = (energy_at(h) - energy_at(-h)) / (2 * h)
    an = float(np.sum(g * dA))
    print(f"unrolled gradient: {an:.10f}, central difference {fd:.10f}")
    assert abs(e.item() - energy_at(0.0)) <= 1e-12
    assert abs(fd - an) <= 2e-5 * max(abs(an), 1e-3)


def test_unit_cell_gradient_at_full_size_matches_central_differences():
    """The 3x3 unit cell at D=5, chi=100, p=5 (k = 105, N = 2500): energy per
    site of the triangular lattice (h, v and d bonds of every site) after 30
    SI iterations from a state converged to delta ~ 1e-12 (nine different
    site tensors near a product state), differentiated with respect to the
    nine site tensors by unrolling the iterations with checkpoints at every
    iteration boundary, against central differences of GPU runs along a
    random direction.  Measured on MI355X: agreement to 7e-9 relative at
    h = 1e-6 (1e-9 at h = 1e-7); from an unconverged state the energy after
    30 iterations is not smooth on the scale of h and no step gives a clean
    difference."""
    import time
    cfg = P.CellConfig(3, 3, d=2, D=5, chi=100, p=5, n_si=2)
    A = sites_of(cfg, 40, noise=0.05)
    c, st = full_state(cfg, A, warm=3, si=25)
    c.close()
    ops = {"h": HEIS, "v": HEIS, "d": HEIS}
    moves = 30
    sites = stacked(cfg, A).requires_grad_(True)
    t0 = time.time()
    e = P.unrolled_cell_energy(sites, cfg, ops, st, moves)
    e.backward()
    torch.cuda.synchronize()
    t_grad = time.time() - t0
    g = sites.grad.cpu().numpy()
    rng = np.random.default_rng(17)
    dA = rng.standard_normal(g.shape)

    def energy_at(t):
        cc = P.Cell(cfg, (stacked(cfg, A) + t * torch.from_numpy(dA).to(DEV)).contiguous())
        cc.set_state_device(st)
        for _ in range(moves):
            cc.iterate("si")
        v = cc.energy_vjp(cc.get_state_device(), ops, grad=False)
        cc.close()
        return v

    an = float(np.sum(g * dA))
    print(f"energy {e.item():.12f}; gradient through {moves} iterations of the 3x3 cell in "
          f"{t_grad:.1f} s", flush=True)
    errs = []
    for h in (1e-5, 1e-6):
        fd = (energy_at(h) - energy_at(-h)) / (2 * h)
        errs.append(abs(fd - an) / abs(an))
        print(f"h = {h:.0e}: central difference {fd:.10f}, unrolled gradient {an:.10f}, "
              f"rel diff {errs[-1]:.2e}", flush=True)
    assert errs[-1] <= 1e-6
