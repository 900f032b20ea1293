"""GPU parity of the adjoint of one SI move (ctm_move_vjp).

* against the reverse-mode reference (PyTorch CPU autograd of the oracle's
  move, itself pinned to finite differences of the NumPy move), element by
  element for the cotangents of C, T, X, Y^T and the site tensor, at sizes
  that span one and several GEMM tiles;
* the move recomputed by the adjoint equals ctm_move from the same state;
* against central finite differences of the GPU's own moves at a larger
  size (D=3, chi=18), where the autograd reference would be slow.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle.adjoint as J  # noqa: E402
import paper_2607_15158_amd as P  # noqa: E402
import synth as S  # noqa: E402


def make_state(D, chi, p, seed=11, noise=1.0):
    A = S.product_plus_noise_site(2, D, seed, noise=noise)
    Dl, N, k = D * D, chi * D * D, min(chi + p, chi * D * D)
    C = [S.gaussian_block(chi, chi, 60 + i) for i in range(4)]
    T = [S.gaussian_block(chi * Dl, chi, 70 + i).reshape(chi, Dl, chi) for i in range(4)]
    X = [np.linalg.qr(S.gaussian_block(N, k, 20 + b))[0] for b in range(4)]
    Y = [np.linalg.qr(S.gaussian_block(N, k, 30 + b))[0] for b in range(4)]
    return A, C, T, X, Y


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("D,chi,p,n_si", [(2, 4, 4, 1), (2, 4, 4, 2), (2, 8, 4, 2), (3, 9, 5, 2)])
def test_move_vjp_matches_autograd_reference(D, chi, p, n_si):
    A, C, T, X, Y = make_state(D, chi, p)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=n_si)
    dev = torch.device("cuda", 0)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    state = ctx.pack_state(C, T, np.stack(X), np.stack(Y))
    rng = np.random.default_rng(5)
    bars_C = [rng.standard_normal((chi, chi)) for _ in range(4)]
    bars_T = [rng.standard_normal((chi, D * D, chi)) for _ in range(4)]
    bars_X = [rng.standard_normal(x.shape) for x in X]
    bars_Y = [rng.standard_normal(y.shape) for y in Y]
    bar = ctx.pack_state(bars_C, bars_T, np.stack(bars_X), np.stack(bars_Y))
    in_bar, out, site_bar = ctx.move_vjp(torch.from_numpy(state), torch.from_numpy(bar))
    ib = in_bar.cpu().numpy()
    assert not ib[-4:].any()
    ib[-4] = chi                      # counters of a cotangent are zero; unpack at chi
    g = ctx.unpack_state(ib)
    gC, gT, gX, gY, gA = J.move_vjp(C, T, X, Y, A, (bars_C, bars_T, bars_X, bars_Y), chi, n_si)
    errs = {"C": max(rel(a, b) for a, b in zip(g["C"], gC)),
            "T": max(rel(a, b) for a, b in zip(g["T"], gT)),
            "X": max(rel(a, b) for a, b in zip(g["X"], gX)),
            "Y": max(rel(a, b) for a, b in zip(g["Yt"], gY)),
            "A": rel(site_bar.cpu().numpy(), gA)}
    print(errs)
    assert all(e <= 1e-8 for e in errs.values()), errs
    # the recomputed move is the library's move
    ctx.set_state(state)
    ctx.move()
    ref = ctx.unpack_state(ctx.get_state())
    got = ctx.unpack_state(out.cpu().numpy())
    for key in ("C", "T"):
        assert max(rel(a, b) for a, b in zip(got[key], ref[key])) <= 1e-10, key
    for key in ("X", "Yt"):
        assert rel(got[key], ref[key]) <= 1e-10, key


def test_move_vjp_matches_finite_differences_of_gpu_moves():
    D, chi, p, n_si = 3, 18, 6, 2
    A, C, T, X, Y = make_state(D, chi, p, seed=4, noise=0.5)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=n_si)
    dev = torch.device("cuda", 0)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    state = ctx.pack_state(C, T, np.stack(X), np.stack(Y))
    n = state.size
    rng = np.random.default_rng(9)
    bar = rng.standard_normal(n)
    bar[-4:] = 0.0
    in_bar, _, site_bar = ctx.move_vjp(torch.from_numpy(state), torch.from_numpy(bar))
    in_bar = in_bar.cpu().numpy()

    def f(st):
        ctx.set_state(st)
        ctx.move()
        return float(ctx.get_state()[:-4] @ bar[:-4])

    for trial in range(3):
        d = rng.standard_normal(n)
        d[-4:] = 0.0
        h = 1e-6
        fd = (f(state + h * d) - f(state - h * d)) / (2 * h)
        an = float(in_bar[:-4] @ d[:-4])
        print(trial, fd, an)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (trial, fd, an)


def test_fixed_point_gradient_matches_finite_differences_of_converged_environments():
    """eq. implicit: the site-tensor gradient of a functional of the
    converged environment, from the Neumann series of reverse passes at the
    fixed point, equals central differences of fully converged GPU runs."""
    D, chi, p = 2, 8, 4
    A = S.product_plus_noise_site(2, D, 2, noise=0.3)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=2)
    N, k = cfg.N, cfg.k
    X0 = np.stack([S.gaussian_block(N, k, 20 + b) for b in range(4)])
    Y0 = np.stack([S.gaussian_block(N, k, 30 + b) for b in range(4)])
    dev = torch.device("cuda", 0)

    def converged(site):
        ctx = P.Ctm(cfg, torch.from_numpy(site).to(dev))
        ctx.set_isometries(torch.from_numpy(X0).to(dev), torch.from_numpy(Y0).to(dev))
        r = ctx.converge(1e-14, 400)
        assert r["delta"] < 1e-12, r
        return ctx, ctx.get_state()

    ctx, star = converged(A)
    rng = np.random.default_rng(12)
    n_ct = 4 * chi * chi + 4 * chi * D * D * chi
    w = np.zeros_like(star)
    w[:n_ct] = rng.standard_normal(n_ct)
    x_bar, site_bar, passes, rel_norm = ctx.fixed_point_vjp(
        torch.from_numpy(star), torch.from_numpy(w), tol=1e-12, max_iter=400)
    print("passes", passes, "last term", rel_norm)
    site_bar = site_bar.cpu().numpy()
    for trial in range(2):
        d = rng.standard_normal(A.shape)
        h = 1e-5
        lp = float(converged(A + h * d)[1] @ w)
        lm = float(converged(A - h * d)[1] @ w)
        fd = (lp - lm) / (2 * h)
        an = float((site_bar * d).sum())
        print(trial, fd, an)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1.0), (trial, fd, an)


@pytest.mark.parametrize("D,chi", [(2, 4), (3, 9)])
def test_energy_gradient_matches_autograd_reference(D, chi):
    A, C, T, X, Y = make_state(D, chi, 4)
    cfg = P.Config(d=2, D=D, chi=chi, p=4, n_si=2)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(torch.device("cuda", 0)))
    state = torch.from_numpy(ctx.pack_state(C, T, np.stack(X), np.stack(Y)))
    h = S.heisenberg_bond()
    e, bar, site_bar = ctx.energy_vjp(state, h)
    ref_e, gC, gT, gA = J.energy_vjp(C, T, A, h)
    assert abs(e - ref_e) <= 1e-12 * max(1.0, abs(ref_e))
    b = bar.cpu().numpy()
    assert not b[-4:].any()
    b[-4] = chi
    g = ctx.unpack_state(b)
    errs = {"C": max(rel(a, r) for a, r in zip(g["C"], gC)),
            "T": max(rel(a, r) for a, r in zip(g["T"], gT)),
            "A": rel(site_bar.cpu().numpy(), gA)}
    print(errs)
    assert all(v <= 1e-10 for v in errs.values()), errs
    assert not g["X"].any() and not g["Yt"].any()


@pytest.mark.parametrize("bonds", ["d", "a", "hvd", "hvda"])
@pytest.mark.parametrize("D,chi", [(2, 4), (3, 9)])
def test_bond_energy_gradient_matches_autograd_reference(D, chi, bonds):
    """Energy over a set of bonds, including the diagonal pair of the
    plaquette (hand-written reverse pass) and the anti-diagonal (the diagonal
    of the turned network), against the autograd reference, for an operator
    that is not symmetric under exchange of the two sites."""
    A, C, T, X, Y = make_state(D, chi, 4)
    cfg = P.Config(d=2, D=D, chi=chi, p=4, n_si=2)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(torch.device("cuda", 0)))
    state = torch.from_numpy(ctx.pack_state(C, T, np.stack(X), np.stack(Y)))
    h = S.heisenberg_bond() + 0.3 * np.kron(S.pauli("x"), S.pauli("z"))
    e, bar, site_bar = ctx.energy_vjp(state, h, bonds=bonds)
    ref_e, gC, gT, gA = J.energy_vjp(C, T, A, h, bonds)
    assert abs(e - ref_e) <= 1e-12 * max(1.0, abs(ref_e))
    b = bar.cpu().numpy()
    assert not b[-4:].any()
    b[-4] = chi
    g = ctx.unpack_state(b)
    errs = {"C": max(rel(a, r) for a, r in zip(g["C"], gC)),
            "T": max(rel(a, r) for a, r in zip(g["T"], gT)),
            "A": rel(site_bar.cpu().numpy(), gA)}
    print(bonds, errs)
    assert all(v <= 1e-10 for v in errs.values()), errs
    assert not g["X"].any() and not g["Yt"].any()


@pytest.mark.parametrize("bonds", ["hv", "hvd"])
def test_gradient_of_the_converged_energy_matches_finite_differences(bonds):
    """The full gradient of the converged Heisenberg energy (nearest-neighbour
    bonds, and the triangular lattice's h + v + d) with respect to the site
    tensor (direct term + fixed-point term, eq. implicit) against central
    differences of converged GPU runs."""
    D, chi, p = 2, 8, 4
    A = S.product_plus_noise_site(2, D, 2, noise=0.3)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=2)
    N, k = cfg.N, cfg.k
    X0 = np.stack([S.gaussian_block(N, k, 20 + b) for b in range(4)])
    Y0 = np.stack([S.gaussian_block(N, k, 30 + b) for b in range(4)])
    h = S.heisenberg_bond()
    dev = torch.device("cuda", 0)

    def converged(site):
        ctx = P.Ctm(cfg, torch.from_numpy(site).to(dev))
        ctx.set_isometries(torch.from_numpy(X0).to(dev), torch.from_numpy(Y0).to(dev))
        r = ctx.converge(1e-14, 400)
        assert r["delta"] < 1e-12, r
        return ctx

    kinds = {"h": P.OBS_BOND_H, "v": P.OBS_BOND_V, "d": P.OBS_BOND_D}

    def bond_sum(c):
        return sum(c.observable(kinds[bd], h)[0] for bd in bonds)

    ctx = converged(A)
    e, grad, passes = ctx.energy_gradient(h, bonds=bonds)
    grad = grad.cpu().numpy()
    assert abs(e - bond_sum(ctx)) <= 1e-12
    print("energy", e, "passes", passes)
    rng = np.random.default_rng(21)
    for trial in range(2):
        d = rng.standard_normal(A.shape)
        hh = 1e-5

        def energy(site):
            return bond_sum(converged(site))

        fd = (energy(A + hh * d) - energy(A - hh * d)) / (2 * hh)
        an = float((grad * d).sum())
        print(trial, fd, an)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3), (trial, fd, an)


def test_bond_energy_gradient_with_three_level_sites():
    """d = 3 (nine open-leg pairs: the batched products run in two launches
    of eight and one): energy h + v + d against the autograd reference."""
    D, chi, d = 2, 4, 3
    rng = np.random.default_rng(31)
    A = rng.standard_normal((d, D, D, D, D))
    Dl = D * D
    C = [S.gaussian_block(chi, chi, 60 + i) for i in range(4)]
    T = [S.gaussian_block(chi * Dl, chi, 70 + i).reshape(chi, Dl, chi) for i in range(4)]
    cfg = P.Config(d=d, D=D, chi=chi, p=4, n_si=2)
    X = np.stack([S.gaussian_block(cfg.N, cfg.k, 20 + b) for b in range(4)])
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(torch.device("cuda", 0)))
    state = torch.from_numpy(ctx.pack_state(C, T, X, X))
    op = rng.standard_normal((d * d, d * d))
    e, bar, site_bar = ctx.energy_vjp(state, op, bonds="hvd")
    ref_e, gC, gT, gA = J.energy_vjp(C, T, A, op, "hvd")
    assert abs(e - ref_e) <= 1e-12 * max(1.0, abs(ref_e))
    b = bar.cpu().numpy()
    b[-4] = chi
    g = ctx.unpack_state(b)
    errs = {"C": max(rel(a, r) for a, r in zip(g["C"], gC)),
            "T": max(rel(a, r) for a, r in zip(g["T"], gT)),
            "A": rel(site_bar.cpu().numpy(), gA)}
    assert all(v <= 1e-10 for v in errs.values()), errs


def spiral_ops():
    th = 2 * np.pi / 3
    return P.spiral_bond_operators(S.heisenberg_bond(), {"h": th, "v": th, "d": 2 * th})


def test_gradient_with_per_bond_operators_matches_finite_differences():
    """Converged energy with a different operator on each bond (the spiral
    ansatz of the triangular lattice: h, v and the diagonal, each rotated by
    its bond angle) against central differences of converged GPU runs."""
    D, chi, p = 2, 8, 4
    A = S.product_plus_noise_site(2, D, 3, noise=0.4)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=2)
    N, k = cfg.N, cfg.k
    X0 = np.stack([S.gaussian_block(N, k, 20 + b) for b in range(4)])
    Y0 = np.stack([S.gaussian_block(N, k, 30 + b) for b in range(4)])
    ops = spiral_ops()
    kinds = {"h": P.OBS_BOND_H, "v": P.OBS_BOND_V, "d": P.OBS_BOND_D}
    dev = torch.device("cuda", 0)

    def converged(site):
        ctx = P.Ctm(cfg, torch.from_numpy(site).to(dev))
        ctx.set_isometries(torch.from_numpy(X0).to(dev), torch.from_numpy(Y0).to(dev))
        r = ctx.converge(1e-14, 400)
        assert r["delta"] < 1e-12, r
        return ctx

    def energy(ctx):
        return sum(ctx.observable(kinds[bd], op)[0] for bd, op in ops.items())

    ctx = converged(A)
    e, grad, _ = ctx.energy_gradient(ops)
    assert abs(e - energy(ctx)) <= 1e-12
    grad = grad.cpu().numpy()
    d = np.random.default_rng(8).standard_normal(A.shape)
    hh = 1e-5
    fd = (energy(converged(A + hh * d)) - energy(converged(A - hh * d))) / (2 * hh)
    an = float((grad * d).sum())
    assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3), (fd, an)


def test_lbfgs_lowers_the_triangular_lattice_energy():
    """L-BFGS over the site tensor with the converged energy of the spiral
    ansatz and its fixed-point gradient, each evaluation starting from the
    previous environment and SI blocks: the energy per site decreases and
    stays above the paper's extrapolated ground-state energy (-0.55184)."""
    D, chi = 2, 8
    A0 = torch.from_numpy(S.product_plus_noise_site(2, D, 5, noise=0.5)).cuda()
    cfg = P.Config(d=2, D=D, chi=chi, p=4, n_si=2)
    A, hist = P.optimize_lbfgs(A0, cfg, spiral_ops(), iterations=6)
    energies = [h[0] for h in hist]
    print(hist)
    assert energies[-1] < energies[0] - 0.05, energies
    assert min(energies) > -0.55184 - 0.02, energies
    assert hist[-1][2] < hist[0][2], hist          # recycled environments converge faster


def test_converged_energy_as_a_torch_function_descends():
    """The differentiable converged energy plugs into torch autograd: its
    gradient equals the library's, and a small step against it lowers the
    converged energy by the first-order amount."""
    D, chi, p = 2, 8, 4
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=2)
    N, k = cfg.N, cfg.k
    X0 = np.stack([S.gaussian_block(N, k, 20 + b) for b in range(4)])
    Y0 = np.stack([S.gaussian_block(N, k, 30 + b) for b in range(4)])
    h = S.heisenberg_bond()
    dev = torch.device("cuda", 0)
    A = torch.from_numpy(S.product_plus_noise_site(2, D, 2, noise=0.3)).to(dev).requires_grad_(True)
    e = P.converged_energy(A, cfg, h, X0, Y0)
    e.backward()
    g = A.grad.detach().clone()
    step = 1e-4 * g / g.norm()
    with torch.no_grad():
        e2 = P.converged_energy(A - step, cfg, h, X0, Y0)
    drop = float(e.detach() - e2)
    first_order = float((g * step).sum())
    print(float(e), float(e2), drop, first_order)
    assert drop > 0
    assert abs(drop - first_order) <= 1e-2 * first_order


def test_unrolled_triangular_energy_matches_autograd():
    """The unrolled energy with one operator per bond (spiral ansatz of the
    triangular lattice, the diagonal bond included) against PyTorch CPU
    autograd through the oracle's moves and the reference bond energies."""
    D, chi, p, n_si, moves = 2, 4, 4, 2, 2
    A, C, T, X, Y = make_state(D, chi, p)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=n_si)
    ops = spiral_ops()
    dev = torch.device("cuda", 0)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    state0 = torch.from_numpy(ctx.pack_state(C, T, np.stack(X), np.stack(Y))).to(dev)
    At = torch.from_numpy(A).to(dev).requires_grad_(True)
    e = P.unrolled_energy(At, cfg, ops, state0, moves)
    e.backward()
    g = At.grad.cpu().numpy()
    leaf = torch.tensor(A, requires_grad=True)
    tt = lambda L: [torch.tensor(v) for v in L]   # noqa: E731
    Cs, Ts, Xs, Ys = tt(C), tt(T), tt(X), tt(Y)
    for _ in range(moves):
        Cs, Ts, Xs, Ys = J.move_torch(Cs, Ts, Xs, Ys, leaf, chi, n_si)
    e_ref = sum(J.energy_torch(Cs, Ts, leaf, torch.tensor(op), bd) for bd, op in ops.items())
    (g_ref,) = torch.autograd.grad(e_ref, leaf)
    assert abs(float(e.detach()) - float(e_ref.detach())) <= 1e-12
    assert rel(g, g_ref.numpy()) <= 1e-9, rel(g, g_ref.numpy())


def test_unrolled_energy_gradient_matches_autograd_and_finite_differences():
    """Energy after n SI moves from a fixed state, differentiated by unrolling
    with move-boundary checkpoints (the adjoint behind a torch autograd
    function): against PyTorch CPU autograd through the oracle's moves, and
    against central differences of the GPU's own moves."""
    D, chi, p, n_si, moves = 2, 4, 4, 2, 3
    A, C, T, X, Y = make_state(D, chi, p)
    cfg = P.Config(d=2, D=D, chi=chi, p=p, n_si=n_si)
    h = S.heisenberg_bond()
    dev = torch.device("cuda", 0)
    ctx = P.Ctm(cfg, torch.from_numpy(A).to(dev))
    state0 = torch.from_numpy(ctx.pack_state(C, T, np.stack(X), np.stack(Y))).to(dev)
    At = torch.from_numpy(A).to(dev).requires_grad_(True)
    e = P.unrolled_energy(At, cfg, h, state0, moves)
    e.backward()
    g = At.grad.cpu().numpy()
    # CPU autograd through the oracle's moves
    leaf = torch.tensor(A, requires_grad=True)
    tt = lambda L: [torch.tensor(v) for v in L]   # noqa: E731
    Cs, Ts, Xs, Ys = tt(C), tt(T), tt(X), tt(Y)
    for _ in range(moves):
        Cs, Ts, Xs, Ys = J.move_torch(Cs, Ts, Xs, Ys, leaf, chi, n_si)
    e_ref = J.energy_torch(Cs, Ts, leaf, torch.tensor(h))
    (g_ref,) = torch.autograd.grad(e_ref, leaf)
    assert abs(float(e.detach()) - float(e_ref.detach())) <= 1e-12
    assert rel(g, g_ref.numpy()) <= 1e-9, rel(g, g_ref.numpy())
    # central differences of GPU moves
    st0 = state0.cpu().numpy()

    def energy(site):
        c = P.Ctm(cfg, torch.from_numpy(site).to(dev))
        c.set_state(st0)
        for _ in range(moves):
            c.move()
        return c.observable(P.OBS_BOND_H, h)[0] + c.observable(P.OBS_BOND_V, h)[0]

    rng = np.random.default_rng(8)
    d = rng.standard_normal(A.shape)
    fd = (energy(A + 1e-6 * d) - energy(A - 1e-6 * d)) / 2e-6
    an = float((g * d).sum())
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2), (fd, an)
