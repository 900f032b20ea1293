"""Pins of the multi-site (Lx x Ly unit cell) oracle, CPU.

* a cell of equal classical Ising tensors reproduces Onsager's free energy
  and Yang's magnetisation at every site;
* the antiferromagnetic Ising model on a 2x2 cell (the ferromagnet with the
  spins of one sublattice flipped, i.e. the B-sublattice tensors built with
  flipped weights) gives +m on one sublattice and -m on the other, and the
  ferromagnetic nearest-neighbour correlation with a minus sign: the site
  placement and the neighbour structure of the cell are those of the lattice;
* a 3x3 cell of nine different product states gives every bond's value
  exactly (horizontal, vertical and diagonal bonds of every site);
* turning the cell by 90 degrees maps the horizontal bonds onto the
  vertical ones;
* randomized-SVD warm-up then SI iterations and full-SVD iterations reach
  the same converged energies.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import oracle.multisite as M
import synth as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "ising_closed_forms.json")))["values"]


def gold(beta, key):
    return float(GOLD[str(beta)][key])


def blocks(Lx, Ly, N, k, seed):
    """Start blocks per direction and cut (the turned cell of direction d is
    Ly x Lx for odd d)."""
    iso = {}
    for d in range(4):
        lx, ly = (Lx, Ly) if d % 2 == 0 else (Ly, Lx)
        iso[d] = {(x, y): (S.gaussian_block(N, k, seed + 100 * d + 10 * x + y),
                           S.gaussian_block(N, k, seed + 100 * d + 10 * x + y + 1000))
                  for x in range(lx) for y in range(ly)}
    return iso


def bond_gauged_ising(beta, Lx, Ly, seed):
    """The Ising ferromagnet on an Lx x Ly cell with every bond's weight
    split as (W G)(W G^-T)^T by its own random non-orthogonal G: all site
    tensors differ, yet the network is the ferromagnet as long as each bond
    pairs the two halves of its own G.  Returns the site tensors, their
    spin impurities and the boundary vectors per (site, leg) (the fixed-+
    neighbour's half of the bond)."""
    rng = np.random.default_rng(seed)
    W = S.ising_weights(beta)
    Gh = {(x, y): np.eye(2) + 0.4 * rng.uniform(-1, 1, (2, 2)) for x in range(Lx) for y in range(Ly)}
    Gv = {(x, y): np.eye(2) + 0.4 * rng.uniform(-1, 1, (2, 2)) for x in range(Lx) for y in range(Ly)}
    inv_t = lambda G: np.linalg.inv(G).T  # noqa: E731
    spin = np.array([1.0, -1.0])
    a, imp, legs = {}, {}, {}
    for x in range(Lx):
        for y in range(Ly):
            up = W @ inv_t(Gv[(x, (y - 1) % Ly)])
            left = W @ inv_t(Gh[((x - 1) % Lx, y)])
            down = W @ Gv[(x, y)]
            right = W @ Gh[(x, y)]
            a[(x, y)] = np.einsum("su,sl,sd,sr->uldr", up, left, down, right)
            imp[(x, y)] = np.einsum("s,su,sl,sd,sr->uldr", spin, up, left, down, right)
            # closing a leg: the other half of that bond with the spin fixed to +1
            legs[(x, y)] = {"u": (W @ Gv[(x, (y - 1) % Ly)])[0], "l": (W @ Gh[((x - 1) % Lx, y)])[0],
                            "d": (W @ inv_t(Gv[(x, y)]))[0], "r": (W @ inv_t(Gh[(x, y)]))[0]}
    return a, imp, (lambda s, leg: legs[s][leg])


def ising_cell_errors(a, imp, e, Lx, Ly, beta, chi=16):
    """Largest deviation from the closed forms (magnetisation at every site,
    nearest-neighbour and diagonal correlations on every bond) after SI
    convergence of the cell."""
    cell = M.cell_initial_env(a, Lx, Ly, e)
    cell, hist = M.run_cell(cell, chi, blocks(Lx, Ly, 2 * chi, chi + 8, 11), warmup=2,
                            tol=1e-12, max_iter=80)
    err = 0.0
    for x in range(Lx):
        for y in range(Ly):
            err = max(err, abs(M.cell_onesite(cell, x, y, imp[(x, y)]) - gold(beta, "magnetisation")))
            for direction, (dx, dy), key in (("h", (1, 0), "nn_correlation"),
                                             ("v", (0, 1), "nn_correlation"),
                                             ("d", (1, 1), "diag_correlation")):
                i2 = imp[((x + dx) % Lx, (y + dy) % Ly)]
                ss = M.cell_classical_bond(cell, x, y, imp[(x, y)], i2, direction)
                err = max(err, abs(ss - gold(beta, key)))
    return err, hist


def test_bond_gauged_ising_on_a_3x3_cell():
    """Nine different site tensors (each bond's weight split by its own
    random gauge) that together are the Ising ferromagnet: Yang's
    magnetisation at every site and the exact nearest-neighbour and
    diagonal correlations on every bond of the 3x3 cell.  Any mix-up of
    sites, bonds or legs in the cell's moves or observables pairs the wrong
    gauges and changes the network."""
    beta = 0.5
    a, imp, e = bond_gauged_ising(beta, 3, 3, 21)
    err, hist = ising_cell_errors(a, imp, e, 3, 3, beta)
    assert hist[-1]["delta"] < 1e-12, hist[-1]
    assert err <= 1e-9, err


def gauged_ising(beta, G):
    """Ising tensors with the bond weight factorised as (W G)(W G^-T)^T:
    site tensor, spin impurity and boundary vector for the two sublattices
    of a checkerboard (every bond joins a G site to a G^-T site, so the
    partition function is the ferromagnet's, while the two tensors differ)."""
    W = S.ising_weights(beta)
    Wa, Wb = W @ G, W @ np.linalg.inv(G).T
    spin = np.array([1.0, -1.0])
    out = {}
    for name, Wx, Wy in (("A", Wa, Wb), ("B", Wb, Wa)):
        a = np.einsum("su,sl,sd,sr->uldr", Wx, Wx, Wx, Wx)
        imp = np.einsum("s,su,sl,sd,sr->uldr", spin, Wx, Wx, Wx, Wx)
        # the fixed-+ neighbour closing an outer leg belongs to the other sublattice
        out[name] = (a, imp, Wy[0].copy())
    return out


@pytest.mark.parametrize("L", [(2, 2), (3, 3)])
def test_uniform_ising_cell_closed_forms(L):
    beta, chi = 0.5, 16
    Lx, Ly = L
    a, asig, e = S.ising_site(beta), S.ising_impurity(beta), S.ising_boundary(beta)
    cell = M.cell_initial_env({(x, y): a for x in range(Lx) for y in range(Ly)}, Lx, Ly, e)
    cell, hist = M.run_cell(cell, chi, blocks(Lx, Ly, 2 * chi, chi + 8, 7), warmup=2,
                            tol=1e-12, max_iter=80)
    assert hist[-1]["kind"] == "si" and hist[-1]["delta"] < 1e-12, hist[-1]
    for x in range(Lx):
        for y in range(Ly):
            lnk = np.log(M.cell_kappa(cell, x, y))
            assert abs(lnk - gold(beta, "minus_beta_f")) <= 1e-10 * lnk, (x, y, lnk)
            m = M.cell_onesite(cell, x, y, asig)
            assert abs(m - gold(beta, "magnetisation")) <= 1e-9, (x, y, m)


def test_checkerboard_of_two_different_tensors_is_the_ising_model():
    """A 2x2 cell whose two sublattices carry different tensors (the bond
    weight split as (W G)(W G^-T)^T with a non-orthogonal G): only the
    checkerboard pairing of G and G^-T legs gives back the ferromagnet, so
    Onsager's free energy and Yang's magnetisation at every site pin the
    cell's neighbour structure and site placement."""
    beta, chi = 0.5, 16
    G = np.array([[1.0, 0.35], [-0.2, 0.8]])
    t = gauged_ising(beta, G)
    sub = lambda x, y: "A" if (x + y) % 2 == 0 else "B"  # noqa: E731
    sites = [(x, y) for x in range(2) for y in range(2)]
    a = {s: t[sub(*s)][0] for s in sites}
    e = {s: t[sub(*s)][2] for s in sites}
    assert np.abs(t["A"][0] - t["B"][0]).max() > 0.1
    cell = M.cell_initial_env(a, 2, 2, lambda site, leg: e[site])
    cell, hist = M.run_cell(cell, chi, blocks(2, 2, 2 * chi, chi + 8, 11), warmup=2,
                            tol=1e-12, max_iter=80)
    assert hist[-1]["delta"] < 1e-12, hist[-1]
    for (x, y) in sites:
        m = M.cell_onesite(cell, x, y, t[sub(x, y)][1])
        assert abs(m - gold(beta, "magnetisation")) <= 1e-9, (x, y, m)
        for direction, (dx, dy), key in (("h", (1, 0), "nn_correlation"),
                                         ("v", (0, 1), "nn_correlation"),
                                         ("d", (1, 1), "diag_correlation")):
            i2 = t[sub(x + dx, y + dy)][1]
            ss = M.cell_classical_bond(cell, x, y, t[sub(x, y)][1], i2, direction)
            assert abs(ss - gold(beta, key)) <= 1e-9, (x, y, direction, ss)
    # a wrong pairing (every site with the A tensor) is not the ferromagnet
    bad = M.cell_initial_env({s: t["A"][0] for s in sites}, 2, 2, t["A"][2])
    bad, _ = M.run_cell(bad, chi, blocks(2, 2, 2 * chi, chi + 8, 11), warmup=2, tol=1e-12,
                        max_iter=40)
    assert abs(M.cell_onesite(bad, 0, 0, t["A"][1]) - gold(beta, "magnetisation")) > 1e-3


def product_cell(Lx, Ly, D, seed):
    rng = np.random.default_rng(seed)
    A, phis = {}, {}
    for x in range(Lx):
        for y in range(Ly):
            phi = rng.standard_normal(2)
            vs = [rng.standard_normal(D) for _ in range(4)]
            A[(x, y)] = np.einsum("s,u,l,d,r->suldr", phi, *vs)
            phis[(x, y)] = phi / np.linalg.norm(phi)
    return A, phis


def test_product_states_give_every_bond_exactly():
    """Nine different product states: <op> on the bond between sites s1
    and s2 is <phi_s1 phi_s2| op |phi_s1 phi_s2> exactly, for the horizontal,
    vertical and diagonal bond of every site (a non-symmetric operator, so
    that an exchange of the two sites also shows)."""
    Lx, Ly, D, chi = 3, 3, 2, 6
    A, phis = product_cell(Lx, Ly, D, 3)
    a = {s: O.double_layer(t) for s, t in A.items()}
    cell = M.cell_initial_env(a, Lx, Ly, S.trace_boundary(D), A)
    cell, hist = M.run_cell(cell, chi, blocks(Lx, Ly, chi * D * D, chi + 2, 5), warmup=1,
                            max_iter=3, warm_mode="svd")
    op = np.kron(S.pauli("x"), S.pauli("z")) + 0.3 * np.kron(S.pauli("z"), np.eye(2))
    for x in range(Lx):
        for y in range(Ly):
            for direction, (dx, dy) in (("h", (1, 0)), ("v", (0, 1)), ("d", (1, 1))):
                p1, p2 = phis[(x, y)], phis[((x + dx) % Lx, (y + dy) % Ly)]
                exact = np.kron(p1, p2) @ op @ np.kron(p1, p2)
                got = M.cell_bond_value(cell, x, y, op, direction)
                assert abs(got - exact) <= 1e-12, (x, y, direction, got, exact)


def test_turning_the_cell_exchanges_horizontal_and_vertical_bonds():
    """The converged environment of the turned cell (site (x, y) at
    (y, Lx-1-x), legs turned) gives on the vertical bond from (y, Lx-2-x)
    down to (y, Lx-1-x) the value of the original horizontal bond from (x, y)
    to (x+1, y), with the operator's two sites exchanged (the right site is
    now on top).  The two runs take their moves in a different order
    relative to the lattice, so they agree up to the truncation error,
    negligible at chi = 16 for these D = 2 states."""
    Lx, Ly, D, chi = 2, 3, 2, 16
    A = {(x, y): S.product_plus_noise_site(2, D, 30 + 3 * x + y, noise=0.3)
         for x in range(Lx) for y in range(Ly)}
    a = {s: O.double_layer(t) for s, t in A.items()}
    h = S.heisenberg_bond() + 0.2 * np.kron(S.pauli("z"), np.eye(2))
    cell = M.cell_initial_env(a, Lx, Ly, S.trace_boundary(D), A)
    cell, hist = M.run_cell(cell, chi, blocks(Lx, Ly, chi * D * D, chi + 4, 2), warmup=2,
                            tol=1e-10, max_iter=80)
    assert hist[-1]["delta"] < 1e-10
    At = {(y, Lx - 1 - x): M._turn_A(t) for (x, y), t in A.items()}
    at = {s: O.double_layer(t) for s, t in At.items()}
    tcell = M.cell_initial_env(at, Ly, Lx, S.trace_boundary(D), At)
    tcell, thist = M.run_cell(tcell, chi, blocks(Ly, Lx, chi * D * D, chi + 4, 4), warmup=2,
                              tol=1e-10, max_iter=80)
    assert thist[-1]["delta"] < 1e-10
    # swapping the two sites of the operator: the turned vertical bond runs
    # from the original right site (top) to the original left site (bottom)
    swap = np.eye(4)[[0, 2, 1, 3]]
    hs = swap @ h @ swap
    for x in range(Lx):
        for y in range(Ly):
            orig = M.cell_bond_value(cell, x, y, h, "h")
            tx, ty = y, (Lx - 1 - (x + 1)) % Lx
            turned = M.cell_bond_value(tcell, tx, ty, hs, "v")
            assert abs(orig - turned) <= 1e-9, (x, y, orig, turned)


def test_rsvd_warmup_and_full_svd_reach_the_same_environment():
    """Randomized-SVD warm-up followed by SI iterations, and full-SVD
    iterations throughout, converge to the same bond energies (a 2x2 cell
    of different noisy D=2 states)."""
    Lx, Ly, D, chi = 2, 2, 2, 8
    A = {(x, y): S.product_plus_noise_site(2, D, 50 + 2 * x + y, noise=0.4)
         for x in range(Lx) for y in range(Ly)}
    a = {s: O.double_layer(t) for s, t in A.items()}
    h = S.heisenberg_bond()
    iso = blocks(Lx, Ly, chi * D * D, chi + 4, 9)
    c0 = M.cell_initial_env(a, Lx, Ly, S.trace_boundary(D), A)
    c_si, h_si = M.run_cell(c0, chi, iso, warmup=2, warm_mode="rsvd", tol=1e-12, max_iter=100)
    assert any("rsvd" in h["modes"] for h in h_si)
    assert h_si[-1]["kind"] == "si" and h_si[-1]["delta"] < 1e-12
    c_svd, h_svd = M.run_cell(c0, chi, iso, warmup=200, warm_mode="svd", max_iter=60)
    e_si = M.cell_energy(c_si, {"h": h, "v": h, "d": h})
    e_svd = M.cell_energy(c_svd, {"h": h, "v": h, "d": h})
    assert abs(e_si - e_svd) <= 1e-10, (e_si, e_svd)


def test_planted_cell_mistakes_are_caught(monkeypatch):
    """Plausible mistakes of the cell move fail the gauged-Ising pin: the
    projectors of a cut taken from the wrong cluster (lower corners one row
    too far down), and a turn of the cell that forgets to turn the legs of
    the site tensors.  (Product states are blind to both: every positive
    environment gives their exact bond values.)"""
    beta = 0.5
    a, imp, e = bond_gauged_ising(beta, 3, 3, 21)
    assert ising_cell_errors(a, imp, e, 3, 3, beta)[0] <= 1e-9

    def shifted(cell, x, y):
        sites = (cell.at(x, y), cell.at(x + 1, y), cell.at(x + 1, y + 2), cell.at(x, y + 2))
        return [M._corner(cell.env[s], cell.a[s], i) for i, s in enumerate(sites)]

    monkeypatch.setattr(M, "_cluster_corners", shifted)
    assert not ising_cell_errors(a, imp, e, 3, 3, beta)[0] <= 1e-6
    monkeypatch.undo()
    monkeypatch.setattr(M, "_turn_a", lambda t: t)
    assert not ising_cell_errors(a, imp, e, 3, 3, beta)[0] <= 1e-6


# --------------------------------------------------------------------------
# the reverse-mode reference of the cell iteration and energy
# --------------------------------------------------------------------------
import torch  # noqa: E402

import oracle.multisite_adjoint as MA  # noqa: E402

HEIS = S.heisenberg_bond()


def full_cell(Lx, Ly, D=2, chi=8, p=4, seed=5):
    """A random PEPS cell whose environment has reached chi (two randomized
    warm-up iterations, one SI iteration), with its recycled blocks."""
    A = {(x, y): S.product_plus_noise_site(2, D, seed + 7 * x + 3 * y, noise=0.5)
         for x in range(Lx) for y in range(Ly)}
    a = {s: O.double_layer(t) for s, t in A.items()}
    N, k = chi * D * D, chi + p
    iso0 = blocks(Lx, Ly, N, k, 31)
    cell = M.cell_initial_env(a, Lx, Ly, S.trace_boundary(D), A=A)
    for _ in range(2):
        cell, _, _ = M.ctm_iteration(cell, chi, "rsvd", iso0)
    cell, cur, _ = M.ctm_iteration(cell, chi, "si", {d: dict(iso0[d]) for d in range(4)})
    assert all(e.chi == chi for e in cell.env.values())
    return cell, cur, A


def as_env(cell):
    return {s: ([c.copy() for c in e.C], [t.copy() for t in e.T]) for s, e in cell.env.items()}


def test_torch_cell_iteration_equals_the_numpy_one():
    cell, cur, A = full_cell(3, 2)
    new, iso_n, _ = M.ctm_iteration(cell, 8, "si", cur)
    tt = lambda v: torch.as_tensor(v)  # noqa: E731
    env_t = {s: ([tt(c) for c in C], [tt(t) for t in T]) for s, (C, T) in as_env(cell).items()}
    iso_t = {d: {k: (tt(X), tt(Y)) for k, (X, Y) in cur[d].items()} for d in range(4)}
    env_o, iso_o = MA.cell_iteration_torch(env_t, iso_t, {s: tt(v) for s, v in A.items()}, 3, 2, 8)
    for s, e in new.env.items():
        for g, o in zip(env_o[s][0] + env_o[s][1], e.C + e.T):
            assert np.abs(g.numpy() - o).max() <= 1e-12 * np.abs(o).max()
    # the kept columns of the recycled blocks tightly; the oversampled ones
    # (weak directions, set by rounding) loosely
    for d in range(4):
        for k, (X, Y) in iso_n[d].items():
            for g, o in ((iso_o[d][k][0].numpy(), X), (iso_o[d][k][1].numpy(), Y)):
                assert np.abs(g[:, :8] - o[:, :8]).max() <= 1e-11
                assert np.abs(g - o).max() <= 1e-8


def test_torch_cell_energy_equals_the_numpy_one():
    cell, _, A = full_cell(2, 2)
    ops = {"h": HEIS, "v": 0.5 * HEIS, "d": 0.25 * HEIS}
    e_np = M.cell_energy(cell, ops)
    tt = lambda v: torch.as_tensor(v)  # noqa: E731
    env_t = {s: ([tt(c) for c in C], [tt(t) for t in T]) for s, (C, T) in as_env(cell).items()}
    e_t = float(MA.cell_energy_torch(env_t, {s: tt(v) for s, v in A.items()}, 2, 2, ops))
    assert abs(e_t - e_np) <= 1e-13 * abs(e_np)


def _dot(a, b):
    return float(np.sum(a * b))


def test_cell_move_vjp_matches_central_differences_of_the_numpy_oracle():
    """<bar, d(iteration)> along random directions of every site tensor and of
    the environment, from central differences of the NumPy iteration."""
    Lx, Ly, chi = 2, 2, 8
    cell, cur, A = full_cell(Lx, Ly)
    rng = np.random.default_rng(3)
    new, iso_n, _ = M.ctm_iteration(cell, chi, "si", cur)
    env_b = {s: ([rng.standard_normal(c.shape) for c in e.C], [rng.standard_normal(t.shape) for t in e.T])
             for s, e in new.env.items()}
    # cotangents on the kept columns of the recycled blocks only: the
    # oversampled columns are weak directions set by rounding, whose finite
    # differences are not in the linear regime
    def kept(shape):
        b = rng.standard_normal(shape)
        b[:, chi:] = 0.0
        return b

    iso_b = {d: {k: (kept(X.shape), kept(Y.shape)) for k, (X, Y) in iso_n[d].items()}
             for d in range(4)}
    env_g, iso_g, A_g = MA.cell_move_vjp(as_env(cell), cur, A, Lx, Ly, chi, (env_b, iso_b))

    def f(cell_, A_, cur_):
        c2 = cell_.copy()
        c2.a = {s: O.double_layer(t) for s, t in A_.items()}
        out, iso_o, _ = M.ctm_iteration(c2, chi, "si", cur_)
        v = 0.0
        for s, e in out.env.items():
            v += sum(_dot(o, w) for o, w in zip(e.C + e.T, env_b[s][0] + env_b[s][1]))
        for d in range(4):
            for k, (X, Y) in iso_o[d].items():
                v += _dot(X, iso_b[d][k][0]) + _dot(Y, iso_b[d][k][1])
        return v

    h = 1e-6
    dA = {s: rng.standard_normal(t.shape) for s, t in A.items()}
    fd = (f(cell, {s: A[s] + h * dA[s] for s in A}, cur) -
          f(cell, {s: A[s] - h * dA[s] for s in A}, cur)) / (2 * h)
    an = sum(_dot(A_g[s], dA[s]) for s in A)
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)

def test_energy_after_an_iteration_matches_central_differences_along_the_environment():
    """The environment direction through a gauge-invariant function: the
    energy after one SI iteration (random environment perturbations break
    the ket-bra symmetry that pairs entries of equal magnitude, so the sign
    rule can pick other signs; closed networks do not see the signs)."""
    Lx, Ly, chi = 2, 2, 8
    cell, cur, A = full_cell(Lx, Ly)
    ops = {"h": HEIS, "v": HEIS, "d": HEIS}
    new, _, _ = M.ctm_iteration(cell, chi, "si", cur)
    _, env_b, _ = MA.cell_energy_vjp(as_env(new), A, Lx, Ly, ops)
    iso_b = {d: {k: (np.zeros_like(X), np.zeros_like(Y)) for k, (X, Y) in cur[d].items()}
             for d in range(4)}
    env_g, _, _ = MA.cell_move_vjp(as_env(cell), cur, A, Lx, Ly, chi, (env_b, iso_b))
    rng = np.random.default_rng(5)
    dE = {s: ([rng.standard_normal(c.shape) for c in e.C], [rng.standard_normal(t.shape) for t in e.T])
          for s, e in cell.env.items()}
    # the iteration carries rounding noise of ~1e-11 (weak directions of the
    # blocks), so the step is 1e-4; the central difference then agrees with
    # the adjoint to ~5e-6 relative (1e-6: noise-limited at ~1e-4)
    h = 1e-4

    def f(sign):
        c2 = cell.copy()
        for s, e in c2.env.items():
            c2.env[s] = O.Env([c + sign * h * g for c, g in zip(e.C, dE[s][0])],
                              [t + sign * h * g for t, g in zip(e.T, dE[s][1])])
        out, _, _ = M.ctm_iteration(c2, chi, "si", cur)
        return M.cell_energy(out, ops)

    fd = (f(1) - f(-1)) / (2 * h)
    an = sum(_dot(g, w) for s in env_g for g, w in zip(env_g[s][0] + env_g[s][1], dE[s][0] + dE[s][1]))
    assert abs(fd - an) <= 2e-5 * max(1e-3, abs(an)), (fd, an)


def test_cell_energy_vjp_matches_central_differences_of_the_numpy_oracle():
    Lx, Ly = 2, 2
    cell, _, A = full_cell(Lx, Ly)
    ops = {"h": HEIS, "v": HEIS, "d": HEIS}
    e, env_g, A_g = MA.cell_energy_vjp(as_env(cell), A, Lx, Ly, ops)
    assert abs(e - M.cell_energy(cell, ops)) <= 1e-13
    rng = np.random.default_rng(4)
    h = 1e-6
    dA = {s: rng.standard_normal(t.shape) for s, t in A.items()}

    def fa(sign):
        c2 = cell.copy()
        c2.A = {s: A[s] + sign * h * dA[s] for s in A}
        c2.a = {s: O.double_layer(t) for s, t in c2.A.items()}   # closed layers of the diagonal bonds
        return M.cell_energy(c2, ops)

    fd = (fa(1) - fa(-1)) / (2 * h)
    an = sum(_dot(A_g[s], dA[s]) for s in A)
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)
