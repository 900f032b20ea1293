"""Pins of the reverse-mode reference (oracle.adjoint), on the CPU.

The autograd reference is pinned to something other than itself:

* its forward move equals the NumPy move of oracle.ctmrg (pinned by the
  closed forms and invariances of test_oracle_pins) to rounding;
* its vector-Jacobian product, contracted with a random direction, equals
  the central finite difference of the NumPy move along that direction, for
  each input group separately (corners, edges, X, Y^T, site tensor), so a
  wrong or missing term in any group fails;
* a planted gradient mistake that leaves the forward move unchanged (the
  pseudo-inverse square root detached) is caught by the finite differences.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import oracle.adjoint as J  # noqa: E402
import synth as S  # noqa: E402


def case(D=2, chi=4, p=4, seed=11):
    A = S.product_plus_noise_site(2, D, seed, noise=1.0)
    Dl, N, k = D * D, chi * D * D, chi + p
    C = [S.gaussian_block(chi, chi, 60 + i) for i in range(4)]
    T = [S.gaussian_block(chi * Dl, chi, 70 + i).reshape(chi, Dl, chi) for i in range(4)]
    X = [np.linalg.qr(S.gaussian_block(N, k, 20 + b))[0] for b in range(4)]
    Y = [np.linalg.qr(S.gaussian_block(N, k, 30 + b))[0] for b in range(4)]
    return A, C, T, X, Y


def move_np(C, T, X, Y, A, chi, n_si):
    env, info = O.ctm_move(O.Env([c.copy() for c in C], [t.copy() for t in T]),
                           O.double_layer(A), chi, "si", O.SIState(list(X), list(Y)), n_si,
                           1e-12, True)
    return env.C, env.T, info["si"].X, info["si"].Yt


def tens(vs):
    return [torch.tensor(v) for v in vs]


@pytest.mark.parametrize("n_si", [1, 2])
def test_torch_move_equals_numpy_move(n_si):
    A, C, T, X, Y = case()
    ref = move_np(C, T, X, Y, A, 4, n_si)
    got = J.move_torch(tens(C), tens(T), tens(X), tens(Y), torch.tensor(A), 4, n_si)
    for r, g in zip(ref, got):
        for u, v in zip(r, g):
            assert np.abs(u - v.numpy()).max() <= 1e-12


@pytest.mark.parametrize("group", ["C", "T", "X", "Y", "A"])
def test_vjp_matches_central_differences_of_the_numpy_move(group):
    chi, n_si = 4, 2
    A, C, T, X, Y = case()
    rng = np.random.default_rng(3)
    out = move_np(C, T, X, Y, A, chi, n_si)
    bars = [[rng.standard_normal(v.shape) for v in grp] for grp in out]
    gC, gT, gX, gY, gA = J.move_vjp(C, T, X, Y, A, bars, chi, n_si)
    ins = {"C": C, "T": T, "X": X, "Y": Y, "A": [A]}
    grads = {"C": gC, "T": gT, "X": gX, "Y": gY, "A": [gA]}
    for trial in range(2):
        d = [rng.standard_normal(v.shape) for v in ins[group]]

        def f(h):
            moved = {g: [v.copy() for v in vs] for g, vs in ins.items()}
            moved[group] = [v + h * dv for v, dv in zip(ins[group], d)]
            o = move_np(moved["C"], moved["T"], moved["X"], moved["Y"], moved["A"][0],
                        chi, n_si)
            return sum((oo * w).sum() for grp, wg in zip(o, bars) for oo, w in zip(grp, wg))

        h = 1e-6
        fd = (f(h) - f(-h)) / (2 * h)
        an = sum((g * dv).sum() for g, dv in zip(grads[group], d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (group, trial, fd, an)


def test_planted_detached_pinv_is_caught(monkeypatch):
    """A gradient mistake that leaves the forward move unchanged (s^-1/2
    treated as a constant) must fail the finite-difference comparison."""
    chi, n_si = 4, 2
    A, C, T, X, Y = case()
    rng = np.random.default_rng(3)
    out = move_np(C, T, X, Y, A, chi, n_si)
    bars = [[rng.standard_normal(v.shape) for v in grp] for grp in out]
    good = J._pinv_sqrt
    monkeypatch.setattr(J, "_pinv_sqrt", lambda s, eps: good(s.detach(), eps))
    gA = J.move_vjp(C, T, X, Y, A, bars, chi, n_si)[4]
    d = rng.standard_normal(A.shape)

    def f(h):
        o = move_np(C, T, X, Y, A + h * d, chi, n_si)
        return sum((oo * w).sum() for grp, wg in zip(o, bars) for oo, w in zip(grp, wg))

    fd = (f(1e-6) - f(-1e-6)) / 2e-6
    an = (gA * d).sum()
    assert abs(fd - an) > 1e-3 * abs(fd)


@pytest.mark.parametrize("bonds", ["hv", "da", "hvd"])
def test_energy_gradient_matches_central_differences_of_bond_values(bonds):
    """The torch energy equals the NumPy bond values, and its autograd
    gradient matches central differences of oracle.ctmrg.bond_value for the
    corners, the edges and the site tensor (nearest-neighbour bonds, the two
    diagonals, and the triangular-lattice sum h + v + d).  The operator is
    not symmetric under exchange of the two sites, so a swapped site order
    in the diagonal reference would show."""
    A, C, T, _, _ = case(D=2, chi=4)
    h = S.heisenberg_bond() + 0.3 * np.kron(S.pauli("x"), S.pauli("z"))
    env = O.Env(C, T)
    names = {"h": "h", "v": "v", "d": "d", "a": "ad"}

    def e_np(C_, T_, A_):
        en = O.Env(C_, T_)
        return sum(O.bond_value(en, A_, h, names[b]) for b in bonds)

    e, gC, gT, gA = J.energy_vjp(C, T, A, h, bonds)
    assert abs(e - e_np(env.C, env.T, A)) <= 1e-12
    rng = np.random.default_rng(4)
    for group in ("C", "T", "A"):
        d = ([rng.standard_normal(c.shape) for c in C] if group == "C" else
             [rng.standard_normal(t.shape) for t in T] if group == "T" else
             rng.standard_normal(A.shape))

        def f(hh):
            if group == "C":
                return e_np([c + hh * dc for c, dc in zip(C, d)], T, A)
            if group == "T":
                return e_np(C, [t + hh * dt for t, dt in zip(T, d)], A)
            return e_np(C, T, A + hh * d)

        fd = (f(1e-6) - f(-1e-6)) / 2e-6
        an = (sum((g * dd).sum() for g, dd in zip(gC, d)) if group == "C" else
              sum((g * dd).sum() for g, dd in zip(gT, d)) if group == "T" else (gA * d).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (group, fd, an)
