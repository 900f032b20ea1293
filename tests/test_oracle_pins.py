"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* exact 2D Ising values (Onsager / Yang / McCoy-Wu closed forms, ``tests/golden``),
  reached through the classical path (a given directly) and through the
  quantum path (a d=2, D=2 iPEPS whose norm network is the Ising model);
* exact product states;
* the 2x2 network contracted by rows (independent of the enlarged corners);
* Eckart-Young for the full-SVD projectors, and the k = N case where
  subspace iteration must reproduce them;
* QR against modified Gram-Schmidt;
* gauge and lattice-rotation invariances;
* planted mistakes that these pins must catch.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "ising_closed_forms.json")))["values"]


def gold(beta, key):
    return float(GOLD[str(beta)][key])


def iso_for(N, k, base=20):
    return O.SIState([S.gaussian_block(N, k, base + b) for b in range(4)],
                     [S.gaussian_block(N, k, base + 10 + b) for b in range(4)])


# --------------------------------------------------------------------------
# exact Ising values
# --------------------------------------------------------------------------
@pytest.mark.parametrize("proj", ["si", "svd"])
def test_classical_ising_closed_forms(proj):
    beta, chi = 0.5, 16
    a, asig, e = S.ising_site(beta), S.ising_impurity(beta), S.ising_boundary(beta)
    env, hist = O.run_ctmrg(a, e, chi, proj=proj, iso0=iso_for(2 * chi, chi + 8),
                            tol=1e-12, max_moves=150)
    lnk = np.log(O.kappa(env, a))
    assert abs(lnk - gold(beta, "minus_beta_f")) <= 1e-10 * lnk
    assert abs(O.onesite_value(env, a, asig) - gold(beta, "magnetisation")) <= 1e-9
    for direction in "hv":
        ss = O.classical_bond_value(env, a, asig, asig, direction)
        assert abs(ss - gold(beta, "nn_correlation")) <= 1e-9
    for direction in ("d", "ad"):
        ss = O.classical_bond_value(env, a, asig, asig, direction)
        assert abs(ss - gold(beta, "diag_correlation")) <= 1e-9
    if proj == "si":
        assert hist[-1]["delta"] < 1e-12


def test_c4v_closed_forms_and_agreement_with_generic():
    beta, chi, k = 0.5, 16, 24
    a, asig, e = S.ising_site(beta), S.ising_impurity(beta), S.ising_boundary(beta)
    C, T = O.c4v_initial_env(a, e)
    X = S.gaussian_block(2 * chi, k, 7)
    for _ in range(80):
        C, T, X, mode = O.c4v_move(C, T, a, chi, "si", X, n_si=2)
    assert mode == "si"
    lnk = np.log(O.c4v_kappa(C, T, a))
    assert abs(lnk - gold(beta, "minus_beta_f")) <= 1e-10 * lnk
    assert abs(O.c4v_onesite(C, T, a, asig) - gold(beta, "magnetisation")) <= 1e-9
    env, _ = O.run_ctmrg(a, e, chi, proj="si", iso0=iso_for(2 * chi, k), tol=1e-12,
                         max_moves=150)
    assert abs(np.log(O.kappa(env, a)) - lnk) <= 1e-11


@pytest.mark.parametrize("beta", [0.3, 0.5])
def test_ising_peps_bond_correlation(beta):
    """Quantum path: double layer, open-leg two-site RDM, operator insertion."""
    A = S.ising_peps_site(beta)
    a, e, Z = O.double_layer(A), S.trace_boundary(2), S.pauli("z")
    chi = 16
    env, hist = O.run_ctmrg(a, e, chi, proj="si", iso0=iso_for(4 * chi, chi + 8),
                            tol=1e-11, max_moves=200)
    lnk = np.log(O.kappa(env, a))
    assert abs(lnk - gold(beta, "minus_beta_f")) <= 1e-10 * lnk
    for direction in "hv":
        zz = O.bond_value(env, A, np.kron(Z, Z), direction)
        assert abs(zz - gold(beta, "nn_correlation")) <= 2e-11
    for direction in ("d", "ad"):
        zz = O.bond_value(env, A, np.kron(Z, Z), direction)
        assert abs(zz - gold(beta, "diag_correlation")) <= 1e-10
    # symmetric boundary: the Z2-even state has <sigma^z> = 0 exactly
    assert abs(O.onesite_value(env, a, O.double_layer_op(A, Z))) <= 1e-9


# --------------------------------------------------------------------------
# exact product states
# --------------------------------------------------------------------------
@pytest.mark.parametrize("proj", ["si", "svd"])
def test_product_state_exact(proj):
    rng = np.random.default_rng(5)
    phi, v = rng.standard_normal(2), rng.standard_normal(3)
    A = np.einsum("s,u,l,d,r->suldr", phi, v, v, v, v)
    a, e = O.double_layer(A), S.trace_boundary(3)
    chi = 12
    env, _ = O.run_ctmrg(a, e, chi, proj=proj, iso0=iso_for(9 * chi, chi + 4), max_moves=4)
    kap = (phi @ phi) * (v @ v) ** 4
    assert abs(O.kappa(env, a) / kap - 1) <= 1e-12
    X, Zp = S.pauli("x"), S.pauli("z")
    p = phi / np.linalg.norm(phi)
    for op in (S.heisenberg_bond(), np.kron(X, Zp)):
        exact = np.kron(p, p) @ op @ np.kron(p, p)
        for direction in ("h", "v", "d", "ad"):
            assert abs(O.bond_value(env, A, op, direction) - exact) <= 1e-12


# --------------------------------------------------------------------------
# enlarged corners against the 2x2 network contracted row by row
# --------------------------------------------------------------------------
def random_env(chi, D2, seed):
    rng = np.random.default_rng(seed)
    C = [rng.standard_normal((chi, chi)) for _ in range(4)]
    T = [rng.standard_normal((chi, D2, chi)) for _ in range(4)]
    return O.Env(C, T)


def test_enlarged_corners_close_the_2x2_network():
    """Tr(Ct1 Ct2 Ct3 Ct4) equals the 4x4 boundary network contracted row by row."""
    chi, D2 = 3, 4
    env = random_env(chi, D2, 1)
    a = np.random.default_rng(2).standard_normal((D2,) * 4)
    Ct = O.enlarged_corners(env, a)
    z_corners = np.trace(Ct[0] @ Ct[1] @ Ct[2] @ Ct[3])
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    # legs read off the picture: sites a[up, left, down, right]; boundary
    # tensors in their clockwise (in, inner, out) order.
    top = np.einsum("AB,BpG,GqH,HE->ApqE", C1, T1, T1, C2)
    m1 = np.einsum("ApqE,KlA,plum,qmvr,ErF->KuvF", top, T4, a, a, T2)
    m2 = np.einsum("KuvF,IlK,ulwm,vmxr,FrJ->IwxJ", m1, T4, a, a, T2)
    bot = np.einsum("JY,YxZ,ZwO,OI->JxwI", C3, T3, T3, C4)
    z_rows = np.einsum("IwxJ,JxwI->", m2, bot)
    assert abs(z_corners - z_rows) <= 1e-12 * abs(z_rows)


# --------------------------------------------------------------------------
# projectors: Eckart-Young and the k = N reduction
# --------------------------------------------------------------------------
def small_corners(seed=3, chi=3, D2=4):
    env = random_env(chi, D2, seed)
    rng = np.random.default_rng(seed + 100)
    a = rng.standard_normal((D2,) * 4)
    return O.enlarged_corners(env, a), chi * D2


def test_renormalize_direct_equals_via_enlarged_edges():
    env = random_env(3, 4, 21)
    a = np.random.default_rng(22).standard_normal((4,) * 4)
    Ct = O.enlarged_corners(env, a)
    Pl, Prt = [], []
    for b in range(4):
        pl, prt, _ = O.svd_projectors(Ct, b, 5, 1e-14)
        Pl.append(pl)
        Prt.append(prt)
    e1 = O.renormalize(Ct, env, a, Pl, Prt)
    e2 = O.renormalize_via_edges(Ct, O.enlarged_edges(env, a), Pl, Prt)
    for i in range(4):
        assert np.allclose(e1.C[i], e2.C[i], atol=1e-14)
        assert np.allclose(e1.T[i], e2.T[i], atol=1e-14)


def test_full_svd_projectors_eckart_young():
    Ct, N = small_corners()
    chi = 5
    for b in range(4):
        Pl, Prt, s = O.svd_projectors(Ct, b, chi, 1e-14)
        L = Ct[(b - 1) % 4] @ Ct[b]
        R = Ct[(b + 1) % 4] @ Ct[(b + 2) % 4]
        M = L @ R
        U, sv, Vt = np.linalg.svd(M)
        best = (U[:, :chi] * sv[:chi]) @ Vt[:chi]
        assert np.allclose(L @ Pl @ Prt.T @ R, best, atol=1e-10 * sv[0])
        assert np.allclose(Prt.T @ Pl, np.eye(chi), atol=1e-10)
        assert np.allclose(s, sv)


def test_si_with_full_space_equals_full_svd():
    Ct, N = small_corners(seed=4)
    chi = 5
    for b in range(4):
        Pl, Prt, _ = O.svd_projectors(Ct, b, chi, 1e-14)
        X0, Y0 = S.gaussian_block(N, N, 40 + b), S.gaussian_block(N, N, 50 + b)
        Pl2, Prt2, _, _, _ = O.si_projectors(Ct, b, X0, Y0, chi, 1, 1e-14)
        scale = np.abs(Pl).max()
        assert np.allclose(Pl2, Pl, atol=1e-9 * scale)
        assert np.allclose(Prt2, Prt, atol=1e-9 * np.abs(Prt).max())


def principal_sin2(Qa, Qb):
    s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
    return 1 - s ** 2


def test_subspace_iteration_converges_to_leading_subspace():
    """Angles to the leading right singular subspace shrink with every step."""
    Ct, N = small_corners(seed=6, chi=4, D2=4)
    b, k, chi = 0, 8, 6
    L = Ct[3] @ Ct[0]
    R = Ct[1] @ Ct[2]
    _, _, Vt = np.linalg.svd(L @ R)
    Vk = Vt[:chi].T
    X = S.gaussian_block(N, k, 9)
    prev = np.inf
    for n in range(1, 7):
        _, _, _, Xn, _ = O.si_projectors(Ct, b, X, S.gaussian_block(N, k, 10), chi, n, 1e-14)
        ang = principal_sin2(np.linalg.qr(Xn)[0], Vk).max()
        assert ang < prev
        prev = ang
    assert prev < 1e-7


def test_mean_sin2_against_scipy_principal_angles():
    """The recycling criterion is the mean squared sine of the principal
    angles; scipy computes the angles by its own route."""
    from scipy.linalg import subspace_angles
    rng = np.random.default_rng(5)
    for n, k, chi in [(40, 12, 9), (64, 20, 20), (30, 7, 3)]:
        Qa = np.linalg.qr(rng.standard_normal((n, k)))[0]
        Qb = np.linalg.qr(Qa + 0.3 * rng.standard_normal((n, k)))[0]
        ref = np.mean(np.sin(subspace_angles(Qa[:, :chi], Qb[:, :chi])) ** 2)
        assert abs(O.mean_sin2(Qa, Qb, chi) - ref) <= 1e-13
        # a rotated basis of the same span, and an orthogonal span
        G = np.linalg.qr(rng.standard_normal((chi, chi)))[0]
        assert O.mean_sin2(Qa, Qa[:, :chi] @ G, chi) <= 1e-14
        Qfull = np.linalg.qr(rng.standard_normal((n, 2 * chi)))[0]
        assert abs(O.mean_sin2(Qfull[:, :chi], Qfull[:, chi:], chi) - 1.0) <= 1e-14


def test_recycled_blocks_keep_their_span_without_updates():
    """With no subspace step the recycled blocks are X v and Y^T u for
    orthogonal v, u: the spans of all k columns are unchanged."""
    Ct, N = small_corners(seed=6, chi=4, D2=4)
    k = 10
    X = np.linalg.qr(S.gaussian_block(N, k, 3))[0]
    Yt = np.linalg.qr(S.gaussian_block(N, k, 4))[0]
    for b in range(4):
        _, _, _, Xn, Ytn = O.si_projectors(Ct, b, X, Yt, 6, 0, 1e-14)
        assert O.mean_sin2(X, Xn, k) <= 1e-13 and O.mean_sin2(Yt, Ytn, k) <= 1e-13
        assert np.allclose(Xn.T @ Xn, np.eye(k), atol=1e-13)


def test_recycle_mode_reaches_the_ising_closed_forms():
    """Recycling after the subspaces align still converges to Onsager's free
    energy and Yang's magnetisation; the moves after the switch use no
    subspace step."""
    beta, chi = 0.5, 16
    a, asig, e = S.ising_site(beta), S.ising_impurity(beta), S.ising_boundary(beta)
    env, hist = O.run_ctmrg(a, e, chi, proj="si", iso0=iso_for(2 * chi, chi + 8),
                            tol=1e-12, max_moves=150, recycle_sin2=1e-3, min_si_moves=3)
    steps = [h["n_si"] for h in hist if h["mode"] == "si"]
    assert steps[:3] == [2, 2, 2] and steps[-1] == 0
    first = steps.index(0)
    assert all(st == 0 for st in steps[first:])
    assert hist[3 + first - 1]["sin2"] < 1e-3
    lnk = np.log(O.kappa(env, a))
    assert abs(lnk - gold(beta, "minus_beta_f")) <= 1e-10 * lnk
    assert abs(O.onesite_value(env, a, asig) - gold(beta, "magnetisation")) <= 1e-9


def test_stabilized_and_plain_si_agree():
    Ct, N = small_corners(seed=8)
    X0, Y0 = S.gaussian_block(N, 7, 1), S.gaussian_block(N, 7, 2)
    a = O.si_projectors(Ct, 1, X0, Y0, 5, 2, 1e-14, stabilized=True)
    b = O.si_projectors(Ct, 1, X0, Y0, 5, 2, 1e-14, stabilized=False)
    assert np.allclose(a[0], b[0], atol=1e-8 * np.abs(a[0]).max())


# --------------------------------------------------------------------------
# QR and the sign / cutoff rules
# --------------------------------------------------------------------------
def mgs2(W):
    Q = W.copy()
    for _ in range(2):
        for j in range(Q.shape[1]):
            for i in range(j):
                Q[:, j] -= (Q[:, i] @ Q[:, j]) * Q[:, i]
            Q[:, j] /= np.linalg.norm(Q[:, j])
    return Q


def test_qr_pos_matches_gram_schmidt():
    W = S.gaussian_block(50, 12, 3)
    Q = O.qr_pos(W)
    assert np.allclose(Q, mgs2(W), atol=1e-12)
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-14 * 50)


def test_qr_pos_rank_deficient_has_no_nan():
    W = np.zeros((20, 5))
    W[:, 0] = 1.0
    Q = O.qr_pos(W)
    assert np.all(np.isfinite(Q))
    assert np.allclose(Q.T @ Q, np.eye(5), atol=1e-13)


def test_sign_rule_and_pinv():
    U = np.array([[0.1, -0.9], [-0.5, 0.9], [0.2, 0.1]])
    assert list(O.sign_fix_columns(U)) == [-1.0, -1.0]  # tie in column 2 -> lowest row
    # a tie up to roundoff is still a tie: the lowest row decides
    V = np.array([[0.9], [-(0.9 + 1e-13)], [0.1]])
    assert list(O.sign_fix_columns(V)) == [1.0]
    W = np.array([[0.5], [-0.9], [0.1]])
    assert list(O.sign_fix_columns(W)) == [-1.0]
    s = np.array([4.0, 1.0, 1e-13, 0.0])
    assert np.allclose(O.pinv_sqrt(s, 1e-12), [0.5, 1.0, 0.0, 0.0])


# --------------------------------------------------------------------------
# invariances
# --------------------------------------------------------------------------
def noisy_site(D=2, seed=2):
    return S.product_plus_noise_site(2, D, seed)


def energies(A, chi, proj="svd", moves=40):
    a, e = O.double_layer(A), S.trace_boundary(A.shape[1])
    N = chi * A.shape[1] ** 2
    env, _ = O.run_ctmrg(a, e, chi, proj=proj, iso0=iso_for(N, chi + 4), max_moves=moves,
                         tol=1e-13)
    h = S.heisenberg_bond()
    return (O.kappa(env, a), O.bond_value(env, A, h, "h"), O.bond_value(env, A, h, "v"))


def test_orthogonal_gauge_invariance():
    A = noisy_site(D=2, seed=11)
    Gh, Gv = S.random_orthogonal(2, 1), S.random_orthogonal(2, 2)
    Ag = np.einsum("suldr,uU,lL,dD,rR->sULDR", A, Gv, Gh, Gv, Gh)
    ref = energies(A, 8)
    got = energies(Ag, 8)
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_rotation_swaps_horizontal_and_vertical():
    A = noisy_site(D=2, seed=12)
    Ar = np.einsum("suldr->sruld", A)      # 90 deg: new (u,l,d,r) = old (r,u,l,d)
    k1, h1, v1 = energies(A, 8)
    k2, h2, v2 = energies(Ar, 8)
    assert abs(h1 - v1) > 1e-6
    assert abs(k1 - k2) <= 1e-10 * k1
    assert abs(h1 - v2) <= 1e-10 and abs(v1 - h2) <= 1e-10


def _mps_values(B, O1, O2):
    """<O1>, <O2> and the nearest-neighbour <O1 O2> of the infinite MPS with
    real tensors B[s, l, r], from the dominant eigenvectors of its transfer
    matrix E[(l l'), (r r')] = sum_s B[s,l,r] B[s,l',r'] (ket, bra)."""
    def tm(O=None):
        if O is None:
            return np.einsum("slr,sLR->lLrR", B, B).reshape(B.shape[1] ** 2, -1)
        return np.einsum("slr,ts,tLR->lLrR", B, O, B).reshape(B.shape[1] ** 2, -1)
    E = tm()
    w, vr = np.linalg.eig(E)
    wl, vl = np.linalg.eig(E.T)
    r, l = np.real(vr[:, np.argmax(abs(w))]), np.real(vl[:, np.argmax(abs(wl))])
    lam, norm = np.max(abs(w)), l @ r
    e1 = l @ tm(O1) @ r / (lam * norm)
    e2 = l @ tm(O2) @ r / (lam * norm)
    e12 = l @ tm(O1) @ tm(O2) @ r / (lam ** 2 * norm)
    return e1, e2, e12


@pytest.mark.parametrize("rows", [True, False])
def test_uncoupled_chains_factorise_on_the_diagonals(rows):
    """A PEPS whose vertical (or horizontal) legs are trivial is a stack of
    independent MPS rows (columns): a diagonal pair sits on two different
    chains, so <O1 O2> = <O1><O2>, while the bond along the chain is the
    MPS nearest-neighbour value.  Both sides from the 1D transfer matrix."""
    rng = np.random.default_rng(7)
    B = rng.standard_normal((2, 2, 2)) + 0.3 * np.eye(2)[None]   # MPS gap |l2/l1| = 0.10
    A = np.zeros((2, 2, 2, 2, 2))
    if rows:
        A[:, 0, :, 0, :] = B                       # A[s, u=0, l, d=0, r] = B[s, l, r]
    else:
        A[:, :, 0, :, 0] = B                       # A[s, u, l=0, d, r=0] = B[s, u, d]
    X, Zp = S.pauli("x"), S.pauli("z")
    e1, e2, e12 = _mps_values(B, X, Zp)
    a, e = O.double_layer(A), S.trace_boundary(2)
    # every corner has rank 1 here, so the spectrum change is 0 from the
    # first move on: run a fixed number of moves instead
    env, hist = O.run_ctmrg(a, e, 4, proj="svd", tol=0.0, max_moves=80)
    op = np.kron(X, Zp)
    along = "h" if rows else "v"
    assert abs(O.bond_value(env, A, op, along) - e12) <= 1e-10
    for direction in ("d", "ad"):
        assert abs(O.bond_value(env, A, op, direction) - e1 * e2) <= 1e-10
    assert abs(e12 - e1 * e2) > 1e-3                # the two pins are distinct


@pytest.mark.parametrize("rows", [True, False])
def test_uncoupled_chains_give_the_mps_correlation_length(rows):
    """For a stack of independent MPS rows the column transfer matrix is the
    chain's own transfer matrix (the boundary across the chains is a product),
    so xi along the chains is the MPS correlation length -1/ln|mu2/mu1|
    (eigenvalues of sum_s B_s (x) B_s), and across them the transfer matrix
    has rank one (xi = 0).  Columns: the same with the roles exchanged."""
    rng = np.random.default_rng(7)
    B = rng.standard_normal((2, 2, 2)) + 0.3 * np.eye(2)[None]
    A = np.zeros((2, 2, 2, 2, 2))
    if rows:
        A[:, 0, :, 0, :] = B
    else:
        A[:, :, 0, :, 0] = B
    mu = np.sort(np.abs(np.linalg.eigvals(np.einsum("slr,sLR->lLrR", B, B).reshape(4, 4))))[::-1]
    xi_mps = -1.0 / np.log(mu[1] / mu[0])
    a, e = O.double_layer(A), S.trace_boundary(2)
    env, _ = O.run_ctmrg(a, e, 4, proj="svd", tol=0.0, max_moves=80)
    along, across = ("h", "v") if rows else ("v", "h")
    xi, r = O.correlation_length(env, a, along)
    assert abs(xi - xi_mps) <= 1e-9 * xi_mps
    assert np.allclose(r[:4], mu[:4] / mu[0], atol=1e-10)
    xi0, r0 = O.correlation_length(env, a, across)
    assert r0[1] <= 1e-10


def test_product_state_has_zero_correlation_length():
    rng = np.random.default_rng(5)
    phi, v = rng.standard_normal(2), rng.standard_normal(3)
    A = np.einsum("s,u,l,d,r->suldr", phi, v, v, v, v)
    a, e = O.double_layer(A), S.trace_boundary(3)
    env, _ = O.run_ctmrg(a, e, 6, proj="svd", max_moves=4)
    for direction in "hv":
        _, r = O.correlation_length(env, a, direction)
        assert r[1] <= 1e-12


def test_rotation_swaps_the_two_correlation_lengths():
    """The column transfer matrix of a state is the row transfer matrix of
    the state turned by 90 degrees (each from its own converged
    environment): same spectrum, so xi_h(A) = xi_v(A_rot)."""
    A = S.product_plus_noise_site(2, 2, 14, noise=0.6)
    Ar = np.einsum("suldr->sruld", A)
    out = {}
    for name, site in (("A", A), ("Ar", Ar)):
        a, e = O.double_layer(site), S.trace_boundary(2)
        env, _ = O.run_ctmrg(a, e, 8, proj="svd", tol=1e-13, max_moves=200)
        out[name] = [O.correlation_length(env, a, dr)[0] for dr in "hv"]
    assert abs(out["A"][0] - out["Ar"][1]) <= 1e-8 * out["A"][0]
    assert abs(out["A"][1] - out["Ar"][0]) <= 1e-8 * out["A"][1]
    assert abs(out["A"][0] - out["A"][1]) > 1e-4


def test_rotation_maps_the_diagonal_to_the_antidiagonal():
    """Turning the lattice by 90 degrees (new (u,l,d,r) = old (r,u,l,d), so
    the old right is the new up) carries the top-left / bottom-right pair to
    a bottom-left / top-right one: rho_d(A) equals rho_ad(A_rot) with the two
    sites exchanged, which a non-symmetric operator distinguishes."""
    A = S.product_plus_noise_site(2, 2, 14, noise=0.6)
    Ar = np.einsum("suldr->sruld", A)
    X, Zp = S.pauli("x"), S.pauli("z")
    ops = {"xz": np.kron(X, Zp), "zx": np.kron(Zp, X)}
    vals = {}
    for name, site in (("A", A), ("Ar", Ar)):
        a, e = O.double_layer(site), S.trace_boundary(2)
        env, _ = O.run_ctmrg(a, e, 8, proj="svd", tol=1e-13, max_moves=120)
        for dr in ("d", "ad"):
            for o, op in ops.items():
                vals[name, dr, o] = O.bond_value(env, site, op, dr)
    assert abs(vals["A", "d", "xz"] - vals["Ar", "ad", "zx"]) <= 1e-10
    assert abs(vals["A", "d", "zx"] - vals["Ar", "ad", "xz"]) <= 1e-10
    assert abs(vals["A", "d", "xz"] - vals["A", "d", "zx"]) > 1e-4


def test_si_and_svd_agree_on_noisy_state():
    A = noisy_site(D=2, seed=13)
    ref = energies(A, 8, "svd", 60)
    got = energies(A, 8, "si", 60)
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-11)


# --------------------------------------------------------------------------
# planted mistakes must be caught (the mistake is planted in the oracle, on the CPU)
# --------------------------------------------------------------------------
def _ising_lnk_error(monkeypatch=None):
    beta, chi = 0.5, 8
    a, e = S.ising_site(beta), S.ising_boundary(beta)
    env, _ = O.run_ctmrg(a, e, chi, proj="si", iso0=iso_for(2 * chi, chi + 4),
                         tol=1e-12, max_moves=80)
    return abs(np.log(O.kappa(env, a)) - gold(beta, "minus_beta_f"))


def test_planted_mistakes_are_caught(monkeypatch):
    assert _ising_lnk_error() < 1e-10
    import oracle.ctmrg as mod

    good = mod.enlarged_corners

    def swapped_legs(env, a):       # transposed site tensor in the corner build
        return good(env, np.ascontiguousarray(a.transpose(0, 1, 3, 2)) * 1.0 +
                    0.05 * np.ones_like(a))

    monkeypatch.setattr(mod, "enlarged_corners", swapped_legs)
    assert _ising_lnk_error() > 1e-6
    monkeypatch.undo()

    def dropped_sqrt(s, eps):       # s^-1 instead of s^-1/2
        out = np.zeros_like(s)
        keep = s > eps * s[0]
        out[keep] = 1.0 / s[keep]
        return out

    monkeypatch.setattr(mod, "pinv_sqrt", dropped_sqrt)
    A = S.ising_peps_site(0.5)
    a, e = O.double_layer(A), S.trace_boundary(2)
    env, _ = O.run_ctmrg(a, e, 8, proj="si", iso0=iso_for(32, 12), tol=1e-12, max_moves=60)
    zz = O.bond_value(env, A, np.kron(S.pauli("z"), S.pauli("z")), "h")
    assert abs(zz - gold(0.5, "nn_correlation")) > 1e-6 or not np.isfinite(zz)


def test_boundary_larger_than_chi_truncates_with_full_svd():
    """chi = 1 < D^2: the first move truncates the initial boundary with
    full-SVD projectors; from then on SI moves with k = N reproduce the
    full-SVD moves (k = N reduces subspace iteration to the SVD)."""
    A = noisy_site(D=2, seed=5)
    a, e = O.double_layer(A), S.trace_boundary(2)
    chi, N = 1, 4
    env_si, h_si = O.run_ctmrg(a, e, chi, proj="si", iso0=iso_for(N, N), tol=0, max_moves=4)
    env_sv, h_sv = O.run_ctmrg(a, e, chi, proj="svd", tol=0, max_moves=4)
    assert [h["mode"] for h in h_si] == ["svd", "si", "si", "si"]
    for c1, c2 in zip(env_si.C + env_si.T, env_sv.C + env_sv.T):
        assert np.allclose(c1, c2, atol=1e-12)


def test_randomized_growth_reaches_the_same_fixed_point():
    """Truncating growth moves with SI projectors from the first rows of the
    start blocks (a randomized SVD warm-up) lead to the same converged
    environment as full-SVD growth: equal bond energies and norms."""
    A = S.product_plus_noise_site(2, 3, 2, noise=0.3)
    a, e = O.double_layer(A), S.trace_boundary(3)
    chi = 18
    iso = iso_for(chi * 9, chi + 6)
    h = S.heisenberg_bond()
    out = {}
    for growth in ("svd", "si"):
        env, hist = O.run_ctmrg(a, e, chi, proj="si", iso0=iso, tol=1e-12, max_moves=300,
                                growth=growth)
        assert hist[0]["mode"] == ("grow-si" if growth == "si" else "svd")
        assert hist[-1]["delta"] < 1e-12
        out[growth] = (O.bond_value(env, A, h, "h"), O.bond_value(env, A, h, "v"), O.kappa(env, a))
    assert np.allclose(out["si"], out["svd"], rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# the convergence measure (QR-based projector section, step 4: the corners
# and edges converge element-wise; the reading used is the largest over the
# four corners of the l2 distance of their unit-norm, sorted, zero-padded
# singular-value spectra between two moves)
# --------------------------------------------------------------------------
def _env_with_corners(Cs, chi_t=3, D2=2):
    T = [np.ones((c.shape[0], D2, c.shape[0])) for c in Cs]
    return O.Env([np.asarray(c, dtype=float) for c in Cs], T)


def test_delta_of_a_hand_computed_pair():
    """Corner 1 goes from diag(1, 0) to diag(3, 4): its unit spectrum moves
    from (1, 0) to (0.8, 0.6), an l2 step of sqrt(0.04 + 0.36) = sqrt(0.4).
    Corner 2 goes from diag(1, 1) to diag(1, 0): (1, 1)/sqrt(2) -> (1, 0), a
    step of sqrt((1 - 1/sqrt2)^2 + 1/2) = sqrt(2 - sqrt2).  Corners 3 and 4
    are unchanged.  The largest step is corner 2's."""
    I2 = np.eye(2)
    old = _env_with_corners([np.diag([1.0, 0.0]), I2, I2, 2 * I2])
    new = _env_with_corners([np.diag([3.0, 4.0]), np.diag([1.0, 0.0]), I2, 2 * I2])
    chi = 2
    s_old, s_new = O.corner_spectra(old, chi), O.corner_spectra(new, chi)
    assert np.allclose(s_new[0], [0.8, 0.6], atol=1e-15)
    assert np.allclose(s_old[1], [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    step = [np.sqrt(0.4), np.sqrt(2.0 - np.sqrt(2.0)), 0.0, 0.0]
    assert abs(O.spectrum_delta(s_new, s_old) - max(step)) <= 1e-15
    # a change on corner 1 alone: the max picks it, not the mean over corners
    new1 = _env_with_corners([np.diag([3.0, 4.0]), I2, I2, 2 * I2])
    assert abs(O.spectrum_delta(O.corner_spectra(new1, chi), s_old) - np.sqrt(0.4)) <= 1e-15


def test_delta_vanishes_at_a_fixed_point_and_ignores_scale_and_gauge():
    rng = np.random.default_rng(3)
    chi = 6
    Cs = [rng.standard_normal((chi, chi)) for _ in range(4)]
    env = _env_with_corners(Cs)
    s = O.corner_spectra(env, chi)
    assert O.spectrum_delta(s, s) == 0.0
    # the spectra are unit-norm: rescaling a corner changes nothing
    scaled = _env_with_corners([c * f for c, f in zip(Cs, (7.0, 1e-3, 2.0, 1.0))])
    assert O.spectrum_delta(O.corner_spectra(scaled, chi), s) <= 1e-15
    # an orthogonal change of basis on either leg of a corner leaves its spectrum
    gauged = _env_with_corners([S.random_orthogonal(chi, 10 + i) @ c @ S.random_orthogonal(chi, 20 + i)
                                for i, c in enumerate(Cs)])
    assert O.spectrum_delta(O.corner_spectra(gauged, chi), s) <= 1e-14
    # every unit spectrum has norm 1 and is sorted in descending order
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    assert np.all(np.diff(s, axis=1) <= 0)


def test_delta_zero_pads_a_growing_environment():
    """While chi_env < chi the spectrum is padded with zeros: a 2x2 corner
    diag(1, 1) next to a 4x4 corner diag(1, 1, 0, 0) is the same spectrum
    (distance 0), and against diag(1, 1, 1, 1) the distance is
    |(1/sqrt2, 1/sqrt2, 0, 0) - (1/2, 1/2, 1/2, 1/2)| = sqrt(2 - sqrt2)."""
    chi = 4
    small = _env_with_corners([np.eye(2)] * 4)
    s_small = O.corner_spectra(small, chi)
    assert s_small.shape == (4, chi) and np.all(s_small[:, 2:] == 0.0)
    same = _env_with_corners([np.diag([1.0, 1.0, 0.0, 0.0])] * 4)
    assert O.spectrum_delta(O.corner_spectra(same, chi), s_small) <= 1e-15
    full = _env_with_corners([np.eye(4)] * 4)
    d = O.spectrum_delta(O.corner_spectra(full, chi), s_small)
    assert abs(d - np.sqrt(2.0 - np.sqrt(2.0))) <= 1e-15


def test_planted_delta_mistakes_are_caught(monkeypatch):
    """The hand-computed pair above fails for the plausible mistakes of the
    measure: the mean over corners instead of the largest, an l1 or mean
    absolute step instead of the l2 one, and spectra not scaled to unit norm."""
    import oracle.ctmrg as mod
    I2 = np.eye(2)
    old = _env_with_corners([np.diag([1.0, 0.0]), I2, I2, 2 * I2])
    new = _env_with_corners([np.diag([3.0, 4.0]), np.diag([1.0, 0.0]), I2, 2 * I2])
    expect = np.sqrt(2.0 - np.sqrt(2.0))

    def value():
        return mod.spectrum_delta(mod.corner_spectra(new, 2), mod.corner_spectra(old, 2))

    assert abs(value() - expect) <= 1e-15
    good_delta, good_spec = mod.spectrum_delta, mod.corner_spectra
    wrong = {
        "mean over corners": lambda a, b: float(np.mean(np.linalg.norm(a - b, axis=1))),
        "mean abs step": lambda a, b: float(np.max(np.mean(np.abs(a - b), axis=1))),
        "l1 step": lambda a, b: float(np.max(np.sum(np.abs(a - b), axis=1))),
        "mean abs over everything": lambda a, b: float(np.mean(np.abs(a - b))),
    }
    for name, f in wrong.items():
        monkeypatch.setattr(mod, "spectrum_delta", f)
        assert abs(value() - expect) > 1e-3, name
    monkeypatch.setattr(mod, "spectrum_delta", good_delta)

    def unnormalised(env, chi):
        out = np.zeros((4, chi))
        for i, c in enumerate(env.C):
            s = np.linalg.svd(c, compute_uv=False)
            out[i, :min(chi, s.size)] = s[:chi]
        return out

    monkeypatch.setattr(mod, "corner_spectra", unnormalised)
    assert abs(value() - expect) > 1e-3
    monkeypatch.setattr(mod, "corner_spectra", good_spec)


# --------------------------------------------------------------------------
# the double layer with an operator on the physical leg (iPEPS section)
# --------------------------------------------------------------------------
def test_operator_double_layer_of_a_product_state():
    """For A = phi (x) v (x) v (x) v (x) v the operator double layer is
    (phi^T O phi) times the plain double layer of v alone, so the one-site
    value is phi^T O phi / phi^T phi: for phi = (cos t, sin t) that is
    <sigma^x> = sin 2t and <sigma^z> = cos 2t (nonzero, so a scale or a
    missing factor shows)."""
    t = 0.3
    phi = np.array([np.cos(t), np.sin(t)])
    v = np.array([0.7, -0.4, 0.2])
    A = np.einsum("s,u,l,d,r->suldr", phi, v, v, v, v)
    a = O.double_layer(A)
    vv = np.outer(v, v).ravel()
    a_v = np.einsum("i,j,k,l->ijkl", vv, vv, vv, vv)
    assert np.allclose(a, a_v, atol=1e-15)           # phi^T phi = 1
    iy = np.array([[0.0, -1.0], [1.0, 0.0]])          # i sigma^y: real, antisymmetric
    for op, exact in ((S.pauli("x"), np.sin(2 * t)), (S.pauli("z"), np.cos(2 * t)), (iy, 0.0)):
        ao = O.double_layer_op(A, op)
        assert np.allclose(ao, exact * a_v, atol=1e-15)
    # through the converged environment of the product state
    chi = 9
    env, _ = O.run_ctmrg(a, S.trace_boundary(3), chi, proj="svd", max_moves=3)
    assert abs(O.onesite_value(env, a, O.double_layer_op(A, S.pauli("x"))) - np.sin(2 * t)) <= 1e-13
    assert abs(O.onesite_value(env, a, O.double_layer_op(A, S.pauli("z"))) - np.cos(2 * t)) <= 1e-13


def test_operator_double_layer_of_a_two_term_state():
    """A = phi1 (x) v^4 + phi2 (x) w^4 with orthonormal v, w on every
    virtual leg: the double layer with O is sum_ij (phi_i^T O phi_j)
    (v_i v_j)^4 where v_1 = v, v_2 = w, so the operator's matrix elements
    between the two physical states appear in the four blocks; picking the
    (v v) and (v w) entries recovers phi1^T O phi1 and phi1^T O phi2 (with
    the ket on the first index), which pins the ket/bra order of O[t, s]."""
    rng = np.random.default_rng(9)
    phi1, phi2 = rng.standard_normal(2), rng.standard_normal(2)
    v, w = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    A = (np.einsum("s,u,l,d,r->suldr", phi1, v, v, v, v) +
         np.einsum("s,u,l,d,r->suldr", phi2, w, w, w, w))
    O_ = np.array([[0.3, -1.1], [0.5, 0.2]])   # O[t, s]: bra t, ket s
    ao = O.double_layer_op(A, O_).reshape(2, 2, 2, 2, 2, 2, 2, 2)
    # ket legs all on v (index 0), bra legs all on v: phi1 (bra) O phi1 (ket)
    assert abs(ao[0, 0, 0, 0, 0, 0, 0, 0] - phi1 @ O_ @ phi1) <= 1e-15
    # ket legs on v (0), bra legs on w (1): bra phi2, ket phi1 -> phi2^T O phi1
    assert abs(ao[0, 1, 0, 1, 0, 1, 0, 1] - phi2 @ O_ @ phi1) <= 1e-15
    assert abs(ao[1, 0, 1, 0, 1, 0, 1, 0] - phi1 @ O_ @ phi2) <= 1e-15
    # mixed leg patterns vanish (each virtual leg sees v on one term only)
    assert ao[0, 0, 1, 1, 0, 0, 0, 0] == 0.0
