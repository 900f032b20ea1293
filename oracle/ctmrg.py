"""Plain FP64 NumPy implementation of CTMRG with full-SVD and SI projectors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading of the paper used throughout (each choice is also listed with its
reason in the design notes of the repository):

* Environment (Standard CTMRG section; Fig. 1): corners ``C1..C4`` (chi x chi)
  clockwise from the top-left, edges ``T1`` (top), ``T2`` (right), ``T3``
  (bottom), ``T4`` (left).  Every tensor is ordered (in, [inner], out) going
  clockwise:  ``C1[a,b] T1[b,u,g] C2[g,h] T2[h,r,e] C3[e,z] T3[z,d,n]
  C4[n,t] T4[t,l,a]``; the inner leg of ``T1/T2/T3/T4`` meets the site leg
  ``u/r/d/l`` of ``a[u,l,d,r]``.
* Enlarged corners (Fig. 1; eq. rho_M_diag), row = in pair, column = out
  pair, each pair chi-major:
  ``Ct1[(t,d),(g,r)] = T4[t,l,a] C1[a,b] T1[b,u,g] a[u,l,d,r]`` and the
  three rotations of it.  Then ``Z_2x2 = Tr(Ct1 Ct2 Ct3 Ct4)``.
* Bond ``b`` (0 = top, 1 = right, 2 = bottom, 3 = left) sits between
  ``Ct[b]`` and ``Ct[b+1]``.  ``L_b = Ct[b-1] Ct[b]``, ``R_b = Ct[b+1]
  Ct[b+2]``, ``M_b = L_b R_b`` (indices mod 4).  The projector formulas of
  eq. svd_projectors_diag and eq. projectors_diag (``P_l = Ct2 Ct3 X v s^-1/2``,
  ``P_r = s^-1/2 u^T Y Ct4 Ct1`` for the top bond) satisfy ``P_r P_l = 1`` only
  for this ordering, so it is the one used.
* Full-SVD projectors: ``M_b = U S V^T``; ``P_l = R_b V_chi S^-1/2``,
  ``P_r = S^-1/2 U_chi^T L_b``.
* SI projectors (QR-based projector section, steps 1-3; eqs. xy_iter,
  rho_hat_diag, projectors_diag, xy_recycle): ``X <- QR(M^T M X)``,
  ``Y^T <- QR(M M^T Y^T)`` (the LQ of ``Y M M^T``), ``rho = Y M X = u s v^T``,
  ``P_l = R_b X v_chi s^-1/2``, ``P_r = s^-1/2 u_chi^T Y L_b``, then
  ``X <- X v`` and ``Y <- u^T Y`` with the full ``k x k`` factors.  With
  ``stabilized=True`` the block is re-orthonormalised after ``M`` and after
  ``M^T`` (same subspace in exact arithmetic, no loss of the weak directions
  to the squared condition number).
* QR convention: ``R_ii >= 0``.
* Sign rule (replaces the cited Bro-Acar-Kolda fix by a deterministic one):
  for every singular triple, the dominant entry of the N-dimensional left
  vector (column ``i`` of ``U``, or of ``Y^T u``) is made positive; the
  dominant entry is the lowest-index one within a relative 1e-8 of the
  largest magnitude (roundoff-level ties are resolved by index).
* Pseudo-inverse: ``s_i <= eps * s_1`` gives ``s_i^-1/2 := 0``.
* Normalisation: every new ``C`` and ``T`` is scaled to unit Frobenius norm.
* Growth phase: while the environment dimension differs from ``chi`` the
  move uses full-SVD projectors (this includes an initial boundary larger
  than ``chi``), or no truncation at all when ``chi_env * D^2 <= chi``; SI
  starts at the first move with ``chi_env == chi``.
* Convergence measure ``delta``: max over the four corners of the 2-norm of
  the change of the unit-2-norm, zero-padded singular-value spectrum.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Env",
    "SIState",
    "double_layer",
    "double_layer_op",
    "double_layer_open",
    "initial_env",
    "enlarged_corners",
    "enlarged_edges",
    "qr_pos",
    "sign_fix_columns",
    "pinv_sqrt",
    "svd_projectors",
    "si_projectors",
    "renormalize",
    "corner_spectra",
    "spectrum_delta",
    "ctm_move",
    "mean_sin2",
    "run_ctmrg",
    "norm_values",
    "kappa",
    "onesite_value",
    "bond_rdm",
    "bond_value",
    "c4v_initial_env",
    "c4v_move",
    "c4v_kappa",
    "c4v_onesite",
]

_EIN = dict(optimize=True)


# --------------------------------------------------------------------------
# data
# --------------------------------------------------------------------------
@dataclass
class Env:
    """Corner and edge tensors of a single-site environment (Fig. 1)."""

    C: List[np.ndarray]
    T: List[np.ndarray]

    @property
    def chi(self) -> int:
        return self.C[0].shape[0]

    def copy(self) -> "Env":
        return Env([c.copy() for c in self.C], [t.copy() for t in self.T])


@dataclass
class SIState:
    """Isometries of the four bonds: ``X[b]`` and ``Yt[b]`` (= Y^T), N x k."""

    X: List[np.ndarray]
    Yt: List[np.ndarray]


# --------------------------------------------------------------------------
# a1: double layer (iPEPS section, eq. double_layer)
# --------------------------------------------------------------------------
def double_layer(A: np.ndarray) -> np.ndarray:
    """``a[(uU),(lL),(dD),(rR)] = sum_s A[s,u,l,d,r] A[s,U,L,D,R]`` (ket-major)."""
    D = A.shape[1]
    a = np.einsum("sijkl,sIJKL->iIjJkKlL", A, A, **_EIN)
    return np.ascontiguousarray(a.reshape(D * D, D * D, D * D, D * D))


def double_layer_op(A: np.ndarray, O: np.ndarray) -> np.ndarray:
    """Double layer with operator ``O[t, s]`` (bra t, ket s) on the physical leg."""
    D = A.shape[1]
    a = np.einsum("sijkl,ts,tIJKL->iIjJkKlL", A, O, A, **_EIN)
    return np.ascontiguousarray(a.reshape(D * D, D * D, D * D, D * D))


def double_layer_open(A: np.ndarray) -> np.ndarray:
    """``a_open[s, t, (uU), ...] = A[s,u,l,d,r] A[t,U,L,D,R]`` (ket s, bra t)."""
    d, D = A.shape[0], A.shape[1]
    a = np.einsum("sijkl,tIJKL->stiIjJkKlL", A, A, **_EIN)
    return np.ascontiguousarray(a.reshape(d, d, D * D, D * D, D * D, D * D))


# --------------------------------------------------------------------------
# initial environment (not given by the paper; see module docstring)
# --------------------------------------------------------------------------
def initial_env(a: np.ndarray, e: np.ndarray) -> Env:
    """Close every outer leg of a boundary site with the vector ``e``."""
    C1 = np.einsum("uldr,u,l->dr", a, e, e)
    T1 = np.einsum("uldr,u->ldr", a, e)
    C2 = np.einsum("uldr,u,r->ld", a, e, e)
    T2 = np.einsum("uldr,r->uld", a, e)
    C3 = np.einsum("uldr,d,r->ul", a, e, e)
    T3 = np.einsum("uldr,d->rul", a, e)
    C4 = np.einsum("uldr,l,d->ru", a, e, e)
    T4 = np.einsum("uldr,l->dru", a, e)
    env = Env([C1, C2, C3, C4], [T1, T2, T3, T4])
    return normalize_env(env)


def normalize_env(env: Env) -> Env:
    C = [c / np.linalg.norm(c) for c in env.C]
    T = [t / np.linalg.norm(t) for t in env.T]
    return Env(C, T)


# --------------------------------------------------------------------------
# a2: enlarged corners and edges (Fig. 1; eq. rho_M_diag)
# --------------------------------------------------------------------------
def enlarged_corners(env: Env, a: np.ndarray) -> List[np.ndarray]:
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    N = env.chi * a.shape[0]
    Ct1 = np.einsum("tla,ab,bug,uldr->tdgr", T4, C1, T1, a, **_EIN)
    Ct2 = np.einsum("bug,gh,hre,uldr->bled", T1, C2, T2, a, **_EIN)
    Ct3 = np.einsum("hre,ez,zdn,uldr->hunl", T2, C3, T3, a, **_EIN)
    Ct4 = np.einsum("zdn,nt,tla,uldr->zrau", T3, C4, T4, a, **_EIN)
    return [np.ascontiguousarray(c.reshape(N, N)) for c in (Ct1, Ct2, Ct3, Ct4)]


def enlarged_edges(env: Env, a: np.ndarray) -> List[np.ndarray]:
    """``Tt_j[(in, o1), m, (out, o2)]`` with the new inner leg ``m`` in the middle."""
    T1, T2, T3, T4 = env.T
    x, D2 = env.chi, a.shape[0]
    N = x * D2
    Tt1 = np.einsum("bug,uldr->bldgr", T1, a, **_EIN)
    Tt2 = np.einsum("hre,uldr->huled", T2, a, **_EIN)
    Tt3 = np.einsum("zdn,uldr->zrunl", T3, a, **_EIN)
    Tt4 = np.einsum("tla,uldr->tdrau", T4, a, **_EIN)
    return [np.ascontiguousarray(t.reshape(N, D2, N)) for t in (Tt1, Tt2, Tt3, Tt4)]


# --------------------------------------------------------------------------
# decompositions and the sign / cutoff rules
# --------------------------------------------------------------------------
def qr_pos(W: np.ndarray) -> np.ndarray:
    """Thin Householder QR (LAPACK) with the convention ``R_ii >= 0``; returns Q."""
    q, r = np.linalg.qr(W, mode="reduced")
    sg = np.sign(np.diag(r))
    sg[sg == 0] = 1.0
    return q * sg


SIGN_TIE_RTOL = 1e-8


def sign_fix_columns(U: np.ndarray) -> np.ndarray:
    """Signs that make the dominant entry of every column positive.

    The dominant entry is the lowest-index entry whose magnitude is within a
    relative ``SIGN_TIE_RTOL`` of the column's largest magnitude, so that
    entries equal up to roundoff (frequent: the double layer is symmetric
    under exchanging ket and bra, which pairs entries of equal magnitude) are
    resolved by index and not by rounding.
    """
    A = np.abs(U)
    mx = A.max(axis=0)
    near = A >= (1.0 - SIGN_TIE_RTOL) * mx
    idx = np.argmax(near, axis=0)          # first True
    sg = np.sign(U[idx, np.arange(U.shape[1])])
    sg[sg == 0] = 1.0
    return sg


def pinv_sqrt(s: np.ndarray, eps: float) -> np.ndarray:
    """``s^-1/2`` with ``s_i <= eps * s_1`` mapped to 0."""
    out = np.zeros_like(s)
    if s.size == 0 or s[0] <= 0.0:
        return out
    keep = s > eps * s[0]
    out[keep] = 1.0 / np.sqrt(s[keep])
    return out


# --------------------------------------------------------------------------
# projectors
# --------------------------------------------------------------------------
def _L(Ct, b):
    return Ct[(b - 1) % 4] @ Ct[b]


def _R(Ct, b):
    return Ct[(b + 1) % 4] @ Ct[(b + 2) % 4]


def _apply_R(Ct, b, W):
    return Ct[(b + 1) % 4] @ (Ct[(b + 2) % 4] @ W)


def _apply_L(Ct, b, W):
    return Ct[(b - 1) % 4] @ (Ct[b] @ W)


def _apply_Rt(Ct, b, W):
    return Ct[(b + 2) % 4].T @ (Ct[(b + 1) % 4].T @ W)


def _apply_Lt(Ct, b, W):
    return Ct[b].T @ (Ct[(b - 1) % 4].T @ W)


def svd_projectors(Ct, b: int, chi: int, eps: float):
    """Standard projectors from the truncated SVD of ``M_b`` (eq. svd_projectors_diag).

    Returns ``(Pl, Prt, s)`` with ``Pl`` N x chi', ``Prt = P_r^T`` N x chi' and
    the full singular-value list of ``M_b``; ``chi' = min(chi, N)``.
    """
    L, R = _L(Ct, b), _R(Ct, b)
    U, s, Vt = np.linalg.svd(L @ R)
    sg = sign_fix_columns(U)
    U = U * sg
    Vt = Vt * sg[:, None]
    keep = min(chi, s.size)
    sinv = pinv_sqrt(s[:keep], eps)
    Pl = (R @ Vt[:keep].T) * sinv
    Prt = (L.T @ U[:, :keep]) * sinv
    return Pl, Prt, s


def si_projectors(Ct, b: int, X: np.ndarray, Yt: np.ndarray, chi: int, n_si: int,
                  eps: float, stabilized: bool = True):
    """SI-CTMRG projectors for bond ``b`` (QR-based projector section, steps 1-3).

    Returns ``(Pl, Prt, s, X_new, Yt_new)``; ``X_new = X v`` and
    ``Yt_new = Yt u`` are the gauge-recycled isometries of eq. xy_recycle.
    """
    M = lambda W: _apply_L(Ct, b, _apply_R(Ct, b, W))      # noqa: E731
    Mt = lambda W: _apply_Rt(Ct, b, _apply_Lt(Ct, b, W))   # noqa: E731
    for _ in range(n_si):
        if stabilized:
            X = qr_pos(Mt(qr_pos(M(X))))
            Yt = qr_pos(M(qr_pos(Mt(Yt))))
        else:
            X = qr_pos(Mt(M(X)))
            Yt = qr_pos(M(Mt(Yt)))
    A = _apply_R(Ct, b, X)          # R_b X
    Bt = _apply_Lt(Ct, b, Yt)       # (Y L_b)^T
    rho = Bt.T @ A                  # Y M X
    u, s, vt = np.linalg.svd(rho)
    v = vt.T
    sg = sign_fix_columns(Yt @ u)
    u = u * sg
    v = v * sg
    keep = min(chi, s.size)
    sinv = pinv_sqrt(s[:keep], eps)
    Pl = (A @ v[:, :keep]) * sinv
    Prt = (Bt @ u[:, :keep]) * sinv
    return Pl, Prt, s, X @ v, Yt @ u


# --------------------------------------------------------------------------
# a6: renormalisation (Fig. 1)
# --------------------------------------------------------------------------
def renormalize(Ct, env: Env, a: np.ndarray, Pl, Prt) -> Env:
    """``C_i' = P_r^{b(i-1)} Ct_i P_l^{b(i)}``; ``T_j' = P_r^{b(j)} Tt_j P_l^{b(j)}``.

    The enlarged edge ``Tt_j`` (see :func:`enlarged_edges`) is contracted in
    the same expression instead of being formed, which keeps memory at
    ``O(N^2)``; the result is the same sum.
    """
    x, D2 = env.chi, a.shape[0]
    T1, T2, T3, T4 = env.T
    C = [Prt[(i - 1) % 4].T @ Ct[i] @ Pl[i] for i in range(4)]
    r = lambda P: P.reshape(x, D2, P.shape[1])   # noqa: E731  (chi, D^2, chi')
    # edge j: contract the out pair with P_l, then the site, then P_r
    z = np.einsum("bug,gry->buyr", T1, r(Pl[0]), **_EIN)
    z = np.einsum("buyr,uldr->blyd", z, a, **_EIN)
    T = [np.einsum("blx,blyd->xdy", r(Prt[0]), z, **_EIN)]
    z = np.einsum("hre,edy->hyrd", T2, r(Pl[1]), **_EIN)
    z = np.einsum("hyrd,uldr->huyl", z, a, **_EIN)
    T.append(np.einsum("hux,huyl->xly", r(Prt[1]), z, **_EIN))
    z = np.einsum("zdn,nly->zydl", T3, r(Pl[2]), **_EIN)
    z = np.einsum("zydl,uldr->zryu", z, a, **_EIN)
    T.append(np.einsum("zrx,zryu->xuy", r(Prt[2]), z, **_EIN))
    z = np.einsum("tla,auy->tylu", T4, r(Pl[3]), **_EIN)
    z = np.einsum("tylu,uldr->tdyr", z, a, **_EIN)
    T.append(np.einsum("tdx,tdyr->xry", r(Prt[3]), z, **_EIN))
    return normalize_env(Env(C, T))


def renormalize_via_edges(Ct, Tt, Pl, Prt) -> Env:
    """Same as :func:`renormalize`, with the enlarged edges formed explicitly."""
    C = [Prt[(i - 1) % 4].T @ Ct[i] @ Pl[i] for i in range(4)]
    T = [np.einsum("Xx,XmY,Yy->xmy", Prt[j], Tt[j], Pl[j], **_EIN) for j in range(4)]
    return normalize_env(Env(C, T))


__all__.append("renormalize_via_edges")


def corner_spectra(env: Env, chi: int) -> np.ndarray:
    """Unit-2-norm singular values of every corner, zero-padded to ``chi``."""
    out = np.zeros((4, chi))
    for i, c in enumerate(env.C):
        s = np.linalg.svd(c, compute_uv=False)
        nrm = np.linalg.norm(s)
        s = s / nrm if nrm > 0 else s
        n = min(chi, s.size)
        out[i, :n] = s[:n]
    return out


def spectrum_delta(s_new: np.ndarray, s_old: np.ndarray) -> float:
    return float(np.max(np.linalg.norm(s_new - s_old, axis=1)))


# --------------------------------------------------------------------------
# one move (Fig. 1) and the loop around it
# --------------------------------------------------------------------------
def ctm_move(env: Env, a: np.ndarray, chi: int, proj: str = "si",
             si: Optional[SIState] = None, n_si: int = 2, eps: float = 1e-12,
             stabilized: bool = True, grow_iso: Optional[SIState] = None):
    """One simultaneous four-direction CTMRG move.

    ``proj`` is ``"si"`` or ``"svd"``.  Returns ``(env_new, info)`` where
    ``info`` holds the mode used (``grow``, ``svd``, ``grow-si`` or ``si``),
    the singular values found for each bond and the updated ``SIState`` (or
    None).

    ``grow_iso`` selects randomized projectors for a truncating growth move
    (the warm-up the paper allows to use a randomized SVD instead of the full
    one, multi-site passage): with ``chi_env < chi`` and ``N = chi_env D^2``
    at least the block width k, the SI projectors are built from the first N
    rows of the start blocks ``grow_iso``; the start blocks themselves are
    left for the first SI move.
    """
    x, D2 = env.chi, a.shape[0]
    N = x * D2
    Ct = enlarged_corners(env, a)
    info = {"svals": []}
    if N <= chi:
        Pl = [np.eye(N)] * 4
        Prt = [np.eye(N)] * 4
        info["mode"] = "grow"
    elif (proj == "si" and grow_iso is not None and x < chi
          and N >= grow_iso.X[0].shape[1]):
        Pl, Prt = [], []
        for b in range(4):
            pl, prt, s, _, _ = si_projectors(Ct, b, grow_iso.X[b][:N], grow_iso.Yt[b][:N], chi,
                                             n_si, eps, stabilized)
            Pl.append(pl)
            Prt.append(prt)
            info["svals"].append(s)
        info["mode"] = "grow-si"
    elif proj == "svd" or x != chi:
        Pl, Prt = [], []
        for b in range(4):
            pl, prt, s = svd_projectors(Ct, b, chi, eps)
            Pl.append(pl)
            Prt.append(prt)
            info["svals"].append(s)
        info["mode"] = "svd"
    else:
        if si is None:
            raise ValueError("SI move needs the isometries X, Y^T of every bond")
        Pl, Prt, Xn, Ytn = [], [], [], []
        for b in range(4):
            pl, prt, s, xn, ytn = si_projectors(Ct, b, si.X[b], si.Yt[b], chi, n_si,
                                                eps, stabilized)
            Pl.append(pl)
            Prt.append(prt)
            Xn.append(xn)
            Ytn.append(ytn)
            info["svals"].append(s)
        si = SIState(Xn, Ytn)
        info["mode"] = "si"
    info["si"] = si
    return renormalize(Ct, env, a, Pl, Prt), info


def mean_sin2(Q_old: np.ndarray, Q_new: np.ndarray, chi: int) -> float:
    """Mean squared sine of the principal angles between the spans of the
    first ``chi`` columns of two blocks (the recycling criterion of the
    triangular Heisenberg benchmark passage).  The angles come from the
    singular values of the product of orthonormal bases of the two spans."""
    A = np.linalg.qr(Q_old[:, :chi])[0]
    B = np.linalg.qr(Q_new[:, :chi])[0]
    cos = np.clip(np.linalg.svd(A.T @ B, compute_uv=False), 0.0, 1.0)
    return float(np.mean(1.0 - cos ** 2))


RECYCLE_GUARD = 10.0


def run_ctmrg(a: np.ndarray, e: np.ndarray, chi: int, proj: str = "si", k: Optional[int] = None,
              iso0: Optional[SIState] = None, n_si: int = 2, eps: float = 1e-12,
              tol: float = 0.0, max_moves: int = 100, stabilized: bool = True,
              env0: Optional[Env] = None, recycle_sin2: float = 0.0, min_si_moves: int = 3,
              growth: str = "svd"):
    """Moves from ``initial_env(a, e)`` (or ``env0``) until ``delta < tol``.

    In SI mode ``iso0`` supplies the Gaussian start blocks; they are used at
    the first move with ``chi_env == chi``.

    Recycling (QR-based projector section, step 4, and the triangular
    Heisenberg benchmark passage): with ``recycle_sin2 > 0`` the subspace
    updates stop once, after at least ``min_si_moves`` SI moves with updates,
    the largest over the eight blocks (X and Y of four bonds) of the mean
    sin^2 of the principal angles between the kept subspaces of two
    successive moves is below ``recycle_sin2``; later moves build rho and the
    projectors from the recycled blocks alone (``n_si = 0``).  The angles are
    measured only when the previous move was an SI move (the Gaussian start
    blocks are no subspace estimate).  Updates resume, and the count starts
    again, when delta grows by more than ``RECYCLE_GUARD`` from one move to
    the next (a stale subspace shows up in the corner spectra).

    ``growth = "si"`` builds the projectors of truncating growth moves from
    the first rows of ``iso0`` (see :func:`ctm_move`); ``"svd"`` uses the full
    SVD.

    Returns ``(env, history)``; each history entry holds the move number, the
    mode, delta, the subspace steps used and the measured sin^2 (or None).
    """
    env = initial_env(a, e) if env0 is None else env0.copy()
    si = None
    hist = []
    spec = corner_spectra(env, chi)
    recycling, updates, prev_delta = False, 0, None
    for n in range(max_moves):
        use_si = None
        if proj == "si" and env.chi == chi:
            if si is None:
                if iso0 is None:
                    raise ValueError("SI needs iso0")
                si = iso0
                first_si = True
            else:
                first_si = False
            use_si = si
        steps = 0 if recycling else n_si
        env, info = ctm_move(env, a, chi, proj, use_si, steps, eps, stabilized,
                             grow_iso=iso0 if growth == "si" else None)
        sin2 = None
        if info["mode"] == "si":
            new = info["si"]
            if recycle_sin2 > 0 and steps > 0:
                updates += 1
                if not first_si:
                    sin2 = max(max(mean_sin2(si.X[b], new.X[b], chi),
                                   mean_sin2(si.Yt[b], new.Yt[b], chi)) for b in range(4))
                    if updates >= min_si_moves and sin2 < recycle_sin2:
                        recycling = True
            si = new
        new_spec = corner_spectra(env, chi)
        delta = spectrum_delta(new_spec, spec)
        spec = new_spec
        if (info["mode"] == "si" and steps == 0 and prev_delta is not None
                and delta > RECYCLE_GUARD * prev_delta):
            recycling, updates = False, 0
        prev_delta = delta if info["mode"] == "si" else None
        hist.append({"move": n + 1, "mode": info["mode"], "delta": delta,
                     "n_si": steps if info["mode"] == "si" else None, "sin2": sin2})
        if delta < tol:
            break
    return env, hist


# --------------------------------------------------------------------------
# a11: observables (iPEPS section: norm network and operator insertion)
# --------------------------------------------------------------------------
def _z11(env: Env, x: np.ndarray) -> np.ndarray:
    """One-site network with site tensor ``x`` (rank 4, or rank 6 with open legs)."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    top = np.einsum("ab,bug,gh->auh", C1, T1, C2)
    bot = np.einsum("ez,zdn,nt->edt", C3, T3, C4)
    x1 = np.einsum("tla,auh->tluh", T4, top)
    x2 = np.einsum("tluh,hre->tlure", x1, T2)
    x3 = np.einsum("tlure,...uldr->...tde", x2, x)
    return np.einsum("...tde,edt->...", x3, bot)


def norm_values(env: Env, a: np.ndarray):
    """``(Z11, Z00, Z10, Z01)``: one site, no site, one column, one row."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    Z11 = _z11(env, a)
    Z00 = np.trace(C1 @ C2 @ C3 @ C4)
    Z10 = np.einsum("ab,bug,gh,hz,zun,na->", C1, T1, C2, C3, T3, C4, **_EIN)
    Z01 = np.einsum("ab,bh,hre,ez,zt,tra->", C1, C2, T2, C3, C4, T4, **_EIN)
    return float(Z11), float(Z00), float(Z10), float(Z01)


def kappa(env: Env, a: np.ndarray) -> float:
    """Norm per site ``Z11 Z00 / (Z10 Z01)``; for a classical ``a``, ln kappa = -beta f."""
    Z11, Z00, Z10, Z01 = norm_values(env, a)
    return Z11 * Z00 / (Z10 * Z01)


def onesite_value(env: Env, a: np.ndarray, a_op: np.ndarray) -> float:
    """``<O> = Z11(a_O) / Z11(a)`` for a double layer (or impurity) ``a_op``."""
    return float(_z11(env, a_op) / _z11(env, a))


def _two_site_h(env: Env, x1: np.ndarray, x2: np.ndarray) -> np.ndarray:
    """Horizontal pair (site 1 left of site 2), contracted column by column.

    ``x1, x2`` are rank-4 double layers, or rank-6 open ones ``[s, t, u, l, d, r]``
    (then the result keeps ``[s1, t1, s2, t2]``).
    """
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    left = np.einsum("ab,kla,jk->blj", C1, T4, C4)
    y1 = np.einsum("blj,bug->gulj", left, T1)
    y2 = np.einsum("gulj,...uldm->...gdmj", y1, x1)
    y3 = np.einsum("...gdmj,idj->...gmi", y2, T3)
    right = np.einsum("hc,cwe,ef->hwf", C2, T2, C3)
    w1 = np.einsum("gvh,hwf->gvwf", T1, right)
    w2 = np.einsum("gvwf,...vmyw->...gmyf", w1, x2)
    w3 = np.einsum("...gmyf,fyi->...gmi", w2, T3)
    if x1.ndim == 4:
        return np.einsum("gmi,gmi->", y3, w3)
    return np.einsum("ABgmi,EFgmi->ABEF", y3, w3)


def _two_site_v(env: Env, x1: np.ndarray, x2: np.ndarray) -> np.ndarray:
    """Vertical pair (site 1 above site 2), contracted row by row."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    top = np.einsum("ab,bug,gh->auh", C1, T1, C2)
    p1 = np.einsum("nla,auh->nluh", T4, top)
    p2 = np.einsum("nluh,...ulxr->...nxrh", p1, x1)
    p3 = np.einsum("...nxrh,hrc->...nxc", p2, T2)
    bot = np.einsum("ij,jwk,km->iwm", C3, T3, C4)
    q1 = np.einsum("csi,iwm->cswm", T2, bot)
    q2 = np.einsum("cswm,...xpws->...cxpm", q1, x2)
    q3 = np.einsum("...cxpm,mpn->...cxn", q2, T4)
    if x1.ndim == 4:
        return np.einsum("nxc,cxn->", p3, q3)
    return np.einsum("ABnxc,EFcxn->ABEF", p3, q3)


_CORNER_SPECS = ("tla,ab,bug,...uldr->...tdgr", "bug,gh,hre,...uldr->...bled",
                 "hre,ez,zdn,...uldr->...hunl", "zdn,nt,tla,...uldr->...zrau")


def _corner_with(env: Env, i: int, x: np.ndarray) -> np.ndarray:
    """Enlarged corner ``i`` (the index order of ``enlarged_corners``) with the
    site tensor ``x`` in place of ``a``: ``N x N``, or ``[s, t, N, N]`` for an
    open double layer ``x[s, t, u, l, d, r]``."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    env_ops = ((T4, C1, T1), (T1, C2, T2), (T2, C3, T3), (T3, C4, T4))[i]
    c = np.einsum(_CORNER_SPECS[i], *env_ops, x, **_EIN)
    N = env.chi * x.shape[-1]
    return c.reshape(c.shape[:-4] + (N, N))


def _two_site_diag(env: Env, x1: np.ndarray, x2: np.ndarray, anti: bool) -> np.ndarray:
    """Next-nearest (diagonal) pair on the 2x2 plaquette ``Tr(Ct1 Ct2 Ct3 Ct4)``:
    site 1 top-left and site 2 bottom-right (``anti``: site 1 top-right and
    site 2 bottom-left); the other two sites carry the plain double layer
    ``x`` closed over its physical legs."""
    o = 1 if anti else 0
    a = x1 if x1.ndim == 4 else np.einsum("ss...->...", x1)
    Ct = [_corner_with(env, i, x1 if i == o else x2 if i == o + 2 else a) for i in range(4)]
    c0, c1, c2, c3 = (Ct[(o + j) % 4] for j in range(4))
    if x1.ndim == 4:
        return np.einsum("ij,jk,kl,li->", c0, c1, c2, c3, **_EIN)
    return np.einsum("ABij,jk,EFkl,li->ABEF", c0, c1, c2, c3, **_EIN)


def bond_rdm(env: Env, A: np.ndarray, direction: str) -> np.ndarray:
    """Two-site reduced density matrix ``rho[(s1 s2), (t1 t2)]`` (ket s, bra t), trace 1.

    ``direction``: ``h`` (site 1 left of site 2), ``v`` (site 1 above site 2),
    ``d`` (site 1 top-left, site 2 bottom-right of a plaquette) or ``ad``
    (site 1 top-right, site 2 bottom-left).  The diagonal bonds are the extra
    interaction of the triangular lattice drawn on the square one
    (triangular-lattice section)."""
    ao = double_layer_open(A)
    if direction in ("d", "ad"):
        E = _two_site_diag(env, ao, ao, direction == "ad")
    else:
        E = _two_site_h(env, ao, ao) if direction == "h" else _two_site_v(env, ao, ao)
    d = A.shape[0]
    rho = E.transpose(0, 2, 1, 3).reshape(d * d, d * d)
    return rho / np.trace(rho)


def bond_value(env: Env, A: np.ndarray, op: np.ndarray, direction: str) -> float:
    """``<op>`` on a nearest-neighbour bond; ``op[(t1 t2), (s1 s2)]`` (bra, ket)."""
    rho = bond_rdm(env, A, direction)
    return float(np.trace(op @ rho))


def transfer_matrix(env: Env, a: np.ndarray, direction: str = "h") -> np.ndarray:
    """The transfer matrix of one column (``h``: moving right along a row,
    between the top edge T1 and the bottom edge T3) or of one row (``v``:
    moving down a column, between the left edge T4 and the right edge T2) of
    the converged environment (the transfer matrix whose eigenvalues give
    the correlation length, iPEPS benchmark section):
    ``E_h[(b, l, n), (g, r, z)] = T1[b,u,g] a[u,l,d,r] T3[z,d,n]``,
    ``E_v[(a, u, h), (t, d, e)] = T4[t,l,a] a[u,l,d,r] T2[h,r,e]``."""
    T1, T2, T3, T4 = env.T
    x, Dl = env.chi, a.shape[0]
    if direction == "h":
        E = np.einsum("bug,uldr,zdn->blngrz", T1, a, T3, **_EIN)
    else:
        E = np.einsum("tla,uldr,hre->auhtde", T4, a, T2, **_EIN)
    return E.reshape(x * Dl * x, x * Dl * x)


def correlation_length(env: Env, a: np.ndarray, direction: str = "h", nvals: int = 4):
    """``xi = -1 / ln(|lambda_2| / |lambda_1|)`` from the two eigenvalues of
    largest modulus of ``transfer_matrix`` (0 when lambda_2 vanishes), and the
    moduli ``|lambda_i / lambda_1|`` of the leading ``nvals`` eigenvalues."""
    w = np.sort(np.abs(np.linalg.eigvals(transfer_matrix(env, a, direction))))[::-1]
    r = w[:nvals] / w[0]
    xi = 0.0 if r[1] <= 0.0 else float(-1.0 / np.log(r[1]))
    return xi, r


__all__ += ["transfer_matrix", "correlation_length"]


def classical_bond_value(env: Env, a: np.ndarray, a1: np.ndarray, a2: np.ndarray,
                         direction: str) -> float:
    """Two impurities on a bond of a classical network, divided by the plain
    network; ``direction`` as in ``bond_rdm``."""
    if direction in ("d", "ad"):
        anti = direction == "ad"
        num, den = _two_site_diag_plain(env, a, a1, a2, anti), _two_site_diag_plain(env, a, a, a, anti)
        return float(num / den)
    f = _two_site_h if direction == "h" else _two_site_v
    return float(f(env, a1, a2) / f(env, a, a))


def _two_site_diag_plain(env: Env, a: np.ndarray, a1: np.ndarray, a2: np.ndarray,
                         anti: bool) -> float:
    """Plaquette value with rank-4 tensors ``a1``, ``a2`` on the diagonal pair
    and ``a`` on the other two sites."""
    o = 1 if anti else 0
    Ct = [_corner_with(env, i, a1 if i == o else a2 if i == o + 2 else a) for i in range(4)]
    c0, c1, c2, c3 = (Ct[(o + j) % 4] for j in range(4))
    return float(np.einsum("ij,jk,kl,li->", c0, c1, c2, c3, **_EIN))


__all__.append("classical_bond_value")


# --------------------------------------------------------------------------
# C4v specialisation (QR-based projector section; the C4v QR-CTMRG it extends)
# --------------------------------------------------------------------------
def c4v_initial_env(a: np.ndarray, e: np.ndarray):
    C = np.einsum("uldr,u,l->dr", a, e, e)
    T = np.einsum("uldr,u->ldr", a, e)
    C = 0.5 * (C + C.T)
    T = 0.5 * (T + T.transpose(2, 1, 0))
    return C / np.linalg.norm(C), T / np.linalg.norm(T)


def _order_abs(w):
    return np.argsort(-np.abs(w), kind="stable")


def c4v_move(C, T, a, chi, proj="si", X=None, n_si=2):
    """One C4v move: single symmetric corner ``Ct`` and isometric projector ``P``.

    ``svd``: ``P`` = eigenvectors of the ``chi`` largest ``|lambda|`` of ``Ct``.
    ``si``: ``X <- QR(Ct X)`` ``n_si`` times, ``rho = X^T Ct X``, eigen-
    decomposition of ``rho``, ``P = X v_chi``, ``X <- X v``.
    Returns ``(C', T', X_new, mode)``.
    """
    x, D2 = C.shape[0], a.shape[0]
    N = x * D2
    Ct = np.einsum("tla,ab,bug,uldr->tdgr", T, C, T, a, **_EIN).reshape(N, N)
    Ct = 0.5 * (Ct + Ct.T)
    Tt = np.einsum("bug,uldr->bldgr", T, a, **_EIN).reshape(N, D2, N)
    mode = "grow"
    if N <= chi:
        P = np.eye(N)
    elif proj == "svd" or x != chi:
        w, V = np.linalg.eigh(Ct)
        order = _order_abs(w)[:chi]
        P = V[:, order]
        P = P * sign_fix_columns(P)
        mode = "svd"
    else:
        for _ in range(n_si):
            X = qr_pos(Ct @ X)
        rho = X.T @ Ct @ X
        rho = 0.5 * (rho + rho.T)
        w, v = np.linalg.eigh(rho)
        order = _order_abs(w)
        v = v[:, order]
        Xv = X @ v
        sg = sign_fix_columns(Xv)
        X = Xv * sg
        P = X[:, :chi]
        mode = "si"
    Cn = P.T @ Ct @ P
    Tn = np.einsum("Xx,XmY,Yy->xmy", P, Tt, P, **_EIN)
    Cn = 0.5 * (Cn + Cn.T)
    Tn = 0.5 * (Tn + Tn.transpose(2, 1, 0))
    return Cn / np.linalg.norm(Cn), Tn / np.linalg.norm(Tn), X, mode


def c4v_env(C, T) -> Env:
    """The C4v environment written as a generic four-direction one."""
    return Env([C.copy() for _ in range(4)], [T.copy() for _ in range(4)])


__all__.append("c4v_env")


def c4v_kappa(C, T, a) -> float:
    return kappa(c4v_env(C, T), a)


def c4v_onesite(C, T, a, a_op) -> float:
    return onesite_value(c4v_env(C, T), a, a_op)
