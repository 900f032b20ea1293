"""Reverse-mode reference for one SI-CTMRG move -- TEST INFRASTRUCTURE ONLY.

The paper differentiates CTMRG by vector-Jacobian products of the single
move (Differentiable fixed point passage, eq. implicit; its timing figure
unrolls the moves instead).  This module writes the move of
:mod:`oracle.ctmrg` a second time, in PyTorch on the CPU in float64, so that
``torch.autograd`` gives the vector-Jacobian product of the move:

    (C, T, X, Y^T, A)  ->  (C', T', X', Y^T')

with the same index conventions, the same order of operations (enlarged
corners, n_si stabilised subspace steps per bond, rho = Y M X and its SVD,
projectors with the pseudo-inverse cut, recycled blocks, renormalisation and
unit-norm scaling) and the same discrete choices.  The discrete choices --
the signs of the QR diagonal, the sign rule on the singular triples and the
pseudo-inverse mask -- are taken from the forward values and held constant,
as they are piecewise constant functions of the input.

It also writes the nearest-neighbour bond energy <op>_H + <op>_V of the
two-site reduced density matrices (iPEPS section, observables) in PyTorch,
for the gradient of the energy's direct dependence on (C, T, A).

Its pins are independent of autograd: central finite differences of the
NumPy move and of the NumPy bond values of :mod:`oracle.ctmrg` along random
directions (``tests/``), and the forward values of both implementations
agree to rounding.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import torch

from .ctmrg import sign_fix_columns

__all__ = ["move_torch", "move_vjp", "si_projectors_torch", "renormalize_torch",
           "enlarged_corners_torch", "double_layer_torch", "energy_torch", "energy_vjp"]

_f64 = torch.float64


def double_layer_torch(A: torch.Tensor) -> torch.Tensor:
    """a[(uU),(lL),(dD),(rR)] = sum_s A[s,u,l,d,r] A[s,U,L,D,R] (iPEPS section)."""
    D = A.shape[1]
    a = torch.einsum("sijkl,sIJKL->iIjJkKlL", A, A)
    return a.reshape(D * D, D * D, D * D, D * D)


def enlarged_corners_torch(C: Sequence[torch.Tensor], T: Sequence[torch.Tensor],
                           a: torch.Tensor) -> List[torch.Tensor]:
    """The four enlarged corners (Fig. 1; eq. rho_M_diag), row = in pair."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    N = C1.shape[0] * a.shape[0]
    Ct1 = torch.einsum("tla,ab,bug,uldr->tdgr", T4, C1, T1, a)
    Ct2 = torch.einsum("bug,gh,hre,uldr->bled", T1, C2, T2, a)
    Ct3 = torch.einsum("hre,ez,zdn,uldr->hunl", T2, C3, T3, a)
    Ct4 = torch.einsum("zdn,nt,tla,uldr->zrau", T3, C4, T4, a)
    return [c.reshape(N, N) for c in (Ct1, Ct2, Ct3, Ct4)]


def _qr_pos(W: torch.Tensor) -> torch.Tensor:
    """Thin QR with R_ii >= 0; the diagonal signs are held constant."""
    q, r = torch.linalg.qr(W, mode="reduced")
    sg = torch.sign(torch.diagonal(r)).detach()
    sg[sg == 0] = 1.0
    return q * sg


def _pinv_sqrt(s: torch.Tensor, eps: float) -> torch.Tensor:
    """s^-1/2 with s_i <= eps * s_1 mapped to 0 (mask held constant)."""
    sd = s.detach()
    keep = sd > eps * sd[0] if sd.numel() and sd[0] > 0 else torch.zeros_like(sd, dtype=bool)
    out = torch.zeros_like(s)
    out[keep] = s[keep] ** -0.5
    return out


def si_projectors_torch(Ct, b: int, X: torch.Tensor, Yt: torch.Tensor, chi: int, n_si: int,
                        eps: float):
    """Stabilised SI projectors of bond b (QR-based projector section, steps
    1-3; eqs. xy_iter, rho_hat_diag, projectors_diag, xy_recycle)."""
    m = lambda i: Ct[i % 4]                                  # noqa: E731
    M = lambda W: m(b - 1) @ (m(b) @ (m(b + 1) @ (m(b + 2) @ W)))           # noqa: E731
    Mt = lambda W: m(b + 2).T @ (m(b + 1).T @ (m(b).T @ (m(b - 1).T @ W)))  # noqa: E731
    for _ in range(n_si):
        X = _qr_pos(Mt(_qr_pos(M(X))))
        Yt = _qr_pos(M(_qr_pos(Mt(Yt))))
    A = m(b + 1) @ (m(b + 2) @ X)
    Bt = m(b).T @ (m(b - 1).T @ Yt)
    rho = Bt.T @ A
    u, s, vt = torch.linalg.svd(rho)
    v = vt.T
    sg = torch.from_numpy(sign_fix_columns((Yt @ u).detach().numpy()))
    u = u * sg
    v = v * sg
    keep = min(chi, s.numel())
    sinv = _pinv_sqrt(s[:keep], eps)
    Pl = (A @ v[:, :keep]) * sinv
    Prt = (Bt @ u[:, :keep]) * sinv
    return Pl, Prt, s, X @ v, Yt @ u


def renormalize_torch(Ct, T, a, Pl, Prt):
    """C_i' = P_r Ct_i P_l and T_j' = P_r (T_j a) P_l, each scaled to unit
    Frobenius norm (Fig. 1); same contraction as :func:`oracle.ctmrg.renormalize`."""
    x, D2 = T[0].shape[0], a.shape[0]
    T1, T2, T3, T4 = T
    C = [Prt[(i - 1) % 4].T @ Ct[i] @ Pl[i] for i in range(4)]
    r = lambda P: P.reshape(x, D2, P.shape[1])   # noqa: E731
    z = torch.einsum("bug,gry->buyr", T1, r(Pl[0]))
    z = torch.einsum("buyr,uldr->blyd", z, a)
    Tn = [torch.einsum("blx,blyd->xdy", r(Prt[0]), z)]
    z = torch.einsum("hre,edy->hyrd", T2, r(Pl[1]))
    z = torch.einsum("hyrd,uldr->huyl", z, a)
    Tn.append(torch.einsum("hux,huyl->xly", r(Prt[1]), z))
    z = torch.einsum("zdn,nly->zydl", T3, r(Pl[2]))
    z = torch.einsum("zydl,uldr->zryu", z, a)
    Tn.append(torch.einsum("zrx,zryu->xuy", r(Prt[2]), z))
    z = torch.einsum("tla,auy->tylu", T4, r(Pl[3]))
    z = torch.einsum("tylu,uldr->tdyr", z, a)
    Tn.append(torch.einsum("tdx,tdyr->xry", r(Prt[3]), z))
    C = [c / torch.linalg.norm(c) for c in C]
    Tn = [t / torch.linalg.norm(t) for t in Tn]
    return C, Tn


def move_torch(C, T, X, Yt, A, chi: int, n_si: int = 2, eps: float = 1e-12):
    """One SI move at chi_env == chi from the site tensor A (iPEPS section
    double layer, then Fig. 1).  Returns (C', T', X', Y^T')."""
    a = double_layer_torch(A)
    Ct = enlarged_corners_torch(C, T, a)
    Pl, Prt, Xn, Ytn = [], [], [], []
    for b in range(4):
        pl, prt, _, xn, ytn = si_projectors_torch(Ct, b, X[b], Yt[b], chi, n_si, eps)
        Pl.append(pl)
        Prt.append(prt)
        Xn.append(xn)
        Ytn.append(ytn)
    Cn, Tn = renormalize_torch(Ct, T, a, Pl, Prt)
    return Cn, Tn, Xn, Ytn


def move_vjp(C, T, X, Yt, A, bars, chi: int, n_si: int = 2, eps: float = 1e-12):
    """Vector-Jacobian product of one SI move.

    ``C, T, X, Yt`` are lists of four NumPy arrays, ``A`` the site tensor;
    ``bars`` = (C_bar, T_bar, X_bar, Yt_bar), cotangents of the four outputs.
    Returns (C_in_bar, T_in_bar, X_in_bar, Yt_in_bar, A_bar) as NumPy arrays.
    """
    leaf = lambda v: torch.tensor(np.asarray(v), dtype=_f64, requires_grad=True)  # noqa: E731
    Cl = [leaf(c) for c in C]
    Tl = [leaf(t) for t in T]
    Xl = [leaf(x) for x in X]
    Yl = [leaf(y) for y in Yt]
    Al = leaf(A)
    out = move_torch(Cl, Tl, Xl, Yl, Al, chi, n_si, eps)
    total = 0.0
    for group, gbar in zip(out, bars):
        for o, w in zip(group, gbar):
            total = total + (o * torch.as_tensor(np.asarray(w), dtype=_f64)).sum()
    grads = torch.autograd.grad(total, Cl + Tl + Xl + Yl + [Al], allow_unused=True)
    g = [np.zeros(v.shape) if gr is None else gr.numpy() for v, gr in
         zip(Cl + Tl + Xl + Yl + [Al], grads)]
    return g[0:4], g[4:8], g[8:12], g[12:16], g[16]


def _double_layer_open_torch(A):
    """a_open[s, t, (uU), (lL), (dD), (rR)] = A[s,u,l,d,r] A[t,U,L,D,R]."""
    d, D = A.shape[0], A.shape[1]
    a = torch.einsum("sijkl,tIJKL->stiIjJkKlL", A, A)
    return a.reshape(d, d, D * D, D * D, D * D, D * D)


def _two_site_h_torch(C, T, x1, x2):
    """Horizontal pair (site 1 left of site 2), as :func:`oracle.ctmrg._two_site_h`."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    left = torch.einsum("ab,kla,jk->blj", C1, T4, C4)
    y1 = torch.einsum("blj,bug->gulj", left, T1)
    y2 = torch.einsum("gulj,ABuldm->ABgdmj", y1, x1)
    y3 = torch.einsum("ABgdmj,idj->ABgmi", y2, T3)
    right = torch.einsum("hc,cwe,ef->hwf", C2, T2, C3)
    w1 = torch.einsum("gvh,hwf->gvwf", T1, right)
    w2 = torch.einsum("gvwf,EFvmyw->EFgmyf", w1, x2)
    w3 = torch.einsum("EFgmyf,fyi->EFgmi", w2, T3)
    return torch.einsum("ABgmi,EFgmi->ABEF", y3, w3)


def _two_site_v_torch(C, T, x1, x2):
    """Vertical pair (site 1 above site 2), as :func:`oracle.ctmrg._two_site_v`."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    top = torch.einsum("ab,bug,gh->auh", C1, T1, C2)
    p1 = torch.einsum("nla,auh->nluh", T4, top)
    p2 = torch.einsum("nluh,ABulxr->ABnxrh", p1, x1)
    p3 = torch.einsum("ABnxrh,hrc->ABnxc", p2, T2)
    bot = torch.einsum("ij,jwk,km->iwm", C3, T3, C4)
    q1 = torch.einsum("csi,iwm->cswm", T2, bot)
    q2 = torch.einsum("cswm,EFxpws->EFcxpm", q1, x2)
    q3 = torch.einsum("EFcxpm,mpn->EFcxn", q2, T4)
    return torch.einsum("ABnxc,EFcxn->ABEF", p3, q3)


_CORNER_SPECS = ("tla,ab,bug,...uldr->...tdgr", "bug,gh,hre,...uldr->...bled",
                 "hre,ez,zdn,...uldr->...hunl", "zdn,nt,tla,...uldr->...zrau")


def _two_site_diag_torch(C, T, ao, anti: bool):
    """Diagonal pair of the 2x2 plaquette Tr(Ct1 Ct2 Ct3 Ct4), as
    :func:`oracle.ctmrg._two_site_diag`: site 1 top-left and site 2
    bottom-right (``anti``: top-right and bottom-left); the two other corners
    hold the closed double layer."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    ops = ((T4, C1, T1), (T1, C2, T2), (T2, C3, T3), (T3, C4, T4))
    a = torch.einsum("ss...->...", ao)
    o = 1 if anti else 0
    Ct = []
    for i in range(4):
        x = ao if i in (o, o + 2) else a
        c = torch.einsum(_CORNER_SPECS[i], *ops[i], x)
        N = C1.shape[0] * x.shape[-1]
        Ct.append(c.reshape(c.shape[:-4] + (N, N)))
    c0, c1, c2, c3 = (Ct[(o + j) % 4] for j in range(4))
    return torch.einsum("ABij,jk,EFkl,li->ABEF", c0, c1, c2, c3)


def energy_torch(C, T, A, op, bonds: str = "hv"):
    """Sum over ``bonds`` (``h``, ``v``, ``d`` for the diagonal, ``a`` for the
    anti-diagonal) of <op> with op[(t1 t2), (s1 s2)] (bra, ket), from the
    two-site reduced density matrices (iPEPS section, observables; the
    diagonal bonds of the triangular-lattice section), as
    :func:`oracle.ctmrg.bond_value` for each bond."""
    d = A.shape[0]
    ao = _double_layer_open_torch(A)
    pairs = {"h": lambda: _two_site_h_torch(C, T, ao, ao),
             "v": lambda: _two_site_v_torch(C, T, ao, ao),
             "d": lambda: _two_site_diag_torch(C, T, ao, False),
             "a": lambda: _two_site_diag_torch(C, T, ao, True)}
    out = 0.0
    for bond in bonds:
        E = pairs[bond]()
        rho = E.permute(0, 2, 1, 3).reshape(d * d, d * d)
        rho = rho / torch.trace(rho)
        out = out + torch.trace(op @ rho)
    return out


def energy_vjp(C, T, A, op, bonds: str = "hv"):
    """(e, C_bar, T_bar, A_bar) for e = the sum of <op> over ``bonds`` (see
    :func:`energy_torch`) at environment (C, T)."""
    leaf = lambda v: torch.tensor(np.asarray(v), dtype=_f64, requires_grad=True)  # noqa: E731
    Cl = [leaf(c) for c in C]
    Tl = [leaf(t) for t in T]
    Al = leaf(A)
    e = energy_torch(Cl, Tl, Al, torch.as_tensor(np.asarray(op), dtype=_f64), bonds)
    g = torch.autograd.grad(e, Cl + Tl + [Al])
    return float(e.detach()), [x.numpy() for x in g[:4]], [x.numpy() for x in g[4:8]], g[8].numpy()

