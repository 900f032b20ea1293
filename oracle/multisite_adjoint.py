"""Reverse-mode reference for the unit-cell iteration -- TEST INFRASTRUCTURE ONLY.

The SI iteration of an Lx x Ly cell (:mod:`oracle.multisite`: left, top,
right and bottom moves, each column by column with the per-cut SI
projectors of the larger unit-cell passage of the End Matter) and the energy
per site of the cell, written a second time in PyTorch on the CPU in
float64, so that ``torch.autograd`` gives their vector-Jacobian products:

    (environments, blocks, site tensors) -> (environments', blocks')
    (environments, site tensors)         -> energy per site

with the conventions, the order of operations and the discrete choices of
the NumPy oracle (the QR diagonal signs, the sign rule and the
pseudo-inverse mask are taken from the forward values and held constant).
Only environments of full dimension chi are handled (every cut an SI cut).

Its pins are independent of autograd: the forward values equal those of
:mod:`oracle.multisite`, and its gradients match central finite differences
of the NumPy oracle along random directions (``tests/``).
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import torch

from .adjoint import _double_layer_open_torch, double_layer_torch, si_projectors_torch

__all__ = ["cell_iteration_torch", "cell_energy_torch", "cell_move_vjp", "cell_energy_vjp"]

_f64 = torch.float64

_CORNERS = ("tla,ab,bug,uldr->tdgr", "bug,gh,hre,uldr->bled",
            "hre,ez,zdn,uldr->hunl", "zdn,nt,tla,uldr->zrau")
_CORNERS_OPEN = ("tla,ab,bug,STuldr->STtdgr", "bug,gh,hre,STuldr->STbled",
                 "hre,ez,zdn,STuldr->SThunl", "zdn,nt,tla,STuldr->STzrau")


def _corner(C, T, x, i):
    """Enlarged corner i of one site with site tensor x (rank 4, or rank 6
    open [s, t, u, l, d, r]): rows its in pair, columns its out pair."""
    ops = ((T[3], C[0], T[0]), (T[0], C[1], T[1]), (T[1], C[2], T[2]), (T[2], C[3], T[3]))[i]
    spec = (_CORNERS if x.dim() == 4 else _CORNERS_OPEN)[i]
    c = torch.einsum(spec, *ops, x)
    sh = c.shape
    return c.reshape(sh[:-4] + (sh[-4] * sh[-3], sh[-2] * sh[-1]))


def _turn(env, a, Lx, Ly):
    """The cell turned by 90 degrees (top edge to the left one): site (x, y)
    goes to (y, Lx-1-x), slot i+1 of every environment to slot i, the legs of
    every network tensor turn with it."""
    env2, a2 = {}, {}
    for (x, y), (C, T) in env.items():
        s = (y, Lx - 1 - x)
        env2[s] = ([C[(i + 1) % 4] for i in range(4)], [T[(i + 1) % 4] for i in range(4)])
        a2[s] = a[(x, y)].permute(3, 0, 1, 2)
    return env2, a2, Ly, Lx


def _left_move(env, a, Lx, Ly, chi, iso, n_si, eps):
    env = dict(env)
    iso = dict(iso)
    at = lambda x, y: (x % Lx, y % Ly)  # noqa: E731
    for x in range(Lx):
        Pl, Prt = {}, {}
        for y in range(Ly):
            sites = (at(x, y), at(x + 1, y), at(x + 1, y + 1), at(x, y + 1))
            Ct = [_corner(*env[s], a[s], i) for i, s in enumerate(sites)]
            X, Yt = iso[(x, y)]
            pl, prt, _, xn, ytn = si_projectors_torch(Ct, 3, X, Yt, chi, n_si, eps)
            Pl[y], Prt[y] = pl, prt
            iso[(x, y)] = (xn, ytn)
        new = {}
        for y in range(Ly):
            s = at(x, y)
            C, T = env[s]
            xc, D2 = C[0].shape[0], a[s].shape[0]
            r = lambda P: P.reshape(xc, D2, P.shape[1])   # noqa: E731
            C1n = torch.einsum("aun,ab,bug->ng", r(Prt[(y - 1) % Ly]), C[0], T[0])
            Tt4 = torch.einsum("tla,uldr->tdrau", T[3], a[s])
            T4n = torch.einsum("tdn,tdrau,aum->nrm", r(Prt[y]), Tt4, r(Pl[(y - 1) % Ly]))
            C4n = torch.einsum("zdn,nt,tdm->zm", T[2], C[3], r(Pl[y]))
            new[at(x + 1, y)] = (C1n, T4n, C4n)
        for s, (C1n, T4n, C4n) in new.items():
            C, T = list(env[s][0]), list(env[s][1])
            C[0] = C1n / torch.linalg.norm(C1n)
            T[3] = T4n / torch.linalg.norm(T4n)
            C[3] = C4n / torch.linalg.norm(C4n)
            env[s] = (C, T)
    return env, iso


def cell_iteration_torch(env: Dict, iso: Dict, A: Dict, Lx: int, Ly: int, chi: int,
                         n_si: int = 2, eps: float = 1e-12):
    """One SI iteration (left, top, right, bottom moves) of the cell:
    ``env[(x, y)] = (C list, T list)``, ``iso[d][(x', y')] = (X, Yt)`` in the
    turned cell's coordinates, ``A[(x, y)]`` site tensors.  Returns the new
    (env, iso)."""
    a = {s: double_layer_torch(t) for s, t in A.items()}
    iso = {d: dict(iso[d]) for d in range(4)}
    for d in range(4):
        e, aa, lx, ly = env, a, Lx, Ly
        for _ in range(d):
            e, aa, lx, ly = _turn(e, aa, lx, ly)
        e, iso[d] = _left_move(e, aa, lx, ly, chi, iso[d], n_si, eps)
        for _ in range((4 - d) % 4):
            e, aa, lx, ly = _turn(e, aa, lx, ly)
        env = e
    return env, iso


def _pair_h(eL, eR, x1, x2):
    C1, _, _, C4 = eL[0]
    T1, _, T3, T4 = eL[1]
    _, C2, C3, _ = eR[0]
    T1r, T2, T3r, _ = eR[1]
    left = torch.einsum("ab,kla,jk->blj", C1, T4, C4)
    y1 = torch.einsum("blj,bug->gulj", left, T1)
    y2 = torch.einsum("gulj,STuldm->STgdmj", y1, x1)
    y3 = torch.einsum("STgdmj,idj->STgmi", y2, T3)
    right = torch.einsum("hc,cwe,ef->hwf", C2, T2, C3)
    w1 = torch.einsum("gvh,hwf->gvwf", T1r, right)
    w2 = torch.einsum("gvwf,EFvmyw->EFgmyf", w1, x2)
    w3 = torch.einsum("EFgmyf,fyi->EFgmi", w2, T3r)
    return torch.einsum("STgmi,EFgmi->STEF", y3, w3)


def _pair_v(eT, eB, x1, x2):
    C1, C2, _, _ = eT[0]
    T1, T2, _, T4 = eT[1]
    _, _, C3, C4 = eB[0]
    _, T2b, T3, T4b = eB[1]
    top = torch.einsum("ab,bug,gh->auh", C1, T1, C2)
    p1 = torch.einsum("nla,auh->nluh", T4, top)
    p2 = torch.einsum("nluh,STulxr->STnxrh", p1, x1)
    p3 = torch.einsum("STnxrh,hrc->STnxc", p2, T2)
    bot = torch.einsum("ij,jwk,km->iwm", C3, T3, C4)
    q1 = torch.einsum("csi,iwm->cswm", T2b, bot)
    q2 = torch.einsum("cswm,EFxpws->EFcxpm", q1, x2)
    q3 = torch.einsum("EFcxpm,mpn->EFcxn", q2, T4b)
    return torch.einsum("STnxc,EFcxn->STEF", p3, q3)


def _pair_d(envs, xs):
    """Diagonal pair of a 2x2 plaquette: ``envs``, ``xs`` of the sites
    top-left, top-right, bottom-right, bottom-left; xs[0] and xs[2] open."""
    Ct = [_corner(*envs[i], xs[i], i) for i in range(4)]
    return torch.einsum("ABij,jk,EFkl,li->ABEF", *Ct)


def cell_energy_torch(env: Dict, A: Dict, Lx: int, Ly: int, ops: Dict) -> torch.Tensor:
    """(1 / (Lx Ly)) sum over the sites and the bonds in ``ops`` ('h', 'v',
    'd') of <op> from the two-site reduced density matrices, as
    :func:`oracle.multisite.cell_energy`."""
    at = lambda x, y: (x % Lx, y % Ly)  # noqa: E731
    a = {s: double_layer_torch(t) for s, t in A.items()}
    ao = {s: _double_layer_open_torch(t) for s, t in A.items()}
    d = next(iter(A.values())).shape[0]
    total = 0.0
    for x in range(Lx):
        for y in range(Ly):
            s = at(x, y)
            for bond, op in ops.items():
                if bond == "h":
                    E = _pair_h(env[s], env[at(x + 1, y)], ao[s], ao[at(x + 1, y)])
                elif bond == "v":
                    E = _pair_v(env[s], env[at(x, y + 1)], ao[s], ao[at(x, y + 1)])
                else:
                    ss = (s, at(x + 1, y), at(x + 1, y + 1), at(x, y + 1))
                    E = _pair_d([env[q] for q in ss], [ao[ss[0]], a[ss[1]], ao[ss[2]], a[ss[3]]])
                rho = E.permute(0, 2, 1, 3).reshape(d * d, d * d)
                rho = rho / torch.trace(rho)
                total = total + torch.trace(torch.as_tensor(op, dtype=_f64) @ rho)
    return total / (Lx * Ly)


def _leafs(env, iso, A):
    leaf = lambda v: torch.tensor(np.asarray(v), dtype=_f64, requires_grad=True)  # noqa: E731
    env_t = {s: ([leaf(c) for c in C], [leaf(t) for t in T]) for s, (C, T) in env.items()}
    iso_t = None if iso is None else {d: {k: (leaf(X), leaf(Y)) for k, (X, Y) in iso[d].items()}
                                      for d in iso}
    A_t = {s: leaf(t) for s, t in A.items()}
    return env_t, iso_t, A_t


def cell_move_vjp(env, iso, A, Lx, Ly, chi, bars: Tuple, n_si: int = 2, eps: float = 1e-12):
    """Vector-Jacobian product of one SI iteration with NumPy inputs (env as
    {site: (C list, T list)}, iso as {d: {cut: (X, Yt)}}, A as {site: A})
    and ``bars`` = (env_bar, iso_bar) shaped like the outputs.  Returns
    (env_in_bar, iso_in_bar, A_bar) as NumPy arrays."""
    env_t, iso_t, A_t = _leafs(env, iso, A)
    env_o, iso_o = cell_iteration_torch(env_t, iso_t, A_t, Lx, Ly, chi, n_si, eps)
    env_b, iso_b = bars
    total = 0.0
    for s, (C, T) in env_o.items():
        for o, w in zip(C + T, env_b[s][0] + env_b[s][1]):
            total = total + (o * torch.as_tensor(np.asarray(w), dtype=_f64)).sum()
    for d in range(4):
        for k, (X, Y) in iso_o[d].items():
            total = total + (X * torch.as_tensor(iso_b[d][k][0])).sum()
            total = total + (Y * torch.as_tensor(iso_b[d][k][1])).sum()
    leaves = []
    for s in env_t:
        leaves += env_t[s][0] + env_t[s][1]
    for d in range(4):
        for k in iso_t[d]:
            leaves += list(iso_t[d][k])
    leaves += list(A_t.values())
    grads = torch.autograd.grad(total, leaves, allow_unused=True)
    g = iter([np.zeros(v.shape) if gr is None else gr.numpy() for v, gr in zip(leaves, grads)])
    env_g = {s: ([next(g) for _ in range(4)], [next(g) for _ in range(4)]) for s in env_t}
    iso_g = {d: {k: (next(g), next(g)) for k in iso_t[d]} for d in range(4)}
    A_g = {s: next(g) for s in A_t}
    return env_g, iso_g, A_g


def cell_energy_vjp(env, A, Lx, Ly, ops):
    """(e, env_bar, A_bar) of :func:`cell_energy_torch` with NumPy inputs."""
    env_t, _, A_t = _leafs(env, None, A)
    e = cell_energy_torch(env_t, A_t, Lx, Ly, ops)
    leaves = []
    for s in env_t:
        leaves += env_t[s][0] + env_t[s][1]
    leaves += list(A_t.values())
    grads = torch.autograd.grad(e, leaves)
    g = iter([x.numpy() for x in grads])
    env_g = {s: ([next(g) for _ in range(4)], [next(g) for _ in range(4)]) for s in env_t}
    A_g = {s: next(g) for s in A_t}
    return float(e.detach()), env_g, A_g
