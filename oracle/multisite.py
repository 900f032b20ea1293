"""Plain FP64 NumPy CTMRG for an Lx x Ly unit cell of site tensors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The larger unit-cell passage of the paper's End Matter: the environment is
renormalised direction by direction and, within a direction, column by
column across the cell; every cut between two rows of a column has its own
projectors, built as in the single-site case from the four enlarged corners
of the 2x2 cluster at that cut, with its own subspace-iteration blocks X, Y.
A warm-up with randomized SVD projectors (fresh start blocks every move)
prepares the environment before the subspace iteration starts from the
Gaussian start blocks.

Reading used (each choice is also listed in the design notes):

* Site (x, y) is column x (to the right) and row y (downwards), periodic
  in both.  Every site carries its own environment, the tensors that
  surround it with the single-site conventions: C1[x,y] above-left of the
  site, T1[x,y] above it, C2 above-right, T2 right, C3 below-right, T3 below,
  C4 below-left, T4 left, each ordered (in, inner, out) clockwise as in
  ``oracle.ctmrg``.
* The 2x2 cluster (x, y) holds the sites (x, y), (x+1, y), (x+1, y+1),
  (x, y+1); its enlarged corners are those of ``oracle.ctmrg`` built from
  each site's own environment: Ct1 of (x, y), Ct2 of (x+1, y), Ct3 of
  (x+1, y+1), Ct4 of (x, y+1).
* A left move takes x = 0, 1, ..., Lx-1 in turn.  For column x it builds
  the projectors of the left cut of every cluster (x, y) (bond b = 3 of the
  single-site move: M = Ct3 Ct4 Ct1 Ct2, P_l on the out pair of Ct4, P_r on
  the in pair of Ct1), then moves the left environment of column x one
  column to the right:
      C1[x+1,y] = P_r(x, y-1) (C1 T1)[x,y],
      T4[x+1,y] = P_r(x, y) (T4 a)[x,y] P_l(x, y-1),
      C4[x+1,y] = (T3 C4)[x,y] P_l(x, y),
  each normalised to unit Frobenius norm.  The pairs of legs cut by a
  projector are fused chi-major, as everywhere in the oracle.
* One iteration is a left, top, right and bottom move; the top, right and
  bottom moves are the left move of the cell turned by 90, 180 and 270
  degrees (the turn maps the top edge onto the left one).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import ctmrg as _c

__all__ = ["Cell", "cell_initial_env", "turn_cell", "left_move", "ctm_iteration", "run_cell",
           "cell_corner_spectra", "cell_bond_value", "cell_energy", "cell_kappa"]

_EIN = dict(optimize=True)

Site = Tuple[int, int]


@dataclass
class Cell:
    """Site tensors and environments of an Lx x Ly unit cell.

    ``a[(x, y)]`` is the network tensor of site (x, y) (the double layer, or
    the classical tensor), ``A[(x, y)]`` the site tensor itself (None for a
    classical network), ``env[(x, y)]`` its environment."""

    Lx: int
    Ly: int
    a: Dict[Site, np.ndarray]
    A: Optional[Dict[Site, np.ndarray]]
    env: Dict[Site, _c.Env]

    def at(self, x: int, y: int) -> Site:
        return (x % self.Lx, y % self.Ly)

    def copy(self) -> "Cell":
        return Cell(self.Lx, self.Ly, dict(self.a), None if self.A is None else dict(self.A),
                    {s: e.copy() for s, e in self.env.items()})


# --------------------------------------------------------------------------
# initial environment: the outer legs of the neighbouring sites closed
# --------------------------------------------------------------------------
def cell_initial_env(a: Dict[Site, np.ndarray], Lx: int, Ly: int, e,
                     A: Optional[Dict[Site, np.ndarray]] = None) -> Cell:
    """Every environment tensor of site (x, y) from the neighbour in its
    direction with its outer legs closed by ``e`` (the single-site initial
    environment when all sites are equal); ``e`` is one vector, or a
    function e(site, leg) with leg one of 'u', 'l', 'd', 'r' giving the
    vector that closes that leg of that site."""
    vec = e if callable(e) else (lambda site, leg: e)
    env = {}
    for x in range(Lx):
        for y in range(Ly):
            def n(dx, dy):
                s = ((x + dx) % Lx, (y + dy) % Ly)
                return a[s], (lambda leg: vec(s, leg))
            t, v = n(-1, -1)
            C1 = np.einsum("uldr,u,l->dr", t, v("u"), v("l"))
            t, v = n(0, -1)
            T1 = np.einsum("uldr,u->ldr", t, v("u"))
            t, v = n(1, -1)
            C2 = np.einsum("uldr,u,r->ld", t, v("u"), v("r"))
            t, v = n(1, 0)
            T2 = np.einsum("uldr,r->uld", t, v("r"))
            t, v = n(1, 1)
            C3 = np.einsum("uldr,d,r->ul", t, v("d"), v("r"))
            t, v = n(0, 1)
            T3 = np.einsum("uldr,d->rul", t, v("d"))
            t, v = n(-1, 1)
            C4 = np.einsum("uldr,l,d->ru", t, v("l"), v("d"))
            t, v = n(-1, 0)
            T4 = np.einsum("uldr,l->dru", t, v("l"))
            env[(x, y)] = _c.normalize_env(_c.Env([C1, C2, C3, C4], [T1, T2, T3, T4]))
    return Cell(Lx, Ly, dict(a), None if A is None else dict(A), env)


# --------------------------------------------------------------------------
# the 90-degree turn (top edge -> left edge)
# --------------------------------------------------------------------------
def _turn_a(a: np.ndarray) -> np.ndarray:
    """a'[u', l', d', r'] = a[u = l', l = d', d = r', r = u']."""
    return np.ascontiguousarray(a.transpose(3, 0, 1, 2))


def _turn_A(A: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(A.transpose(0, 4, 1, 2, 3))


def turn_cell(cell: Cell) -> Cell:
    """The cell turned by 90 degrees so that its top edge becomes the left
    one: site (x, y) moves to (y, Lx-1-x), the legs of every site tensor
    turn with it, and the environment tensor in slot i+1 (corners and
    edges) becomes the one in slot i."""
    Lx, Ly = cell.Lx, cell.Ly
    a, A, env = {}, ({} if cell.A is not None else None), {}
    for (x, y), t in cell.a.items():
        s = (y, Lx - 1 - x)
        a[s] = _turn_a(t)
        if A is not None:
            A[s] = _turn_A(cell.A[(x, y)])
        e = cell.env[(x, y)]
        env[s] = _c.Env([e.C[(i + 1) % 4].copy() for i in range(4)],
                        [e.T[(i + 1) % 4].copy() for i in range(4)])
    return Cell(Ly, Lx, a, A, env)


def _turn_back(cell: Cell, times: int) -> Cell:
    for _ in range((4 - times) % 4):
        cell = turn_cell(cell)
    return cell


# --------------------------------------------------------------------------
# the left move, column by column
# --------------------------------------------------------------------------
def _corner(env: _c.Env, t: np.ndarray, i: int) -> np.ndarray:
    """Enlarged corner i of one site (the contraction of
    ``oracle.ctmrg.enlarged_corners``) with the site tensor t (rank 4, or an
    open double layer [s, t, u, l, d, r]); rows are its in pair and columns
    its out pair, whose sizes may differ while the environment grows (a move
    has renormalised some of the site's tensors but not yet the others)."""
    C1, C2, C3, C4 = env.C
    T1, T2, T3, T4 = env.T
    ops = ((T4, C1, T1), (T1, C2, T2), (T2, C3, T3), (T3, C4, T4))[i]
    c = np.einsum(_c._CORNER_SPECS[i], *ops, t, **_EIN)
    sh = c.shape
    return c.reshape(sh[:-4] + (sh[-4] * sh[-3], sh[-2] * sh[-1]))


def _cluster_corners(cell: Cell, x: int, y: int) -> List[np.ndarray]:
    sites = (cell.at(x, y), cell.at(x + 1, y), cell.at(x + 1, y + 1), cell.at(x, y + 1))
    return [_corner(cell.env[s], cell.a[s], i) for i, s in enumerate(sites)]


def _cut_projectors(Ct, chi: int, x_env: int, mode: str, X, Yt, n_si: int, eps: float,
                    stabilized: bool):
    """Projectors of the left cut (bond 3) of a cluster; returns
    (P_l, P_r^T, X', Yt', mode used)."""
    N = Ct[3].shape[1]
    if N <= chi:
        return np.eye(N), np.eye(N), X, Yt, "grow"
    if mode == "svd" or (mode == "si" and x_env != chi):
        pl, prt, _ = _c.svd_projectors(Ct, 3, chi, eps)
        return pl, prt, X, Yt, "svd"
    if mode == "rsvd":
        # X lives on the columns of R = Ct1 Ct2, Y^T on the rows of L = Ct3 Ct4
        # (sizes that can differ from the cut's while the environment grows)
        nx, ny = Ct[1].shape[1], Ct[2].shape[0]
        if min(nx, ny) < X.shape[1]:
            pl, prt, _ = _c.svd_projectors(Ct, 3, chi, eps)
            return pl, prt, X, Yt, "svd"
        # randomized SVD: power steps from the cut's start blocks, no recycling
        pl, prt, _, _, _ = _c.si_projectors(Ct, 3, X[:nx], Yt[:ny], chi, n_si, eps, stabilized)
        return pl, prt, X, Yt, "rsvd"
    pl, prt, _, xn, ytn = _c.si_projectors(Ct, 3, X, Yt, chi, n_si, eps, stabilized)
    return pl, prt, xn, ytn, "si"


def left_move(cell: Cell, chi: int, mode: str, iso: Optional[dict], n_si: int = 2,
              eps: float = 1e-12, stabilized: bool = True):
    """One left move of the cell (module docstring).  ``mode``: ``svd``
    (full-SVD projectors), ``rsvd`` (randomized SVD from the start blocks in
    ``iso``, which are left unchanged) or ``si`` (subspace iteration on the
    blocks in ``iso``, recycled).  ``iso[(x, y)] = (X, Yt)`` for the left cut
    of cluster (x, y).  Returns (new cell, new iso, modes used)."""
    cell = cell.copy()
    iso = None if iso is None else dict(iso)
    modes = []
    for x in range(cell.Lx):
        Pl, Prt = {}, {}
        for y in range(cell.Ly):
            Ct = _cluster_corners(cell, x, y)
            x_env = cell.env[cell.at(x, y)].chi
            X, Yt = (None, None) if iso is None else iso[(x, y)]
            Pl[y], Prt[y], X, Yt, m = _cut_projectors(Ct, chi, x_env, mode, X, Yt, n_si, eps,
                                                      stabilized)
            if iso is not None:
                iso[(x, y)] = (X, Yt)
            modes.append(m)
        new = {}
        for y in range(cell.Ly):
            s = cell.at(x, y)
            e, a = cell.env[s], cell.a[s]
            C1, T1, T3, C4, T4 = e.C[0], e.T[0], e.T[2], e.C[3], e.T[3]
            xc, D2 = e.chi, a.shape[0]
            up = Prt[(y - 1) % cell.Ly]
            dn = Pl[(y - 1) % cell.Ly]
            r = lambda P: P.reshape(xc, D2, P.shape[1])   # noqa: E731
            C1n = np.einsum("aun,ab,bug->ng", r(up), C1, T1, **_EIN)
            Tt4 = np.einsum("tla,uldr->tdrau", T4, a, **_EIN)
            T4n = np.einsum("tdn,tdrau,aum->nrm", r(Prt[y]), Tt4, r(dn), **_EIN)
            C4n = np.einsum("zdn,nt,tdm->zm", T3, C4, r(Pl[y]), **_EIN)
            new[cell.at(x + 1, y)] = (C1n, T4n, C4n)
        for s, (C1n, T4n, C4n) in new.items():
            e = cell.env[s]
            C = list(e.C)
            T = list(e.T)
            C[0] = C1n / np.linalg.norm(C1n)
            T[3] = T4n / np.linalg.norm(T4n)
            C[3] = C4n / np.linalg.norm(C4n)
            cell.env[s] = _c.Env(C, T)
    return cell, iso, modes


def ctm_iteration(cell: Cell, chi: int, mode: str, iso: Optional[dict], n_si: int = 2,
                  eps: float = 1e-12, stabilized: bool = True):
    """Left, top, right and bottom moves.  ``iso[d]`` holds the blocks of
    direction d (0 left, 1 top, 2 right, 3 bottom) in the turned cell's
    coordinates."""
    iso = None if iso is None else dict(iso)
    modes = []
    for d in range(4):
        turned = cell
        for _ in range(d):
            turned = turn_cell(turned)
        turned, blocks, m = left_move(turned, chi, mode, None if iso is None else iso[d], n_si,
                                      eps, stabilized)
        if iso is not None:
            iso[d] = blocks
        modes += m
        cell = _turn_back(turned, d)
    return cell, iso, modes


def cell_corner_spectra(cell: Cell, chi: int) -> np.ndarray:
    """Unit-norm, zero-padded corner spectra of every site, [site][corner][chi]."""
    return np.stack([_c.corner_spectra(cell.env[(x, y)], chi)
                     for x in range(cell.Lx) for y in range(cell.Ly)])


def run_cell(cell: Cell, chi: int, iso0: dict, warmup: int = 3, warm_mode: str = "rsvd",
             n_si: int = 2, eps: float = 1e-12, tol: float = 0.0, max_iter: int = 100,
             stabilized: bool = True):
    """Warm-up iterations (``rsvd``: randomized SVD projectors from the start
    blocks; ``svd``: full SVD) until the environment has dimension chi and at
    least ``warmup`` of them were made, then SI iterations from the start
    blocks ``iso0`` (per direction and cut) until delta < tol: the largest
    over all sites and corners of the l2 change of the unit-norm corner
    spectra between two iterations."""
    spec = cell_corner_spectra(cell, chi)
    hist = []
    n = 0
    while n < max_iter:
        full = all(e.chi == chi for e in cell.env.values())
        if n < warmup or not full:
            cell, _, modes = ctm_iteration(cell, chi, warm_mode, iso0, n_si, eps, stabilized)
            kind = "warmup"
        else:
            if not hist or hist[-1]["kind"] != "si":
                iso = {d: dict(iso0[d]) for d in range(4)}
            cell, iso, modes = ctm_iteration(cell, chi, "si", iso, n_si, eps, stabilized)
            kind = "si"
        new = cell_corner_spectra(cell, chi)
        delta = float(np.max(np.linalg.norm(new - spec, axis=2)))
        spec = new
        n += 1
        hist.append({"iter": n, "kind": kind, "delta": delta, "modes": sorted(set(modes))})
        if kind == "si" and delta < tol:
            break
    return cell, hist


# --------------------------------------------------------------------------
# observables of the cell
# --------------------------------------------------------------------------
def _pair_h(eL: _c.Env, eR: _c.Env, x1, x2) -> np.ndarray:
    """Horizontal pair, site 1 with environment eL on the left of site 2
    with environment eR (the column-by-column contraction of
    ``oracle.ctmrg._two_site_h`` with each side's own tensors)."""
    C1, _, _, C4 = eL.C
    T1, _, T3, T4 = eL.T
    _, C2, C3, _ = eR.C
    T1r, T2, T3r, _ = eR.T
    left = np.einsum("ab,kla,jk->blj", C1, T4, C4)
    y1 = np.einsum("blj,bug->gulj", left, T1)
    y2 = np.einsum("gulj,...uldm->...gdmj", y1, x1)
    y3 = np.einsum("...gdmj,idj->...gmi", y2, T3)
    right = np.einsum("hc,cwe,ef->hwf", C2, T2, C3)
    w1 = np.einsum("gvh,hwf->gvwf", T1r, right)
    w2 = np.einsum("gvwf,...vmyw->...gmyf", w1, x2)
    w3 = np.einsum("...gmyf,fyi->...gmi", w2, T3r)
    if x1.ndim == 4:
        return np.einsum("gmi,gmi->", y3, w3)
    return np.einsum("ABgmi,EFgmi->ABEF", y3, w3)


def _pair_v(eT: _c.Env, eB: _c.Env, x1, x2) -> np.ndarray:
    """Vertical pair, site 1 with environment eT above site 2 with eB."""
    C1, C2, _, _ = eT.C
    T1, T2, _, T4 = eT.T
    _, _, C3, C4 = eB.C
    _, T2b, T3, T4b = eB.T
    top = np.einsum("ab,bug,gh->auh", C1, T1, C2)
    p1 = np.einsum("nla,auh->nluh", T4, top)
    p2 = np.einsum("nluh,...ulxr->...nxrh", p1, x1)
    p3 = np.einsum("...nxrh,hrc->...nxc", p2, T2)
    bot = np.einsum("ij,jwk,km->iwm", C3, T3, C4)
    q1 = np.einsum("csi,iwm->cswm", T2b, bot)
    q2 = np.einsum("cswm,...xpws->...cxpm", q1, x2)
    q3 = np.einsum("...cxpm,mpn->...cxn", q2, T4b)
    if x1.ndim == 4:
        return np.einsum("nxc,cxn->", p3, q3)
    return np.einsum("ABnxc,EFcxn->ABEF", p3, q3)


def _pair_d(cell: Cell, x: int, y: int, x1, x2) -> np.ndarray:
    """Diagonal pair of cluster (x, y): site 1 = (x, y), site 2 = (x+1, y+1)
    on the 2x2 plaquette of the four enlarged corners, the other two sites
    with their closed double layers."""
    sites = [cell.at(x, y), cell.at(x + 1, y), cell.at(x + 1, y + 1), cell.at(x, y + 1)]
    Ct = []
    for i, s in enumerate(sites):
        t = x1 if i == 0 else x2 if i == 2 else cell.a[s]
        Ct.append(_corner(cell.env[s], t, i))
    if x1.ndim == 4:
        return np.einsum("ij,jk,kl,li->", *Ct, **_EIN)
    return np.einsum("ABij,jk,EFkl,li->ABEF", *Ct, **_EIN)


def cell_bond_value(cell: Cell, x: int, y: int, op: np.ndarray, direction: str) -> float:
    """<op> on the bond from site (x, y) to (x+1, y) (``h``), (x, y+1) (``v``)
    or (x+1, y+1) (``d``); op[(t1 t2), (s1 s2)] (bra, ket) as in
    ``oracle.ctmrg.bond_value``."""
    s1 = cell.at(x, y)
    s2 = cell.at(x + 1, y) if direction == "h" else cell.at(x, y + 1) if direction == "v" \
        else cell.at(x + 1, y + 1)
    o1 = _c.double_layer_open(cell.A[s1])
    o2 = _c.double_layer_open(cell.A[s2])
    if direction == "h":
        E = _pair_h(cell.env[s1], cell.env[s2], o1, o2)
    elif direction == "v":
        E = _pair_v(cell.env[s1], cell.env[s2], o1, o2)
    else:
        E = _pair_d(cell, x, y, o1, o2)
    d = cell.A[s1].shape[0]
    rho = E.transpose(0, 2, 1, 3).reshape(d * d, d * d)
    rho = rho / np.trace(rho)
    return float(np.trace(op @ rho))


def cell_classical_bond(cell: Cell, x: int, y: int, t1: np.ndarray, t2: np.ndarray,
                        direction: str) -> float:
    """Two rank-4 impurities t1 at site (x, y) and t2 at its neighbour in
    ``direction`` (as in ``cell_bond_value``), divided by the plain network."""
    s1 = cell.at(x, y)
    s2 = cell.at(x + 1, y) if direction == "h" else cell.at(x, y + 1) if direction == "v" \
        else cell.at(x + 1, y + 1)
    if direction == "h":
        f = lambda u, v: _pair_h(cell.env[s1], cell.env[s2], u, v)  # noqa: E731
    elif direction == "v":
        f = lambda u, v: _pair_v(cell.env[s1], cell.env[s2], u, v)  # noqa: E731
    else:
        f = lambda u, v: _pair_d(cell, x, y, u, v)  # noqa: E731
    return float(f(t1, t2) / f(cell.a[s1], cell.a[s2]))


def cell_energy(cell: Cell, ops: Dict[str, np.ndarray]) -> float:
    """Energy per site: (1 / (Lx Ly)) sum over the sites and over the bonds
    in ``ops`` ({direction: operator}) of <op>."""
    tot = 0.0
    for x in range(cell.Lx):
        for y in range(cell.Ly):
            for direction, op in ops.items():
                tot += cell_bond_value(cell, x, y, op, direction)
    return tot / (cell.Lx * cell.Ly)


def cell_kappa(cell: Cell, x: int, y: int) -> float:
    """Z11 Z00 / (Z10 Z01) from the environment of site (x, y) alone."""
    return _c.kappa(cell.env[cell.at(x, y)], cell.a[cell.at(x, y)])


def cell_onesite(cell: Cell, x: int, y: int, a_op: np.ndarray) -> float:
    """<O> = Z11(a_O) / Z11(a) at site (x, y)."""
    return _c.onesite_value(cell.env[cell.at(x, y)], cell.a[cell.at(x, y)], a_op)


__all__ += ["cell_onesite", "cell_classical_bond"]
