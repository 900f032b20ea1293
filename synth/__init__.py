"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no CTMRG arithmetic: it only draws tensors from seeded
NumPy generators and builds the fixed problem definitions (site tensors,
Boltzmann weights, boundary vectors, spin operators) that both sides take as
inputs.  Everything is float64 and C-ordered.

Conventions (shared by every caller):

* iPEPS site tensor ``A[s, u, l, d, r]`` (physical, up, left, down, right),
  real, shape ``(d, D, D, D, D)`` (iPEPS section, eq. ipeps_ansatz).
* classical site tensor ``a[u, l, d, r]`` of leg dimension ``Dl``.
* isometry blocks ``X`` and ``Y^T`` are ``N x k`` row-major.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "product_plus_noise_site",
    "gaussian_block",
    "ising_weights",
    "ising_site",
    "ising_impurity",
    "ising_boundary",
    "ising_peps_site",
    "heisenberg_bond",
    "pauli",
    "random_orthogonal",
    "trace_boundary",
]


def product_plus_noise_site(d: int, D: int, seed: int, noise: float = 0.1) -> np.ndarray:
    """Product state (1,0) on every leg plus ``noise * U[-1, 1]`` iid entries.

    ``A = delta_{s0} delta_{u0} delta_{l0} delta_{d0} delta_{r0} + noise * xi``
    with ``xi`` drawn in C order over ``(s, u, l, d, r)`` from
    ``numpy.random.default_rng(seed)``.  No renormalisation afterwards.
    """
    rng = np.random.default_rng(seed)
    A = noise * rng.uniform(-1.0, 1.0, size=(d, D, D, D, D))
    A[0, 0, 0, 0, 0] += 1.0
    return np.ascontiguousarray(A, dtype=np.float64)


def gaussian_block(N: int, k: int, seed: int) -> np.ndarray:
    """iid N(0,1) ``N x k`` block (the random start of a subspace iteration)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((N, k)), dtype=np.float64)


def ising_weights(beta: float) -> np.ndarray:
    """``W[s, x]`` with ``sum_x W[s,x] W[s',x] = exp(beta s s')``, s = +1 -> row 0."""
    c, s = np.sqrt(np.cosh(beta)), np.sqrt(np.sinh(beta))
    return np.array([[c, s], [c, -s]], dtype=np.float64)


def ising_site(beta: float) -> np.ndarray:
    """Rank-4 Boltzmann tensor ``a[u,l,d,r] = sum_s W[s,u] W[s,l] W[s,d] W[s,r]``."""
    W = ising_weights(beta)
    return np.ascontiguousarray(np.einsum("su,sl,sd,sr->uldr", W, W, W, W))


def ising_impurity(beta: float) -> np.ndarray:
    """Same as :func:`ising_site` with an extra factor of the spin ``s``."""
    W = ising_weights(beta)
    spin = np.array([1.0, -1.0])
    return np.ascontiguousarray(np.einsum("s,su,sl,sd,sr->uldr", spin, W, W, W, W))


def ising_boundary(beta: float) -> np.ndarray:
    """Fixed ``s = +1`` boundary vector ``W[+1, :]`` (breaks the Z2 symmetry)."""
    return ising_weights(beta)[0].copy()


def ising_peps_site(beta: float) -> np.ndarray:
    """d=2, D=2 iPEPS whose norm network is the classical Ising model at ``beta``.

    ``|psi> = sum_s exp(beta/2 sum_<ij> s_i s_j) |s>``: each ket and each bra
    carries half of every bond weight, so ``<psi|psi>`` is the Ising partition
    function, ``<sigma^z>`` its magnetisation and ``<sigma^z sigma^z>`` on a
    nearest-neighbour bond its bond correlation.
    """
    W = ising_weights(beta / 2.0)
    A = np.zeros((2, 2, 2, 2, 2))
    for s in range(2):
        A[s] = np.einsum("u,l,d,r->uldr", W[s], W[s], W[s], W[s])
    return np.ascontiguousarray(A)


def heisenberg_bond() -> np.ndarray:
    """``S_i . S_j`` for spin 1/2 in the basis |uu>,|ud>,|du>,|dd> (real)."""
    return 0.25 * np.array(
        [[1, 0, 0, 0], [0, -1, 2, 0], [0, 2, -1, 0], [0, 0, 0, 1]], dtype=np.float64
    )


def pauli(name: str) -> np.ndarray:
    """Real Pauli matrices x and z (y is imaginary and not needed here)."""
    if name == "x":
        return np.array([[0.0, 1.0], [1.0, 0.0]])
    if name == "z":
        return np.array([[1.0, 0.0], [0.0, -1.0]])
    if name == "i":
        return np.eye(2)
    raise ValueError(name)


def random_orthogonal(n: int, seed: int) -> np.ndarray:
    """Haar-ish random orthogonal ``n x n`` matrix (QR of a Gaussian)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def trace_boundary(D: int) -> np.ndarray:
    """``vec(I_D)``: closes a double-layer leg by tracing ket against bra."""
    return np.eye(D).reshape(D * D).copy()
