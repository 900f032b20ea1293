"""Host-side helpers of the package (no GPU): the spiral bond operators.

The single-site spiral ansatz of the triangular lattice (each site rotated
by its lattice vector times the ordering angles) turns the uniform
all-up product state into the classical 120-degree state, whose energy per
bond is cos(120 deg)/4 = -1/8 for the spin-1/2 Heisenberg coupling S.S, so
-3/8 per site over the three bonds h, v and d; evaluated through the
oracle's bond values on an exact product-state environment.
"""
import numpy as np

import oracle as O
import paper_2607_15158_amd as P
import synth as S


def test_spiral_operators_give_the_classical_120_degree_energy():
    th = 2 * np.pi / 3
    ops = P.spiral_bond_operators(S.heisenberg_bond(), {"h": th, "v": th, "d": 2 * th})
    up = np.array([1.0, 0.0])
    A = np.einsum("s,u,l,d,r->suldr", up, [1.0], [1.0], [1.0], [1.0])   # D = 1
    a, e = O.double_layer(A), S.trace_boundary(1)
    env, _ = O.run_ctmrg(a, e, 1, proj="svd", max_moves=2)
    names = {"h": "h", "v": "v", "d": "d"}
    per_bond = {b: O.bond_value(env, A, op, names[b]) for b, op in ops.items()}
    for b, val in per_bond.items():
        assert abs(val - (-1.0 / 8.0)) <= 1e-14, (b, val)
    # without the rotation the same state is the ferromagnet: +1/4 per bond
    assert abs(O.bond_value(env, A, S.heisenberg_bond(), "h") - 0.25) <= 1e-14
    # the operators stay real and symmetric under exchange of bra and ket
    for op in ops.values():
        assert np.allclose(op, op.T, atol=1e-15)


def test_bond_mask_letters():
    assert P.bond_mask("hvd") == 7 and P.bond_mask("a") == 8
    try:
        P.bond_mask("x")
    except ValueError:
        pass
    else:
        raise AssertionError("unknown bond letter accepted")
