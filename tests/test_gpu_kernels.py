"""GPU parity of the building-block kernels through the C ABI.

GEMM against float64 NumPy products (N <= 160 runs the skinny kernel of the
enlarged-corner applications, wide N with long K the 256 x 144 double-
buffered tiles, also with odd leading dimensions, short K the general tiles; the split form of the skinny
kernel with ranges shorter and longer than a tile, mixed transposes, padded
rows, alpha and accumulation, and the cases where it hands over to the
plain tiles); Householder QR against the oracle's
QR convention (R_ii >= 0) and orthogonality; Jacobi SVD against NumPy's
singular values and the reconstruction.  Shapes span several tiles and
ragged tails.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2607_15158_amd as P  # noqa: E402
import synth as S  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("M,N,K,trans", [(5, 7, 3, 0), (130, 70, 33, 0), (130, 70, 33, 1),
                                         (257, 160, 300, 0), (300, 161, 257, 1),
                                         (1000, 144, 520, 0), (64, 1296, 1296, 0),
                                         (5184, 160, 5184, 0), (5184, 160, 5184, 1),
                                         (97, 159, 33, 1), (5600, 300, 600, 0),
                                         (5600, 300, 600, 1),
                                         # odd leading dimensions: pairs loaded one
                                         # element at a time
                                         (1001, 625, 625, 0), (10001, 625, 625, 1),
                                         (2001, 159, 777, 0)])
def test_gemm_f64_matches_numpy(M, N, K, trans):
    rng = np.random.default_rng(M * 7 + N)
    A = [rng.standard_normal((K, M) if trans else (M, K)) for _ in range(3)]
    B = [rng.standard_normal((K, N)) for _ in range(3)]
    Ad, Bd = [dev(a) for a in A], [dev(b) for b in B]
    Cd = [torch.zeros(M, N, dtype=torch.float64, device="cuda") for _ in range(3)]
    P.gemm_f64(Ad, Bd, Cd, M, N, K, trans_a=trans)
    torch.cuda.synchronize()
    for a, b, c in zip(A, B, Cd):
        ref = (a.T if trans else a) @ b
        err = np.abs(c.cpu().numpy() - ref).max()
        assert err <= 1e-12 * np.sqrt(K) * np.abs(ref).max()


def test_gemm_accumulate_and_alpha():
    rng = np.random.default_rng(1)
    A, B, C0 = rng.standard_normal((40, 50)), rng.standard_normal((50, 30)), rng.standard_normal((40, 30))
    Cd = dev(C0.copy())
    P.gemm_f64([dev(A)], [dev(B)], [Cd], 40, 30, 50, alpha=-0.5, accumulate=1)
    torch.cuda.synchronize()
    assert np.allclose(Cd.cpu().numpy(), C0 - 0.5 * A @ B, atol=1e-12)


SPLIT_CASES = [
    # count, M, N, K, trans per problem, lda, CUs, alpha, accumulate, split expected
    (8, 3000, 160, 3000, [0, 0, 0, 0, 1, 1, 1, 1], None, 256, 1.0, 0, True),  # ragged M and K
    (3, 1000, 78, 515, [1, 0, 1], 1000, 32, -0.5, 1, True),   # mixed, padded lda, 0.6-tile ranges
    (1, 4000, 160, 250, [0], None, 8, 1.0, 0, True),          # ranges of 2.6 tiles
    (1, 400, 16, 300, [1], None, 2, 2.0, 1, True),            # two ranges of 1.5 tiles
    (2, 700, 100, 260, [0, 1], 700, 1, 1.0, 0, True),         # one range: every tile whole
    (2, 2000, 33, 4001, [0, 0], None, 256, 1.0, 0, False),    # odd lda: the plain tile kernel
    (8, 500, 160, 500, [0] * 8, None, 256, 1.0, 0, True),     # 24 tiles in 96 ranges of 8 slices
    (4, 3000, 64, 200, [0] * 4, None, 256, 1.0, 0, False),    # 13 K slices: the plain tile kernel
    (6, 2500, 105, 2500, [0, 0, 0, 1, 1, 1], None, 256, 1.0, 0, True),  # odd ldb, 84 long tiles
    (2, 1000, 127, 2100, [1, 0], 2100, 32, -1.0, 1, True),    # odd ldb, 128-wide tiles, ragged
]


@pytest.mark.parametrize("case", range(len(SPLIT_CASES)))
def test_gemm_split_matches_numpy(case):
    count, M, N, K, trans, lda, ncu, alpha, acc, expect = SPLIT_CASES[case]
    rng = np.random.default_rng(100 + case)
    lda = lda or (M if trans[0] else K)
    A = []
    for t in trans:
        rows, cols = (K, M) if t else (M, K)
        full = rng.standard_normal((rows, lda))
        A.append(full)
    B = [rng.standard_normal((K, N)) for _ in range(count)]
    C0 = [rng.standard_normal((M, N)) for _ in range(count)]
    scratch = torch.empty(P.gemm_f64_split_scratch_bytes() // 8, dtype=torch.float64, device="cuda")
    Ad, Bd = [dev(a) for a in A], [dev(b) for b in B]
    outs = []
    for rep in range(2):
        Cd = [dev(c.copy()) for c in C0]
        used = P.gemm_f64_split(Ad, Bd, Cd, M, N, K, trans, scratch, ncu=ncu, lda=lda,
                                alpha=alpha, accumulate=acc)
        torch.cuda.synchronize()
        assert used == expect
        outs.append([c.cpu().numpy() for c in Cd])
    for i, (a, t) in enumerate(zip(A, trans)):
        op = a[:, :M].T if t else a[:, :K]
        ref = alpha * (op @ B[i]) + (C0[i] if acc else 0.0)
        # a length-K float64 dot product in any order is within (K + 2) u of
        # the sum of |terms| (u = 2^-53); twice that covers NumPy's own rounding
        bound = 2 * (K + 2) * 2.0 ** -53 * (abs(alpha) * (np.abs(op) @ np.abs(B[i])) +
                                           (np.abs(C0[i]) if acc else 0.0))
        assert np.all(np.abs(outs[0][i] - ref) <= bound), i
        assert np.array_equal(outs[0][i], outs[1][i]), i      # fixed summation order


def test_gemm_split_without_scratch_runs_plain_tiles():
    rng = np.random.default_rng(5)
    A, B = rng.standard_normal((3000, 3000)), rng.standard_normal((3000, 96))
    Cd = [torch.zeros(3000, 96, dtype=torch.float64, device="cuda") for _ in range(8)]
    used = P.gemm_f64_split([dev(A)] * 8, [dev(B)] * 8, Cd, 3000, 96, 3000, [0] * 8, None)
    torch.cuda.synchronize()
    assert not used
    ref = A @ B
    assert np.abs(Cd[7].cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


# leaf counts 1, 1, 8, 19, 32, 6, 23 and 156: reduction-tree nodes with two,
# three and four children at several strides
@pytest.mark.parametrize("N,k", [(32, 24), (100, 100), (1024, 72), (2500, 105), (5184, 160),
                                 (777, 33), (3000, 40), (20000, 8)])
def test_householder_qr(N, k):
    W = [S.gaussian_block(N, k, 3 + i) for i in range(4)]
    W[1][:, 5] = 0.0                              # a zero column (tau = 0 path)
    W[2][:, 3] = 2.0 * W[2][:, 1]                 # exactly dependent columns
    Wd = [dev(w) for w in W]
    P.qr_f64(Wd)
    torch.cuda.synchronize()
    for i, (w, q) in enumerate(zip(W, Wd)):
        Q = q.cpu().numpy()
        assert np.all(np.isfinite(Q))
        assert np.abs(Q.T @ Q - np.eye(k)).max() <= 1e-13 * np.sqrt(N)
        R = Q.T @ w
        assert np.abs(np.tril(R, -1)).max() <= 1e-12 * np.abs(w).max() * np.sqrt(N)
        assert np.all(np.diag(R) >= -1e-12 * np.abs(w).max())
        if i in (0, 3):                           # full rank: unique, equals the oracle's
            assert np.abs(Q - O.qr_pos(w)).max() <= 1e-11


@pytest.mark.parametrize("n", [7, 24, 72, 105, 160])
def test_jacobi_svd(n):
    rng = np.random.default_rng(n)
    mats = [rng.standard_normal((n, n)),
            rng.standard_normal((n, n)) @ np.diag(np.logspace(0, -13, n)) @ rng.standard_normal((n, n)),
            np.outer(rng.standard_normal(n), rng.standard_normal(n))]
    rd = [dev(m) for m in mats]
    ud = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for _ in mats]
    vd = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for _ in mats]
    sd = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in mats]
    P.svd_f64(rd, ud, sd, vd)
    torch.cuda.synchronize()
    for m, u, s, v in zip(mats, ud, sd, vd):
        U, Sv, V = u.cpu().numpy(), s.cpu().numpy(), v.cpu().numpy()
        ref = np.linalg.svd(m, compute_uv=False)
        assert np.all(np.diff(Sv) <= 0)
        assert np.abs(Sv - ref).max() <= 1e-13 * ref[0] * n
        assert np.abs(U.T @ U - np.eye(n)).max() <= 1e-12 * n
        assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-12 * n
        assert np.abs((U * Sv) @ V.T - m).max() <= 1e-13 * ref[0] * n


@pytest.mark.parametrize("n,r", [(105, 40), (192, 70), (160, 1), (64, 0)])
def test_jacobi_svd_rank_deficient(n, r):
    """Rank-r matrices: the n - r numerically zero columns are completed to an
    orthonormal basis (the staged non-zero columns span several LDS chunks
    at r = 40 and 70; n = 192 gives three rows per lane) and the product still
    reconstructs the input."""
    rng = np.random.default_rng(1000 + n + r)
    m = rng.standard_normal((n, r)) @ rng.standard_normal((r, n)) if r else np.zeros((n, n))
    rd = [dev(m)]
    ud = [torch.zeros(n, n, dtype=torch.float64, device="cuda")]
    vd = [torch.zeros(n, n, dtype=torch.float64, device="cuda")]
    sd = [torch.zeros(n, dtype=torch.float64, device="cuda")]
    P.svd_f64(rd, ud, sd, vd)
    torch.cuda.synchronize()
    U, Sv, V = ud[0].cpu().numpy(), sd[0].cpu().numpy(), vd[0].cpu().numpy()
    ref = np.linalg.svd(m, compute_uv=False)
    scale = max(ref[0], 1.0)
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    assert np.all(np.diff(Sv) <= 0)
    assert np.abs(Sv - ref).max() <= 1e-13 * scale * n
    assert np.abs(U.T @ U - np.eye(n)).max() <= 1e-12 * n
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-12 * n
    assert np.abs((U * Sv) @ V.T - m).max() <= 1e-13 * scale * n


def test_jacobi_svd_values_only():
    rng = np.random.default_rng(9)
    m = rng.standard_normal((50, 50))
    s = torch.zeros(50, dtype=torch.float64, device="cuda")
    P.svd_f64([dev(m)], None, [s], None)
    torch.cuda.synchronize()
    assert np.allclose(s.cpu().numpy(), np.linalg.svd(m, compute_uv=False), rtol=1e-13, atol=1e-13)
