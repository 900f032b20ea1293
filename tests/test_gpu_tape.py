"""The reverse-mode tape behind the cell adjoint, one operation at a time
(ctm_tape_check_*), against torch autograd of the same operation on the CPU
in float64: GEMMs with plain, transposed, two-level-mapped and batched
operands, the thin QR, the projector factors of rho, and the unit-norm
scaling."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle.ctmrg as O  # noqa: E402
import paper_2607_15158_amd as P  # noqa: E402

DEV = torch.device("cuda", 0)
L = P._lib
_vp = ctypes.c_void_p
L.ctm_tape_check_gemm.restype = ctypes.c_int
L.ctm_tape_check_gemm.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_long),
                                  ctypes.c_double, _vp, ctypes.c_long, _vp, ctypes.c_long, _vp,
                                  ctypes.c_long, _vp, _vp, _vp]
L.ctm_tape_check_qr.restype = ctypes.c_int
L.ctm_tape_check_qr.argtypes = [ctypes.c_int] * 3 + [_vp] * 4
L.ctm_tape_check_svdproj.restype = ctypes.c_int
L.ctm_tape_check_svdproj.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double] + [_vp] * 5
L.ctm_tape_check_normalize.restype = ctypes.c_int
L.ctm_tape_check_normalize.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_long), _vp, _vp, _vp, _vp]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def gemm_ref(M, N, K, tA, cdm, cdn, nb, lda, ldb, m1, m0, n1, n0, abs_, bbs, cbs, alpha, A, B, nC):
    """C[b c_bs + map(m, n)] = alpha sum_k A(m, k) B(k, n) with torch tensors."""
    C = torch.zeros(nC, dtype=torch.float64)
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    kk = np.arange(K)
    for b in range(nb):
        ia = (kk[None, :] * lda + np.arange(M)[:, None]) if tA else (np.arange(M)[:, None] * lda + kk[None, :])
        ib = kk[:, None] * ldb + np.arange(N)[None, :]
        Am = A[torch.from_numpy(ia + b * abs_)]
        Bm = B[torch.from_numpy(ib + b * bbs)]
        off = b * cbs + (m // cdm) * m1 + (m % cdm) * m0 + (n // cdn) * n1 + (n % cdn) * n0
        C = C.index_put((torch.from_numpy(off.ravel()),), (alpha * (Am @ Bm)).ravel())
    return C


CASES = {
    # plain
    "plain": (5, 7, 3, 0, 1 << 30, 1 << 30, 1, 3, 7, 0, 7, 0, 1, 0, 0, 0, 1.0),
    # transposed A (stored K x M) and alpha
    "trans": (6, 4, 5, 1, 1 << 30, 1 << 30, 1, 6, 4, 0, 4, 0, 1, 0, 0, 0, -0.5),
    # two-level output map (columns (q, y) stored as [y][q], as the corner stems)
    "map": (3, 9, 3, 0, 1 << 30, 3, 1, 3, 9, 0, 9, 1, 3, 0, 0, 0, 1.0),
    # map on both indices (rows (x, p), columns (y, q))
    "map2": (6, 6, 2, 0, 3, 3, 1, 2, 6, 18, 3, 9, 1, 0, 0, 0, 1.0),
    # inner batch with a shared A (the edge renormalisation)
    "batch": (4, 3, 2, 0, 2, 1 << 30, 3, 2, 9, 18, 1, 0, 6, 0, 3, 2, 1.0),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_taped_gemm_vjp_matches_autograd(case):
    M, N, K, tA, cdm, cdn, nb, lda, ldb, m1, m0, n1, n0, abs_, bbs, cbs, alpha = CASES[case]
    rng = np.random.default_rng(1)
    nA = (K - 1) * lda + M + (nb - 1) * abs_ if tA else (M - 1) * lda + K + (nb - 1) * abs_
    nB = (K - 1) * ldb + N + (nb - 1) * bbs
    mx = lambda n, d, s1, s0: ((n - 1) // d) * s1 + min(d - 1, n - 1) * s0  # noqa: E731
    nC = mx(M, cdm, m1, m0) + mx(N, cdn, n1, n0) + (nb - 1) * cbs + 1
    A = rng.standard_normal(nA)
    B = rng.standard_normal(nB)
    Cb = rng.standard_normal(nC)
    At = torch.tensor(A, requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    C = gemm_ref(M, N, K, tA, cdm, cdn, nb, lda, ldb, m1, m0, n1, n0, abs_, bbs, cbs, alpha, At, Bt, nC)
    (C * torch.from_numpy(Cb)).sum().backward()
    dA, dB, dCb = dev(A), dev(B), dev(Cb)
    gC = torch.zeros(nC, dtype=torch.float64, device=DEV)
    gA = torch.empty_like(dA)
    gB = torch.empty_like(dB)
    dims = (ctypes.c_int * 7)(M, N, K, tA, cdm, cdn, nb)
    st = (ctypes.c_long * 9)(lda, ldb, m1, m0, n1, n0, abs_, bbs, cbs)
    torch.cuda.synchronize()
    assert L.ctm_tape_check_gemm(dims, st, alpha, dA.data_ptr(), nA, dB.data_ptr(), nB, gC.data_ptr(),
                                 nC, dCb.data_ptr(), gA.data_ptr(), gB.data_ptr()) == 0
    assert rel(gC.cpu().numpy(), C.detach().numpy()) <= 1e-14
    assert rel(gA.cpu().numpy(), At.grad.numpy()) <= 1e-13, case
    assert rel(gB.cpu().numpy(), Bt.grad.numpy()) <= 1e-13, case


def test_taped_qr_vjp_matches_autograd():
    count, n, k = 3, 200, 12
    rng = np.random.default_rng(2)
    H = rng.standard_normal((count, n, k))
    Qb = rng.standard_normal((count, n, k))
    Ht = torch.tensor(H, requires_grad=True)
    total = 0.0
    Qs = []
    for j in range(count):
        q, r = torch.linalg.qr(Ht[j])
        sg = torch.sign(torch.diagonal(r)).detach()
        q = q * sg
        Qs.append(q)
        total = total + (q * torch.from_numpy(Qb[j])).sum()
    total.backward()
    dH, dQb = dev(H), dev(Qb)
    Q = torch.empty_like(dH)
    Hb = torch.empty_like(dH)
    torch.cuda.synchronize()
    assert L.ctm_tape_check_qr(count, n, k, dH.data_ptr(), Q.data_ptr(), dQb.data_ptr(),
                               Hb.data_ptr()) == 0
    assert rel(Q.cpu().numpy(), np.stack([q.detach().numpy() for q in Qs])) <= 1e-12
    assert rel(Hb.cpu().numpy(), Ht.grad.numpy()) <= 1e-10


@pytest.mark.parametrize("decades", [3, 10])
def test_taped_projector_factors_vjp_matches_autograd(decades):
    """Singular values over 3 and over 10 decades: the kept values of rho in
    a move span many orders of magnitude, and the inverse gaps of the SVD
    adjoint must stay exact for the small ones (a broadening on the scale
    of s_1^2 would suppress them)."""
    k, keep, nrows = 12, 8, 40
    rng = np.random.default_rng(3)
    rho = (np.linalg.qr(rng.standard_normal((k, k)))[0] @ np.diag(np.logspace(0, -decades, k)) @
           np.linalg.qr(rng.standard_normal((k, k)))[0])
    Yt = rng.standard_normal((nrows, k))
    bars = [rng.standard_normal((k, k)), rng.standard_normal((k, k)), rng.standard_normal((k, keep)),
            rng.standard_normal((k, keep))]
    rt = torch.tensor(rho, requires_grad=True)
    u, s, vt = torch.linalg.svd(rt)
    v = vt.T
    sg = torch.from_numpy(O.sign_fix_columns(Yt @ u.detach().numpy()))
    us, vs = u * sg, v * sg
    sinv = torch.zeros(keep, dtype=torch.float64)
    sinv = s[:keep] ** -0.5
    outs = [us, vs, vs[:, :keep] * sinv, us[:, :keep] * sinv]
    sum((o * torch.from_numpy(b)).sum() for o, b in zip(outs, bars)).backward()
    flat_b = dev(np.concatenate([b.ravel() for b in bars]))
    got = torch.empty_like(flat_b)
    rb = torch.empty(k * k, dtype=torch.float64, device=DEV)
    drho, dY = dev(rho), dev(Yt)
    torch.cuda.synchronize()
    assert L.ctm_tape_check_svdproj(k, keep, nrows, 1e-12, drho.data_ptr(), dY.data_ptr(),
                                    got.data_ptr(), flat_b.data_ptr(), rb.data_ptr()) == 0
    ref = np.concatenate([o.detach().numpy().ravel() for o in outs])
    # the weakest singular vectors are set to ~ eps / (relative gap): 4e-11 at 10 decades
    assert rel(got.cpu().numpy(), ref) <= (1e-11 if decades == 3 else 1e-9)
    # the SVD adjoint's inverse gaps amplify rounding (4e-9 measured)
    assert rel(rb.cpu().numpy().reshape(k, k), rt.grad.numpy()) <= 3e-8, decades


def test_taped_normalize_vjp_matches_autograd():
    ns = [37, 5, 100]
    rng = np.random.default_rng(4)
    x = rng.standard_normal(sum(ns))
    yb = rng.standard_normal(sum(ns))
    xt = torch.tensor(x, requires_grad=True)
    parts = torch.split(xt, ns)
    ys = [p / torch.linalg.norm(p) for p in parts]
    (torch.cat(ys) * torch.from_numpy(yb)).sum().backward()
    dx, dyb = dev(x), dev(yb)
    y = torch.empty_like(dx)
    xb = torch.empty_like(dx)
    n = (ctypes.c_long * 3)(*ns)
    torch.cuda.synchronize()
    assert L.ctm_tape_check_normalize(3, n, dx.data_ptr(), y.data_ptr(), dyb.data_ptr(),
                                      xb.data_ptr()) == 0
    assert rel(y.cpu().numpy(), torch.cat(ys).detach().numpy()) <= 1e-15
    assert rel(xb.cpu().numpy(), xt.grad.numpy()) <= 1e-13
