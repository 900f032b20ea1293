"""The allocation-free QR entry point (ctm_qr_f64_noalloc) against the
allocating one (ctm_qr_f64), through the C ABI: the same kernels on the same
inputs give the same bits, on two calls in a row (the second smaller, so the
static scratch holds the first call's contents), and a workspace beyond the
static scratch is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2607_15158_amd as P  # noqa: E402
import synth as S  # noqa: E402


def blocks(count, N, k, seed):
    return [S.gaussian_block(N, k, seed + i) for i in range(count)]


def run_both(hs):
    a = [torch.from_numpy(h).cuda() for h in hs]
    b = [torch.from_numpy(h).cuda() for h in hs]
    P.qr_f64(a)
    P.qr_f64_noalloc(b)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in a], [x.cpu().numpy() for x in b]


def test_noalloc_qr_equals_allocating_qr_on_two_calls():
    # first call: the benchmark's shape (8 blocks of 5184 x 160, 71 MiB of scratch)
    first = blocks(8, 5184, 160, 300)
    qa, qb = run_both(first)
    for x, y, h in zip(qa, qb, first):
        assert np.array_equal(x, y)
        assert np.abs(x.T @ x - np.eye(160)).max() <= 1e-13
        r = x.T @ h
        assert np.abs(x @ r - h).max() <= 1e-12 * np.abs(h).max()
    # second call, smaller and ragged: the scratch keeps the first call's contents
    second = blocks(3, 1000, 37, 400)
    qa, qb = run_both(second)
    for x, y in zip(qa, qb):
        assert np.array_equal(x, y)
        assert np.abs(x.T @ x - np.eye(37)).max() <= 1e-13


def test_noalloc_qr_refuses_a_workspace_beyond_its_scratch():
    assert P._lib.ctm_qr_f64_noalloc_max_bytes() == 96 << 20
    # 8 blocks of 49152 x 192 (leaves of 192 rows) need about 0.8 GB of workspace
    big = [torch.zeros(49152, 192, dtype=torch.float64, device="cuda") for _ in range(8)]
    with pytest.raises(P.CtmError) as e:
        P.qr_f64_noalloc(big)
    assert e.value.status == P.CTM_E_NOMEM
