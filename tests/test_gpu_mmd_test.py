"""The MMD permutation two-sample test: permutation statistics and p-value
from the library's kernels against the oracle's, on the same pooled Gram
matrix and the same permutations."""
import numpy as np
import pytest

from tests.gpu_common import log_banner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_permutation_stats_match_oracle(sk, dtype, tol):
    from oracle import schemes as S
    from paper_2502_08470_amd import _lib as L
    import ctypes
    log_banner(f"mmd permutation stats {dtype}")
    rng = np.random.default_rng(81)
    m, n = 13, 9
    A = rng.normal(size=(m + n, 4))
    K = np.exp(-0.3 * ((A[:, None, :] - A[None, :, :]) ** 2).sum(-1))
    perms = np.stack([np.arange(m + n)] + [rng.permutation(m + n) for _ in range(40)]).astype(np.int32)
    want = S.mmd_permutation_stats(K, m, perms)
    Kt = torch.tensor(K, dtype=dtype, device="cuda")
    Pt = torch.tensor(perms, device="cuda")
    st = torch.empty(len(perms), dtype=dtype, device="cuda")
    pv = torch.empty(1, dtype=torch.float64, device="cuda")
    dt = L.SK_F32 if dtype == torch.float32 else L.SK_F64
    s = torch.cuda.current_stream().cuda_stream
    L.check(L.lib().sigkernel_mmd_permutation(ctypes.c_void_p(Kt.data_ptr()), m, n,
                                              ctypes.c_void_p(Pt.data_ptr()), len(perms), dt,
                                              ctypes.c_void_p(st.data_ptr()),
                                              ctypes.c_void_p(pv.data_ptr()), ctypes.c_void_p(s)))
    got = st.cpu().double().numpy()
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=0, atol=tol * scale)
    if dtype == torch.float64:  # same decisions in the same precision
        assert float(pv) == pytest.approx(S.mmd_permutation_pvalue(want), abs=0)


def test_two_sample_test_api(sk):
    from oracle import c_oracle as C
    from oracle import schemes as S
    import workloads as W
    log_banner("mmd permutation test api")
    X, Y = W.mmd_sets(0, n=24, steps=64)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    stat, p, null = sk.mmd_permutation_test(torch.tensor(Xd, device="cuda"),
                                            torch.tensor(Yd, device="cuda"),
                                            "approx", 6, n_perm=200, seed=3)
    Z = np.concatenate([Xd, Yd], 0)
    Kzz = C.value(*C.gram(Z, Z, C.APPROX, 6))
    rng = np.random.default_rng(3)
    perms = np.stack([np.arange(48)] + [rng.permutation(48) for _ in range(200)])
    want = S.mmd_permutation_stats(Kzz, 24, perms)
    assert stat == pytest.approx(want[0], rel=1e-10)
    np.testing.assert_allclose(null.cpu().numpy(), want[1:], rtol=1e-10, atol=1e-12)
    # the count is decided in FP64 on both sides; a null statistic within
    # rounding of the observed one may fall either way
    near = np.count_nonzero(np.abs(want[1:] - want[0]) <= 1e-9 * abs(want[0]))
    assert abs(p - S.mmd_permutation_pvalue(want)) <= near / 201 + 1e-12
    # relabelled copies of one sample: the observed split is no longer special
    stat0, p0, _ = sk.mmd_permutation_test(torch.tensor(Xd[:12], device="cuda"),
                                           torch.tensor(Xd[12:], device="cuda"),
                                           "approx", 6, n_perm=200, seed=4)
    assert 0.0 < p0 <= 1.0


def _pair_list(K, nx):
    """The [XX pairs a < b | YY pairs a < b | XY pairs] layout of a pooled
    Gram matrix whose first nx rows are the first set."""
    ny = K.shape[0] - nx
    ia, ib = np.triu_indices(nx, 1)
    ja, jb = np.triu_indices(ny, 1)
    return np.concatenate([K[ia, ib], K[nx + ja, nx + jb], K[:nx, nx:].reshape(-1)])


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_mmd2_pair_list_statistic_and_seeds(sk, dtype, tol):
    """sigkernel_mmd2_pairs against the oracle's unbiased MMD^2 and against
    the permutation kernel's statistic of the observed split (the same
    statistic from the pooled matrix); sigkernel_mmd2_pairs_backward against
    the statistic's weights, group by group."""
    from oracle import schemes as S
    from paper_2502_08470_amd import _lib as L
    import ctypes
    log_banner(f"mmd2 pair list {dtype}")
    rng = np.random.default_rng(83)
    nx, ny = 11, 7
    A = rng.normal(size=(nx + ny, 3))
    K = np.exp(-0.4 * ((A[:, None, :] - A[None, :, :]) ** 2).sum(-1))
    want = S.mmd2_unbiased(K[:nx, :nx], K[nx:, nx:], K[:nx, nx:])
    k = torch.tensor(_pair_list(K, nx), dtype=dtype, device="cuda")
    out = torch.empty(1, dtype=dtype, device="cuda")
    dt = L.SK_F32 if dtype == torch.float32 else L.SK_F64
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    L.check(L.lib().sigkernel_mmd2_pairs(vp(k), nx, ny, dt, vp(out), s))
    got = float(out.cpu())
    assert got == pytest.approx(want, rel=tol, abs=tol * np.abs(K).max())
    # the permutation kernel's observed-split statistic on the pooled matrix
    Kt = torch.tensor(K, dtype=dtype, device="cuda")
    Pt = torch.tensor(np.arange(nx + ny, dtype=np.int32)[None], device="cuda")
    st = torch.empty(1, dtype=dtype, device="cuda")
    L.check(L.lib().sigkernel_mmd_permutation(vp(Kt), nx, ny, vp(Pt), 1, dt, vp(st), None, s))
    assert got == pytest.approx(float(st.cpu()), rel=tol, abs=tol * np.abs(K).max())
    # seeds: dMMD^2/dk times g, constant within each group
    g = torch.tensor([0.75], dtype=dtype, device="cuda")
    gk = torch.empty_like(k)
    L.check(L.lib().sigkernel_mmd2_pairs_backward(vp(g), nx, ny, dt, vp(gk), s))
    nxx, nyy = nx * (nx - 1) // 2, ny * (ny - 1) // 2
    w = np.concatenate([np.full(nxx, 2.0 / (nx * (nx - 1))), np.full(nyy, 2.0 / (ny * (ny - 1))),
                        np.full(nx * ny, -2.0 / (nx * ny))]) * 0.75
    np.testing.assert_allclose(gk.cpu().double().numpy(), w, rtol=tol, atol=0)
    # the statistic is linear in k: the seeds are its exact gradient
    assert float(np.dot(w / 0.75, _pair_list(K, nx))) == pytest.approx(want, rel=1e-12)


def test_mmd2_routes_agree_with_the_permutation_test(sk):
    """The differentiable MMD^2 (pair list, and three Gram matrices with MFMA
    constants) equals the permutation test's observed statistic on the same
    sets (FP64), and both routes give the same gradient."""
    import workloads as W
    log_banner("mmd2 routes")
    X, Y = W.mmd_sets(1, n=10, steps=48)
    Xd = torch.tensor(X.astype(np.float64), device="cuda")
    Yd = torch.tensor(Y.astype(np.float64), device="cuda")
    stat, _, _ = sk.mmd_permutation_test(Xd, Yd, "approx", 6, n_perm=1, seed=0)
    Xa, Ya = Xd.clone().requires_grad_(True), Yd.clone().requires_grad_(True)
    v1 = sk.mmd2(Xa, Ya, "approx", 6)
    v1.backward()
    Xb, Yb = Xd.clone().requires_grad_(True), Yd.clone().requires_grad_(True)
    v2 = sk.mmd2(Xb, Yb, "approx", 6, gram_mode="mfma")
    v2.backward()
    assert float(v1) == pytest.approx(stat, rel=1e-10, abs=1e-14)
    assert float(v2) == pytest.approx(stat, rel=1e-10, abs=1e-14)
    for a, b in ((Xa.grad, Xb.grad), (Ya.grad, Yb.grad)):
        scale = a.abs().max().item()
        assert (a - b).abs().max().item() <= 1e-9 * scale
