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
