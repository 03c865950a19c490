"""Second, independent gradient check of the GPU backward: the GPU computes
the discrete adjoint of its scheme (the exact gradient of the computed
value), the oracle here the continuous adjoint of the exact kernel (Riemann's
method, with the interior of every cell from the double series of
Proposition "prop:a1").  With these cell constants (|c| < 0.1) the schemes'
truncation at N = 8 (approximation) and N = 6 (interpolation) changes the
gradient by less than 2e-15 (checked on the CPU against the complex-step
gradient of the oracle schemes), so the two routes must agree to rounding:
1e-12 relative in the max norm for FP64, 1e-5 for FP32."""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


def dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


_CACHE = {}


def continuous_gram_grad(X, Y, gK):
    # edges at N = 12 and interior series to degree 24 are converged here
    # (1e-16 against N = 24, degree 48)
    from oracle import derivatives as D
    key = X.tobytes() + Y.tobytes()
    if key not in _CACHE:
        _CACHE[key] = {(a, b): D.continuous_adjoint_grad(X[a], Y[b], N=12, M=24)[1:]
                       for a in range(len(X)) for b in range(len(Y))}
    gX, gY = np.zeros_like(X), np.zeros_like(Y)
    for (a, b), (ga, gb) in _CACHE[key].items():
        gX[a] += gK[a, b] * ga
        gY[b] += gK[a, b] * gb
    return gX, gY


@pytest.mark.parametrize("dtype,scheme,order,tol", [
    (torch.float64, "approx", 8, 1e-12),
    (torch.float64, "interp", 6, 1e-12),
    (torch.float32, "approx", 8, 1e-5),
])
def test_discrete_adjoint_matches_continuous_adjoint(sk, dtype, scheme, order, tol):
    log_banner(f"continuous adjoint check {dtype} {scheme} {order}")
    rng = np.random.default_rng(71)
    # x paths of 70 points: two strips, so the adjoint's strip hand-off is in play
    X = bm_paths(rng, 2, 69, 3, 0.1)
    Y = bm_paths(rng, 2, 40, 3, 0.1)
    gK = rng.normal(size=(2, 2))
    if dtype == torch.float32:
        X, Y = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    gX, gY = sk.gram_backward(dev(X, dtype), dev(Y, dtype), dev(gK, dtype), scheme, order)
    oX, oY = continuous_gram_grad(X, Y, gK)
    ex = np.abs(gX.cpu().numpy() - oX).max() / np.abs(oX).max()
    ey = np.abs(gY.cpu().numpy() - oY).max() / np.abs(oY).max()
    assert ex < tol and ey < tol, (ex, ey)
