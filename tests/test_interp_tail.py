"""Host side of the interpolation scheme's tail (no GPU).

The GPU map applies Definition "interpooperator" to the exact edge of
Proposition "propinterp" as the untruncated rows of the approximation map
plus a fixed projection of the rows past N (the tail).  These tests pin the
projection tables the library builds against the Chebyshev-extrema
interpolation of monomials, the decay bound behind the tail's stopping rule,
and -- by running that rule on the host over the tables -- that the compiled
tail caps hold every cell with |c| up to 10 and that the rule's result is the
literal oracle's cell map (oracle.schemes.interp_cell) to the working
precision."""
import math

import numpy as np
import pytest

from oracle import schemes as S
from paper_2502_08470_amd import _lib as L

EPS = {L.SK_F32: 2.0 ** -26, L.SK_F64: 2.0 ** -55}
ORDERS = list(range(2, 13))


def interp_monomial(N, r):
    """Coefficients of the degree-N interpolant of u^r at the order-N
    Chebyshev extrema of [0, 1] (numpy's own solve)."""
    u = S.chebyshev_extrema(N, 0.0, 1.0)
    return np.linalg.solve(np.vander(u, N + 1, increasing=True), u ** r)


@pytest.mark.parametrize("N", ORDERS)
def test_projection_table_interpolates_monomials(N):
    rs, rmax, cmax, cap = L.interp_table(N, L.SK_F64)
    assert cap == 20
    for t in range(L.SK_TAIL_TABLE):
        r = N + 1 + t
        ref = interp_monomial(N, r) * np.array([math.factorial(n) for n in range(N + 1)]) / math.factorial(r)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(rs[:, t] - ref)) <= 1e-7 * scale, (N, t)
        assert rmax[t] == pytest.approx(np.max(np.abs(rs[:, t])), rel=1e-12)


@pytest.mark.parametrize("N", ORDERS)
def test_stopping_rule_decay_bound_holds_far_out(N):
    """cmax[t] promises that every later row's projection weight times
    |c| / (t + 2) shrinks by at least half, for |c| <= cmax[t]."""
    _, _, cmax, _ = L.interp_table(N, L.SK_F64)
    nf = np.array([math.factorial(n) for n in range(N + 1)], dtype=float)
    # log of max_n |R[n][r]| n! / r! for r far past the table
    lw = []
    for r in range(N + 1, N + 1 + 140):
        q = np.max(np.abs(interp_monomial(N, r)) * nf)
        lw.append(math.log(q) - math.lgamma(r + 1))
    lw = np.array(lw)
    ratio = np.exp(np.diff(lw))
    for t in range(L.SK_TAIL_TABLE + 1):
        assert np.all(ratio[t:] * cmax[t] / (t + 2) <= 0.5 * (1 + 1e-6)), (N, t)
        assert cmax[t] > 0


def tail_map(P, Q, c, N, dtype):
    """The stopping rule of the GPU map, in FP64 on the host: returns the
    scaled-basis outputs and the number of folded tail rows (None when the
    cap is exceeded)."""
    rs, rmax, cmax, cap = L.interp_table(N, dtype)
    eps = EPS[dtype]

    def row(r, A, B):
        t = sum(c ** (r - k) / math.factorial(r - k) * A[k] for k in range(0, min(r, N) + 1))
        return t + c ** r * sum(B[k] / math.factorial(r + k) for k in range(1, N + 1))

    Po = np.array([row(r, P, Q) for r in range(N + 1)])
    Qo = np.array([row(r, Q, P) for r in range(N + 1)])
    scale = eps * (abs(Po[0]) + abs(Qo[0]))
    for t in range(cap + 1):
        r = N + 1 + t
        ap, aq = row(r, P, Q), row(r, Q, P)
        need = not (2 * rmax[t] * (abs(ap) + abs(aq)) <= scale) or abs(c) > cmax[t]
        if not need:
            return Po, Qo, t
        if t == cap:
            return Po, Qo, None
        Po = Po + rs[:, t] * ap
        Qo = Qo + rs[:, t] * aq
    raise AssertionError("unreachable")


@pytest.mark.parametrize("dtype", [L.SK_F32, L.SK_F64])
@pytest.mark.parametrize("N", [2, 3, 4, 6, 8])
def test_compiled_tail_caps_hold_cells_up_to_c_10(dtype, N):
    rng = np.random.default_rng(100 * N + dtype)
    fact = np.array([math.factorial(n) for n in range(N + 1)], dtype=float)
    worst = 0
    for c in [0.01, -0.3, 0.7, -1.0, 2.0, -3.5, 5.0, -5.0, 8.0, -8.0, 10.0, -10.0]:
        for _ in range(3):
            g = np.concatenate([[1.0], rng.normal(0, 0.5, N)])
            h = np.concatenate([[1.0], rng.normal(0, 0.5, N)])
            Po, Qo, T = tail_map(g * fact, h * fact, c, N, dtype)
            assert T is not None, (N, c)
            worst = max(worst, T)
            # the rule's map is the literal cell map (0F1 at the nodes + solve)
            top, right = S.interp_cell(g, h, c, 0.0, 1.0, 0.0, 1.0, N)
            ref = np.concatenate([top, right])
            got = np.concatenate([Po, Qo]) / np.concatenate([fact, fact])
            tol = (1e-6 if dtype == L.SK_F32 else 1e-10) * np.max(np.abs(ref))
            assert np.max(np.abs(got - ref)) <= tol, (N, c, np.max(np.abs(got - ref)))
    assert worst >= 3  # large |c| does exercise tails past the unrolled rows


def test_cells_past_the_cap_are_detected():
    # |c| = 60 needs far more than the compiled rows in either precision
    for dtype in (L.SK_F32, L.SK_F64):
        g = np.array([1.0, 0.2, -0.1, 0.05])
        _, _, T = tail_map(g, g, 60.0, 3, dtype)
        assert T is None
