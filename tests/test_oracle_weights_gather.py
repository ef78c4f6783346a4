"""Pins of the oracle's weight functions and field gather (paper Sec. II, eq. "pfields",
B-spline weight list).  Each pin is independent of the oracle's own code: a centred cardinal
B-spline built from truncated powers, moment identities, and brute-force sums over all
periodic images."""
import math

import numpy as np
import pytest


def bspline_truncated_power(order_n: int, x: float) -> float:
    """Centred cardinal B-spline M_n (degree n-1) from its truncated-power expansion
    M_n(x) = 1/(n-1)! sum_k (-1)^k C(n,k) (x + n/2 - k)_+^(n-1)."""
    n = order_n
    s = 0.0
    for k in range(n + 1):
        t = x + n / 2.0 - k
        if t > 0:
            s += (-1) ** k * math.comb(n, k) * t ** (n - 1)
    return s / math.factorial(n - 1)


@pytest.mark.parametrize("O", [1, 2, 3])
def test_weight_is_cardinal_bspline(orc, O):
    # the weight of order O is the shape (B-spline of degree O-1) integrated over a cell,
    # i.e. the centred cardinal B-spline of degree O
    for x in np.linspace(-2.6, 2.6, 1041):
        assert abs(orc.W(O, x) - bspline_truncated_power(O + 1, x)) < 1e-14


@pytest.mark.parametrize("O", [2, 3])
def test_weight_moments(orc, O):
    rng = np.random.default_rng(1)
    for X in rng.uniform(-3, 3, 200):
        nodes = np.arange(math.floor(X) - 4, math.floor(X) + 5)
        w = np.array([orc.W(O, i - X) for i in nodes])
        assert abs(w.sum() - 1.0) < 1e-15
        assert abs(((nodes - X) * w).sum()) < 1e-14
        assert abs(((nodes - X) ** 2 * w).sum() - (O + 1) / 12.0) < 1e-14
        assert np.count_nonzero(w > 1e-300) <= O + 1


def test_weight_support_edges(orc):
    assert orc.W(2, 1.5) == 0.0 and orc.W(3, 2.0) == 0.0
    assert orc.W(2, 0.5) == pytest.approx(0.5) and orc.W(3, 1.0) == pytest.approx(1 / 6)


STAG_E = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
STAG_B = [(0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]


def _brute_gather(F, stag, X, O, n):
    """Sum over every node of every periodic image within reach (no windowing logic)."""
    nx, ny, nz = n
    tot = 0.0
    for k in range(-6, nz + 6):
        wz = bspline_truncated_power(O + 1, k + stag[2] - X[2])
        if wz == 0:
            continue
        for j in range(-6, ny + 6):
            wy = bspline_truncated_power(O + 1, j + stag[1] - X[1])
            if wy == 0:
                continue
            for i in range(-6, nx + 6):
                wx = bspline_truncated_power(O + 1, i + stag[0] - X[0])
                if wx:
                    tot += F[k % nz, j % ny, i % nx] * wx * wy * wz
    return tot


@pytest.mark.parametrize("O", [2, 3])
@pytest.mark.parametrize("n", [(4, 4, 4), (5, 3, 1)])
def test_gather_bruteforce_random_fields(orc, O, n):
    rng = np.random.default_rng(7 + O)
    P = orc.make_params(n=n, shape_order=O)
    E = rng.normal(size=(3, n[2], n[1], n[0]))
    B = rng.normal(size=(3, n[2], n[1], n[0]))
    for _ in range(4):
        X = rng.uniform(0, 1, 3) * np.array(n)
        Ep, Bp = orc.gather(P, E, B, X)
        for c in range(3):
            assert abs(Ep[c] - _brute_gather(E[c], STAG_E[c], X, O, n)) < 1e-12
            assert abs(Bp[c] - _brute_gather(B[c], STAG_B[c], X, O, n)) < 1e-12


@pytest.mark.parametrize("O", [2, 3])
def test_gather_uniform_and_linear_fields(orc, O):
    n = (12, 12, 12)
    P = orc.make_params(n=n, shape_order=O)
    E = np.empty((3, 12, 12, 12))
    B = np.empty((3, 12, 12, 12))
    k, j, i = np.meshgrid(np.arange(12.0), np.arange(12.0), np.arange(12.0), indexing="ij")
    coef = np.array([0.3, -1.1, 0.7])
    for c in range(3):
        sE, sB = STAG_E[c], STAG_B[c]
        E[c] = 2.0 + c + coef[0] * (i + sE[0]) + coef[1] * (j + sE[1]) + coef[2] * (k + sE[2])
        B[c] = -1.0 + c + coef[0] * (i + sB[0]) + coef[1] * (j + sB[1]) + coef[2] * (k + sB[2])
    rng = np.random.default_rng(3)
    for _ in range(20):
        X = rng.uniform(4, 8, 3)  # supports stay away from the periodic seam
        Ep, Bp = orc.gather(P, E, B, X)
        lin = coef @ X
        for c in range(3):
            assert abs(Ep[c] - (2.0 + c + lin)) < 1e-12
            assert abs(Bp[c] - (-1.0 + c + lin)) < 1e-12
