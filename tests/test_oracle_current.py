"""Pins of the oracle's charge-conserving current (paper Sec. III.C: eqs. "cc1", "jj3", "jj6d",
"penta").  Pins: the discrete continuity equation with the oracle's independent charge deposit
(eq. "rho2"), the total current of a moving charge, the unique 1D charge-conserving current, the
high-order line solve's defining property (high-order divergence of J_O equals the second-order
divergence of J_2) and its closed-form action on a Fourier mode."""
import math

import numpy as np
import pytest


def _rand_moves(rng, n, N, maxd=0.95):
    X0 = rng.uniform(0, 1, (n, 3)) * np.array(N)
    d = rng.uniform(-maxd, maxd, (n, 3)) * rng.uniform(0, 1, (n, 1))
    return X0, X0 + d


def _rho(orc, P, q, w, X):
    pos = np.ascontiguousarray(np.array(X, dtype=np.float64).reshape(-1, 3).T)
    return orc.deposit_rho(P, q, w, pos)


@pytest.mark.parametrize("O", [2, 3])
@pytest.mark.parametrize("N", [(6, 5, 4), (8, 3, 1)])
def test_continuity_each_particle(orc, O, N):
    rng = np.random.default_rng(11 + O)
    P = orc.make_params(n=N, d=(0.7, 1.1, 0.9), dt=0.3, shape_order=O, field_order=2)
    q, w = -1.3, 0.25
    X0s, X1s = _rand_moves(rng, 12, N)
    for X0, X1 in zip(X0s, X1s):
        J = orc.deposit_current(P, q, w, X0, X1)
        r0 = _rho(orc, P, q, w, X0 % np.array(N))
        r1 = _rho(orc, P, q, w, X1 % np.array(N))
        resid = (r1 - r0) / P.dt + orc.div_down(P, J)
        assert np.max(np.abs(resid)) < 1e-13 * max(1.0, abs(q * w) / P.dt)


@pytest.mark.parametrize("O", [2, 3])
def test_total_current_is_charge_times_velocity(orc, O):
    rng = np.random.default_rng(5)
    N = (7, 6, 5)
    dx = (0.5, 1.0, 2.0)
    P = orc.make_params(n=N, d=dx, dt=0.25, shape_order=O)
    q, w = 1.0, 0.125
    for X0, X1 in zip(*_rand_moves(rng, 8, N)):
        J = orc.deposit_current(P, q, w, X0, X1)
        for c in range(3):
            # integral of J_c over the box / cell volume = q w (displacement along c) dx_c / dt
            assert abs(J[c].sum() - q * w * (X1[c] - X0[c]) * dx[c] / P.dt) < 1e-13


@pytest.mark.parametrize("O", [2, 3])
def test_motion_along_one_axis_is_one_dimensional(orc, O):
    # moving along x only: J_y = J_z = 0 and J_x(i+1/2,j,k) = J_1D(i+1/2) S(j-Y) S(k-Z),
    # where the 1D charge-conserving current is unique: J_1D(i+1/2) - J_1D(i-1/2) = -(qw dx/dt) dS(i)
    N = (10, 6, 6)
    P = orc.make_params(n=N, dt=0.5, shape_order=O)
    q, w = -1.0, 0.5
    X0 = np.array([4.3, 2.7, 3.1])
    X1 = X0 + np.array([0.61, 0.0, 0.0])
    J = orc.deposit_current(P, q, w, X0, X1)
    assert np.max(np.abs(J[1])) == 0.0 and np.max(np.abs(J[2])) < 1e-300 + 0.0
    dS = np.array([orc.W(O, i - X1[0]) - orc.W(O, i - X0[0]) for i in range(N[0])])
    J1 = -(q * w * 1.0 / P.dt) * np.cumsum(dS)
    Sy = np.array([orc.W(O, j - X0[1]) for j in range(N[1])])
    Sz = np.array([orc.W(O, k - X0[2]) for k in range(N[2])])
    expect = Sz[:, None, None] * Sy[None, :, None] * J1[None, None, :]
    assert np.max(np.abs(J[0] - expect)) < 1e-15


@pytest.mark.parametrize("O", [2, 3])
def test_no_motion_no_current(orc, O):
    P = orc.make_params(n=(5, 5, 5), shape_order=O)
    X = np.array([1.2, 3.4, 0.3])
    J = orc.deposit_current(P, 1.0, 1.0, X, X)
    assert np.max(np.abs(J)) == 0.0


# ---------------------------------------------------------------- high-order current (order 4, 6)
def _divergence_orders(orc, P, J):
    P2 = orc.make_params(n=tuple(P.n), d=tuple(P.d), field_order=2)
    return orc.div_down(P2, J)


@pytest.mark.parametrize("fo", [4, 6])
@pytest.mark.parametrize("N", [(16, 8, 6), (9, 4, 1), (3, 2, 5)])
def test_high_order_current_reproduces_charge_change(orc, fo, N):
    rng = np.random.default_rng(21)
    P = orc.make_params(n=N, d=(0.3, 0.7, 1.0), dt=0.1, shape_order=3, field_order=fo)
    J2 = np.zeros((3, N[2], N[1], N[0]))
    for X0, X1 in zip(*_rand_moves(rng, 20, N)):
        orc.deposit_current(P, rng.choice([-1.0, 1.0]), 0.3, X0, X1, J2)
    JO = orc.current_high_order(P, J2.copy())
    lhs = orc.div_down(P, JO)  # order fo
    rhs = _divergence_orders(orc, P, J2)  # order 2
    scale = np.max(np.abs(rhs))
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * scale
    # line means preserved (component c along its own axis c)
    for c in range(3):
        ax = 2 - c  # array axis of dimension c in [z, y, x] order
        assert np.max(np.abs(JO[c].mean(axis=ax) - J2[c].mean(axis=ax))) < 1e-14 * np.max(np.abs(J2))


def test_high_order_current_order2_is_identity(orc):
    P = orc.make_params(n=(6, 6, 6), field_order=2)
    J = np.random.default_rng(0).normal(size=(3, 6, 6, 6))
    assert np.array_equal(orc.current_high_order(P, J.copy()), J)


@pytest.mark.parametrize("fo", [4, 6])
def test_high_order_current_fourier_mode(orc, fo):
    # on a single mode exp(i k x) the line operator T (stencil sum_m a_m over |l| < m) has
    # symbol T(k) = sum_l T_l cos(l k); J_O = J_2 / T(k) exactly
    N = 24
    P = orc.make_params(n=(N, 1, 1), field_order=fo)
    a = {4: [9 / 8, -1 / 24], 6: [75 / 64, -25 / 384, 3 / 640]}[fo]
    M = len(a)
    for m in (1, 5, 12):
        k = 2 * math.pi * m / N
        x = np.arange(N) + 0.5
        J = np.zeros((3, 1, 1, N))
        J[0, 0, 0] = np.cos(k * x + 0.3)
        Tk = sum(sum(a[mm - 1] for mm in range(abs(l) + 1, M + 1)) * math.cos(l * k) for l in range(-(M - 1), M))
        JO = orc.current_high_order(P, J.copy())
        assert np.max(np.abs(JO[0, 0, 0] - J[0, 0, 0] / Tk)) < 1e-14
