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


# ---- direct current (eq. "jj2") and the Gauss-law filter ---------------------------------------
@pytest.mark.parametrize("O", [2, 3])
def test_direct_current_moments(orc, O):
    # J_d of one particle sums to q w v_d (partition of unity of the B-splines) and its first
    # moment along every axis is q w v_d times the particle's coordinate (exact first moment;
    # the staggered component's nodes sit at i + 1/2): pins the weights and the position used
    N = (9, 8, 7)
    P = orc.make_params(n=N, shape_order=O)
    rng = np.random.default_rng(O)
    for _ in range(5):
        X = rng.uniform(3, 5, 3)
        v = rng.normal(0, 0.3, 3)
        J = orc.deposit_direct(P, -1.0, 0.5, X, v)
        for d in range(3):
            Jd = J[d]  # [z, y, x]
            assert abs(Jd.sum() - (-0.5 * v[d])) < 1e-14
            coords = [np.arange(N[a]) + (0.5 if a == d else 0.0) for a in range(3)]
            for a in range(3):
                axis = 2 - a
                other = tuple(i for i in range(3) if i != axis)
                first = (Jd.sum(axis=other) * coords[a]).sum()
                assert abs(first - (-0.5 * v[d]) * X[a]) < 1e-12


def test_direct_current_uses_the_time_centred_position(orc):
    # a lone particle moving along x: its direct current is the deposit at (X0 + X1)/2
    N = (12, 6, 6)
    P = orc.make_params(n=N, shape_order=3, current_scheme=1, dt=0.5)
    X0 = np.array([[5.3], [2.2], [3.7]])
    u = np.array([[0.6], [0.0], [0.0]])
    E = np.zeros((3, 6, 6, 12))
    J = np.zeros_like(E)
    pos, uu = X0.copy(), u.copy()
    orc.step_species(P, 1.0, 1.0, 0.25, pos, uu, E, E, J)
    g = math.sqrt(1 + 0.36)
    Xm = X0[:, 0] + np.array([0.25 * 0.6 / g, 0, 0])
    ref = orc.deposit_direct(P, 1.0, 0.25, Xm, np.array([0.6 / g, 0, 0]))
    assert np.max(np.abs(J - ref)) < 1e-15
    assert abs(pos[0, 0] - (5.3 + 0.5 * 0.6 / g)) < 1e-14


@pytest.mark.parametrize("fo", [2, 6])
def test_gauss_filter_damps_each_mode_by_its_symbol(orc, fo):
    # one pass multiplies every Fourier mode of the residual div- E - rho by 1 - kappa K^2 with
    # K_d = (2/d) sum_m a_m sin((m - 1/2) k) (closed form, Sec. III.B coefficients); the
    # correction is a gradient (curl unchanged) and the largest-K mode is removed
    rng = np.random.default_rng(fo)
    N, d = (8, 6, 10), (1.0, 0.9, 1.2)
    P = orc.make_params(n=N, d=d, field_order=fo)
    E = rng.normal(size=(3, N[2], N[1], N[0]))
    rho = rng.normal(size=(N[2], N[1], N[0]))
    rho -= rho.mean()
    r0 = orc.div_down(P, E) - rho
    E1 = orc.gauss_filter(P, E.copy(), rho, 1)
    r1 = orc.div_down(P, E1) - rho
    a = orc.fd_coeffs(fo)
    K2 = np.zeros(r0.shape)
    for dim in range(3):
        k = 2 * math.pi * np.fft.fftfreq(N[dim])
        Kd = (2 / d[dim]) * sum(a[i] * np.sin((i + 0.5) * k) for i in range(3))
        shape = [1, 1, 1]
        shape[2 - dim] = N[dim]
        K2 = K2 + (Kd ** 2).reshape(shape)
    kappa = orc.gauss_kappa(P)
    assert abs(kappa * K2.max() - 1.0) < 1e-12
    want = np.fft.ifftn(np.fft.fftn(r0) * (1 - kappa * K2)).real
    assert np.max(np.abs(r1 - want)) < 1e-11 * np.max(np.abs(r0))
    assert np.max(np.abs(orc.curl_up(P, E1) - orc.curl_up(P, E))) < 1e-12 * np.max(np.abs(E))
    # converges towards Gauss's law; no change where it already holds
    r5 = orc.div_down(P, orc.gauss_filter(P, E.copy(), rho, 5)) - rho
    assert np.max(np.abs(r5)) < np.max(np.abs(r1)) < np.max(np.abs(r0))
    E2 = orc.gauss_filter(P, E1.copy(), orc.div_down(P, E1), 3)
    assert np.max(np.abs(E2 - E1)) < 1e-13 * np.max(np.abs(E1))
