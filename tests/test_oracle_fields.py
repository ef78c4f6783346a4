"""Pins of the oracle's staggered difference operators and implicit field step (paper Sec.
III.B: eqs. "bnplus1", "enplus1", "EllipticB", the 6th-order "ddyup" coefficients).

Pins: consistency and convergence order of the operators on smooth periodic data; the discrete
identities div curl = 0 and curl curl = grad div - lap; the defining update pair "bnplus1" /
"enplus1" (which the derived elliptic form must satisfy; it exposes the sign of the J term);
the closed-form amplification of a vacuum wave; an exact FFT solve of the elliptic equation;
and preservation of div B."""
import math

import numpy as np
import pytest

STAG_E = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
STAG_B = [(0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]


def test_sixth_order_coefficients_are_a_first_derivative(orc):
    a, b, c = orc.fd_coeffs(6)
    assert abs(a + 3 * b + 5 * c - 1.0) < 1e-15  # exact for linear functions
    assert abs(a + 27 * b + 125 * c) < 1e-15  # third-moment (Taylor) condition
    assert abs(a + 243 * b + 3125 * c) < 1e-13  # fifth-moment condition
    a4, b4, _ = orc.fd_coeffs(4)
    assert abs(a4 + 3 * b4 - 1.0) < 1e-15 and abs(a4 + 27 * b4) < 1e-15
    # the printed 25/21 is not consistent
    assert abs(25 / 21 + 3 * b + 5 * c - 1.0) > 1e-2


@pytest.mark.parametrize("fo", [2, 4, 6])
@pytest.mark.parametrize("up", [True, False])
def test_derivative_convergence_order(orc, fo, up):
    errs = []
    for N in (16, 32):
        h = 1.0 / N
        P = orc.make_params(n=(N, 1, 1), d=(h, 1, 1), field_order=fo)
        # input lives on integer nodes for the up operator, on half nodes for the down operator
        xin = np.arange(N) * h + (0.0 if up else 0.5 * h)
        xout = np.arange(N) * h + (0.5 * h if up else 0.0)
        f = np.sin(2 * math.pi * xin)[None, None, :].copy()
        d = orc.deriv(P, f, 0, up)
        errs.append(np.max(np.abs(d[0, 0] - 2 * math.pi * np.cos(2 * math.pi * xout))))
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - fo) < 0.15, (errs, rate)


@pytest.mark.parametrize("fo", [2, 4, 6])
def test_discrete_vector_identities(orc, fo):
    rng = np.random.default_rng(2)
    N = (9, 7, 6)
    P = orc.make_params(n=N, d=(0.5, 1.0, 1.5), field_order=fo)
    A = rng.normal(size=(3, N[2], N[1], N[0]))
    # div+ (curl+ A) = 0 and div- (curl- B) = 0
    assert np.max(np.abs(orc.div_up(P, orc.curl_up(P, A)))) < 1e-12
    assert np.max(np.abs(orc.div_down(P, orc.curl_down(P, A)))) < 1e-12
    # for divergence-free B (= curl+ of something), curl+ curl- B = -lap B
    B = orc.curl_up(P, A)
    lhs = orc.curl_up(P, orc.curl_down(P, B))
    assert np.max(np.abs(lhs + orc.laplacian_B(P, B))) < 1e-11 * np.max(np.abs(lhs))


def _random_state(orc, P, rng):
    N = tuple(P.n)
    shape = (3, N[2], N[1], N[0])
    E = rng.normal(size=shape)
    B = orc.curl_up(P, rng.normal(size=shape))  # divergence free
    J = rng.normal(size=shape)
    return E, B, J


@pytest.mark.parametrize("fo", [2, 4, 6])
@pytest.mark.parametrize("alpha", [0.5, 0.55, 0.9])
def test_field_step_satisfies_update_pair(orc, fo, alpha):
    rng = np.random.default_rng(3)
    P = orc.make_params(n=(8, 6, 5), d=(1.0, 0.8, 1.2), dt=0.3, field_order=fo, alpha=alpha,
                        relax_tol=1e-15, relax_max_iter=500)
    E0, B0, J = _random_state(orc, P, rng)
    E, B = E0.copy(), B0.copy()
    it, res = orc.field_step(P, E, B, J)
    assert res < 1e-14 and it < 500
    beta = 1 - alpha
    # eq. bnplus1
    r1 = (B - B0) / P.dt + orc.curl_up(P, alpha * E + beta * E0)
    # eq. enplus1 (c = eps0 = mu0 = 1)
    r2 = (E - E0) / P.dt - (orc.curl_down(P, alpha * B + beta * B0) - J)
    assert np.max(np.abs(r1)) < 1e-12 * np.max(np.abs(orc.curl_up(P, E0)))
    assert np.max(np.abs(r2)) < 1e-12 * np.max(np.abs(J))
    # div B preserved
    assert np.max(np.abs(orc.div_up(P, B))) < 1e-12


def test_field_step_printed_minus_sign_fails_update_pair(orc):
    # The printed elliptic form has "- alpha mu0 c^2 dt^2 curl J"; flipping the sign of J in the
    # oracle's right-hand side (equivalently stepping with -J and comparing with +J) breaks eq.
    # bnplus1 by O(1), which confirms the reading "+".
    rng = np.random.default_rng(4)
    P = orc.make_params(n=(8, 6, 5), dt=0.3, field_order=2, alpha=0.55)
    E0, B0, J = _random_state(orc, P, rng)
    E, B = E0.copy(), B0.copy()
    # stepping with the J term reversed and E update kept correct:
    orc.field_step(P, E, B, -J)
    Ec = E0 + P.dt * (orc.curl_down(P, 0.55 * B + 0.45 * B0) - J)
    r1 = (B - B0) / P.dt + orc.curl_up(P, 0.55 * Ec + 0.45 * E0)
    assert np.max(np.abs(r1)) > 1e-2


@pytest.mark.parametrize("fo", [2, 6])
@pytest.mark.parametrize("alpha", [0.5, 0.55])
def test_vacuum_wave_amplification(orc, fo, alpha):
    # 1D vacuum wave E_y, B_z along x.  For a mode exp(ikx), every staggered derivative acts
    # as i K(k) with K = (2/dx) sum_m a_m sin((m - 1/2) k dx); one step multiplies the
    # right-moving eigenmode (E_y = c B_z) by lambda = (1 - i th beta)/(1 + i th alpha),
    # th = c dt K.  |lambda| = 1 at alpha = 1/2.
    N, dx, dt = 32, 1.0, 0.4
    P = orc.make_params(n=(N, 1, 1), d=(dx, 1, 1), dt=dt, field_order=fo, alpha=alpha,
                        relax_tol=1e-15, relax_max_iter=400)
    a = orc.fd_coeffs(fo)
    for m in (1, 7, 16):
        k = 2 * math.pi * m / (N * dx)
        K = (2 / dx) * sum(a[i] * math.sin((i + 0.5) * k * dx) for i in range(3))
        th = dt * K
        lam = (1 - 1j * th * (1 - alpha)) / (1 + 1j * th * alpha)
        xE = np.arange(N) * dx  # E_y at integer x
        xB = (np.arange(N) + 0.5) * dx  # B_z at half x
        E = np.zeros((3, 1, 1, N))
        B = np.zeros((3, 1, 1, N))
        E[1, 0, 0] = np.cos(k * xE)
        B[2, 0, 0] = np.cos(k * xB)
        J = np.zeros_like(E)
        orc.field_step(P, E, B, J)
        assert np.max(np.abs(E[1, 0, 0] - np.real(lam * np.exp(1j * k * xE)))) < 1e-12
        assert np.max(np.abs(B[2, 0, 0] - np.real(lam * np.exp(1j * k * xB)))) < 1e-12
    if fo == 2 and alpha == 0.55:
        th = dt * 2.0 / dx  # Nyquist
        assert abs(abs((1 - 1j * th * 0.45) / (1 + 1j * th * 0.55)) - 0.972821) < 1e-6


def test_field_step_matches_fft_solve(orc):
    # (1 - alpha^2 c^2 dt^2 lap) B' = rhs solved exactly with FFTs on an 8^3 periodic grid;
    # lap along d has symbol -K_d(k)^2 for every component, K_d as above.
    rng = np.random.default_rng(9)
    N = (8, 8, 8)
    d = (1.0, 0.9, 1.1)
    al, dt = 0.55, 0.35
    P = orc.make_params(n=N, d=d, dt=dt, field_order=6, alpha=al, relax_tol=1e-15, relax_max_iter=500)
    E0, B0, J = _random_state(orc, P, rng)
    E, B = E0.copy(), B0.copy()
    orc.field_step(P, E, B, J)
    a = orc.fd_coeffs(6)
    Ks = []
    for dim in range(3):
        k = 2 * math.pi * np.fft.fftfreq(N[dim])
        Ks.append((2 / d[dim]) * sum(a[i] * np.sin((i + 0.5) * k) for i in range(3)))
    K2 = Ks[2][:, None, None] ** 2 + Ks[1][None, :, None] ** 2 + Ks[0][None, None, :] ** 2
    s = dt * dt
    lapB0 = orc.laplacian_B(P, B0)
    rhs = B0 + al * (1 - al) * s * lapB0 - dt * orc.curl_up(P, E0) + al * dt * dt * orc.curl_up(P, J)
    Bx = np.real(np.fft.ifftn(np.fft.fftn(rhs, axes=(1, 2, 3)) / (1 + al * al * s * K2)[None], axes=(1, 2, 3)))
    assert np.max(np.abs(B - Bx)) < 1e-12 * np.max(np.abs(Bx))


@pytest.mark.parametrize("fo", [2, 6])
def test_poisson_helper_inverts_the_down_divergence(orc, fo):
    # the test helper that builds an E field with a given down divergence: div_down E equals
    # rho minus its mean, and its stencil symbol is minus the sum of K_d^2 (closed form above)
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from _state import poisson_E
    rng = np.random.default_rng(11)
    N = (10, 6, 8)
    d = (1.0, 0.8, 1.2)
    P = orc.make_params(n=N, d=d, field_order=fo)
    rho = rng.normal(size=(N[2], N[1], N[0]))
    E = poisson_E(orc, P, rho)
    assert np.max(np.abs(orc.div_down(P, E) - (rho - rho.mean()))) < 1e-12 * np.max(np.abs(rho))
    a = orc.fd_coeffs(fo)
    delta = np.zeros((N[2], N[1], N[0]))
    delta[0, 0, 0] = 1.0
    for dim in range(3):
        k = 2 * math.pi * np.fft.fftfreq(N[dim])
        K = (2 / d[dim]) * sum(a[i] * np.sin((i + 0.5) * k) for i in range(3))
        sym = np.fft.fftn(orc.deriv(P, orc.deriv(P, delta, dim, True), dim, False))
        line = sym[(0,) * (2 - dim) + (slice(None),) + (0,) * dim]
        assert np.max(np.abs(line - (-K * K))) < 1e-12
