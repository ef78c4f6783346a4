"""Pins of the oracle's momentum update (paper Sec. III.A: Vay default, Boris option) against
closed-form single-particle motion: gyration in a uniform B, acceleration in a uniform E, and the
force-free E x B configuration where the Vay pusher is exact and Boris is not (the paper's reason
for preferring Vay)."""
import math

import numpy as np
import pytest

C = 1.0


@pytest.mark.parametrize("pusher", [0, 1])
def test_gyration_angle_and_speed(orc, pusher):
    q, m, dt, Bz = -1.0, 1.0, 0.4, 0.7
    u0 = np.array([0.9, 0.0, 0.25])
    g = math.sqrt(1 + u0 @ u0)
    # per step the perpendicular proper velocity rotates by 2 atan(q B dt / (2 m gamma))
    dphi = 2 * math.atan(q * Bz * dt / (2 * m * g))
    u = u0.copy()
    for n in range(1, 51):
        u = orc.push(pusher, q, m, dt, C, [0, 0, 0], [0, 0, Bz], u)
        phi = -n * dphi  # rotation sense of u x B for this sign convention
        exp = np.array([u0[0] * math.cos(phi) - u0[1] * math.sin(phi),
                        u0[0] * math.sin(phi) + u0[1] * math.cos(phi), u0[2]])
        assert np.max(np.abs(u - exp)) < 1e-13
        assert abs(math.sqrt(u @ u) - math.sqrt(u0 @ u0)) < 1e-13


@pytest.mark.parametrize("pusher", [0, 1])
def test_uniform_electric_field(orc, pusher):
    q, m, dt = 1.0, 2.0, 0.3
    E = np.array([0.2, -0.1, 0.05])
    u = np.array([0.01, 0.3, -0.2])
    u0 = u.copy()
    for n in range(1, 40):
        u = orc.push(pusher, q, m, dt, C, E, [0, 0, 0], u)
        assert np.max(np.abs(u - (u0 + n * q * E * dt / m))) < 1e-13


def test_force_free_vay_exact_boris_drifts(orc):
    # E + v x B = 0 with v = 0.99 c: the particle must keep its velocity
    v = 0.99
    g = 1 / math.sqrt(1 - v * v)
    B = np.array([0.0, 0.0, 1.3])
    vel = np.array([v, 0.0, 0.0])
    E = -np.cross(vel, B)
    uv = g * vel
    ub = g * vel
    for _ in range(100):
        uv = orc.push(0, -1.0, 1.0, 0.4, C, E, B, uv)
        ub = orc.push(1, -1.0, 1.0, 0.4, C, E, B, ub)
    assert np.max(np.abs(uv - g * vel)) / g < 1e-13
    assert np.max(np.abs(ub - g * vel)) / g > 1e-4  # Boris is not force-free exact


def test_exb_drift_velocity(orc):
    # weak E perpendicular to strong B: guiding centre drifts at E x B / B^2
    q, m, dt = 1.0, 1.0, 0.05
    B = np.array([0.0, 0.0, 2.0])
    E = np.array([0.02, 0.0, 0.0])
    vd = np.cross(E, B) / (B @ B)
    u = np.zeros(3)
    x = np.zeros(3)
    Tc = 2 * math.pi * m / (q * 2.0)
    nsteps = int(round(20 * Tc / dt))
    xs = []
    for _ in range(nsteps):
        u = orc.push(0, q, m, dt, C, E, B, u)
        gam = math.sqrt(1 + u @ u)
        x = x + dt * u / gam
        xs.append(x.copy())
    xs = np.array(xs)
    t = dt * np.arange(1, nsteps + 1)
    slope = np.polyfit(t, xs[:, 1], 1)[0]
    assert abs(slope - vd[1]) < 0.02 * abs(vd[1])


# ---- radiative cooling (Sec. "Radiative cooling") ----------------------------------------------
@pytest.mark.parametrize("c", [1.0, 2.0])
def test_rad_bracket_equals_the_three_velocity_larmor_form(orc, c):
    # eq. "prad" (proper velocities) against eq. "pradv" (three-velocities):
    # |du/dt|^2 + |du/dt x u|^2/c^2 = gamma^4 |dv/dt|^2 + gamma^6 (dv/dt . v)^2 / c^2
    rng = np.random.default_rng(5)
    for _ in range(20):
        u = rng.normal(0, 3, 3)
        ud = rng.normal(0, 2, 3)
        g = math.sqrt(1 + u @ u / c ** 2)
        gd = (u @ ud) / (g * c * c)
        v = u / g
        vd = ud / g - u * gd / g ** 2
        p_three = g ** 4 * (vd @ vd) + g ** 6 * (vd @ v) ** 2 / c ** 2
        assert abs(orc.rad_bracket(c, u, ud) / p_three - 1) < 1e-12


def test_rad_cooling_off_is_the_plain_push(orc):
    rng = np.random.default_rng(6)
    for pusher in (0, 1):
        E, B, u = rng.normal(0, 1, 3), rng.normal(0, 2, 3), rng.normal(0, 3, 3)
        a = orc.push(pusher, -1.0, 1.0, 0.3, 1.0, E, B, u)
        b = orc.push_rad(pusher, -1.0, 1.0, 0.3, 1.0, 0.0, E, B, u)
        assert np.array_equal(a, b)


def test_rad_cooling_acts_against_the_time_centred_velocity(orc):
    rng = np.random.default_rng(7)
    for pusher in (0, 1):
        E, B, u = rng.normal(0, 1, 3), rng.normal(0, 2, 3), rng.normal(0, 3, 3)
        uem = orc.push(pusher, 1.0, 2.0, 0.2, 1.0, E, B, u)
        urad = orc.push_rad(pusher, 1.0, 2.0, 0.2, 1.0, 1e-3, E, B, u)
        du, u0 = urad - uem, 0.5 * (uem + u)
        assert du @ u0 < 0
        assert np.linalg.norm(np.cross(du, u0)) < 1e-12 * np.linalg.norm(du) * np.linalg.norm(u0)
        # size: k gamma0 |bracket| dt / |u0| with k = rad_tau q^2 / m
        ud = (uem - u) / 0.2
        g0 = math.sqrt(1 + u0 @ u0)
        expect = 1e-3 * 1.0 / 2.0 * g0 * orc.rad_bracket(1.0, u0, ud) * 0.2 / math.sqrt(u0 @ u0)
        assert abs(np.linalg.norm(du) / expect - 1) < 1e-12


@pytest.mark.parametrize("pusher", [0, 1])
def test_synchrotron_cooling_in_a_uniform_field(orc, pusher):
    # u perpendicular to a uniform B: d|u|/dt = -k w_c^2 |u| sqrt(1 + u^2/c^2) (k = rad_tau q^2/m,
    # w_c = |q| B / m), so asinh(c/|u|) grows at the constant rate k w_c^2; the explicit scheme
    # follows it to first order in the step
    q, m, B0, tau, x0, T = -1.0, 1.0, 1.0, 0.01, 10.0, 20.0
    k, wc = tau * q * q / m, abs(q) * B0 / m
    exact = 1.0 / math.sinh(math.asinh(1.0 / x0) + k * wc * wc * T)
    errs = []
    for dt in (0.02, 0.01):
        u = np.array([x0, 0.0, 0.0])
        for _ in range(int(round(T / dt))):
            u = orc.push_rad(pusher, q, m, dt, 1.0, tau, np.zeros(3), np.array([0.0, 0.0, B0]), u)
        assert abs(u[2]) < 1e-14  # stays in the plane
        errs.append(abs(np.linalg.norm(u) / exact - 1))
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 1.8


# ---- fourth-order time integration (Sec. III.A, symmetric composition) ------------------------
def _gyro(t, B0=1.0, um=1.0, x0=8.0, y0=8.0, z0=8.0, phi0=0.3):
    # electron (q = -1, m = 1) in B0 z: u turns at w = B0/gamma, radius |u|/B0
    g = math.sqrt(1 + um * um)
    w = B0 / g
    ph = phi0 + w * t
    u = np.array([um * math.cos(ph), um * math.sin(ph), 0.0])
    r = um / B0
    x = np.array([x0 + r * math.sin(ph), y0 - r * math.cos(ph), z0])
    return x, u


def _gyro_error(orc, h, order, T=4.0):
    # leapfrog: x at t, u at t - h/2.  Composition: the state's positions are a drift of
    # theta h / 2 (at the momentum's velocity) ahead of the momenta, x + (theta h/2) v
    th = orc.FR_THETA
    if order == 4:
        x, u = _gyro(0.0)
        x = x + 0.5 * th * h * u / math.sqrt(1 + u @ u)
    else:
        x, _ = _gyro(0.0)
        _, u = _gyro(-h / 2)
    n = (16, 16, 16)
    P = orc.make_params(n=n, dt=h, shape_order=3, field_order=2, time_order=order, relax_tol=1e-15,
                        relax_max_iter=400)
    B = np.zeros((3, 16, 16, 16))
    B[2] = 1.0
    run = orc.Run(P, [dict(q=-1.0, m=1.0, w=1e-15, pos=x.reshape(3, 1), u=u.reshape(3, 1))], B=B)
    steps = int(round(T / h))
    for _ in range(steps):
        run.step()
    xg, ug = run.species[0]["pos"][:, 0], run.species[0]["u"][:, 0]
    if order == 4:
        xg = xg - 0.5 * th * h * ug / math.sqrt(1 + ug @ ug)
        xe, ue = _gyro(T)
    else:
        xe, _ = _gyro(T)
        _, ue = _gyro(T - h / 2)
    return max(np.max(np.abs(xg - xe)), np.max(np.abs(ug - ue)))


def test_fourth_order_composition_converges_at_fourth_order(orc):
    # a test particle gyrating in a uniform B through whole runs (fields advanced every
    # substep): the leapfrog error falls 4x per halving of the step, the composition's 16x
    th = orc.FR_THETA
    assert abs(sum(k for k, _ in orc.FR_SUBSTEPS) - 1) < 1e-15 and abs(sum(d for _, d in orc.FR_SUBSTEPS) - 1) < 1e-15
    assert abs(2 * th ** 3 + (1 - 2 * th) ** 3) < 1e-14  # the third-order condition of the triple jump
    e2 = [_gyro_error(orc, h, 2) for h in (0.2, 0.1)]
    e4 = [_gyro_error(orc, h, 4) for h in (0.2, 0.1)]
    assert 3.5 < e2[0] / e2[1] < 4.5, e2
    assert 14 < e4[0] / e4[1] < 18, e4
    assert e4[1] < e2[1] / 50
