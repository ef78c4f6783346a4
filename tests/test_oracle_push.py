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
