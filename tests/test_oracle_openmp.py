"""CPU: the oracle's OpenMP build (one current and charge buffer per thread, loops over cells and
lines split among the threads) computes what the plain scalar build computes.

The field step, the staggered operators and the high-order line solve do the same arithmetic
per output element in both builds, so they must agree bitwise; the particle loop gives the same
positions and momenta bitwise and the same current and charge density up to the summation
order of the per-thread buffers (relative 1e-14).  This is what lets the full-size GPU tests
use the OpenMP build where the plain one would take minutes."""
import os

import numpy as np

from _state import random_state


def _both(orc, fn):
    a = fn()
    with orc.openmp():
        b = fn()
    return a, b


def test_openmp_build_uses_threads(orc):
    assert orc.num_threads() == 1
    with orc.openmp():
        assert orc.num_threads() >= 1
        if (os.cpu_count() or 1) > 1 and "OMP_NUM_THREADS" not in os.environ:
            assert orc.num_threads() > 1


def test_openmp_field_step_and_line_solve_are_bitwise_the_plain_ones(orc):
    n = (12, 10, 9)
    P = orc.make_params(n=n, field_order=6, relax_tol=1e-14, relax_max_iter=300)
    _, E, B = random_state(orc, n, 1, seed=5, e_amp=0.3, b_amp=0.4)
    rng = np.random.default_rng(6)
    J = rng.normal(0, 0.1, E.shape)

    def step():
        e, b = E.copy(), B.copy()
        it, res = orc.field_step(P, e, b, J)
        return e, b, it, res

    (e0, b0, it0, r0), (e1, b1, it1, r1) = _both(orc, step)
    assert it0 == it1 and r0 == r1 and it0 > 3
    assert np.array_equal(e0, e1) and np.array_equal(b0, b1)
    j0, j1 = _both(orc, lambda: orc.current_high_order(P, J.copy()))
    assert np.array_equal(j0, j1)
    c0, c1 = _both(orc, lambda: orc.curl_up(P, E))
    assert np.array_equal(c0, c1)


def test_openmp_particle_loop_matches_the_plain_one(orc):
    n = (10, 8, 6)
    P = orc.make_params(n=n, shape_order=3, field_order=6)
    species, E, B = random_state(orc, n, 6, seed=7, uth=0.3, e_amp=0.2, b_amp=0.5)

    def run():
        J = np.zeros_like(E)
        out = []
        for s in species:
            pos, u = s["pos"].copy(), s["u"].copy()
            flags = orc.step_species(P, s["q"], s["m"], s["w"], pos, u, E, B, J)
            out.append((pos, u, flags))
        rho = [orc.deposit_rho(P, s["q"], s["w"], s["pos"], np.zeros(E.shape[1:])) for s in species]
        return J, out, rho

    (J0, p0, r0), (J1, p1, r1) = _both(orc, run)
    for (x0, u0, f0), (x1, u1, f1) in zip(p0, p1):
        assert np.array_equal(x0, x1) and np.array_equal(u0, u1) and f0 == f1
    assert np.max(np.abs(J1 - J0)) <= 1e-14 * np.max(np.abs(J0))
    for a, b in zip(r0, r1):  # per species (the pair's sum cancels to rounding)
        assert np.max(np.abs(b - a)) <= 1e-14 * np.max(np.abs(a))


def test_a_non_finite_particle_leaves_the_others_alone(orc):
    # a particle with a non-finite momentum is flagged, left as it was and deposits nothing;
    # every particle after it is stepped as in a run without it
    n = (8, 8, 8)
    P = orc.make_params(n=n, shape_order=2, field_order=2)
    species, E, B = random_state(orc, n, 2, seed=8, uth=0.2)
    s = species[0]
    pos, u = s["pos"].copy(), s["u"].copy()
    u[:, 5] = np.nan
    J = np.zeros_like(E)
    flags = orc.step_species(P, s["q"], s["m"], s["w"], pos, u, E, B, J)
    assert flags & 2
    keep = np.ones(pos.shape[1], dtype=bool)
    keep[5] = False
    pos_ref, u_ref = s["pos"][:, keep].copy(), s["u"][:, keep].copy()
    J_ref = np.zeros_like(E)
    assert orc.step_species(P, s["q"], s["m"], s["w"], pos_ref, u_ref, E, B, J_ref) == 0
    assert np.array_equal(pos[:, keep], pos_ref) and np.array_equal(u[:, keep], u_ref)
    assert np.array_equal(pos[:, 5], s["pos"][:, 5])
    assert np.max(np.abs(J - J_ref)) <= 1e-15 * np.max(np.abs(J_ref))
