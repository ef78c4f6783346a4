"""Whole-run pins of the oracle: invariants the paper states for the complete step (Gauss's law
kept by the charge-conserving current, Sec. III.C and its closing remarks on FP64 runs; div B kept by
the staggered curl, Sec. III.B), diagnostics against closed forms, the loaders' properties, and
the linear growth rate of the symmetric relativistic two-stream instability."""
import math

import numpy as np
import pytest

from paper_1211_4575_amd import inputs as I


def _wl_params(orc, wl, **over):
    return orc.make_params(**wl.params(**over))


def _species(wl):
    return [dict(q=s.q, m=s.m, w=s.w, pos=s.pos, u=s.u) for s in wl.species]


@pytest.mark.parametrize("O,fo", [(2, 2), (3, 6), (3, 4)])
def test_gauss_and_continuity_hold_every_step(orc, O, fo):
    wl = I.plain_heating(n=(8, 6, 5), ppc=4, uth=0.3, shape_order=O, field_order=fo)
    P = _wl_params(orc, wl)
    run = orc.Run(P, _species(wl))
    rho_prev = run.rho()
    assert np.max(np.abs(rho_prev)) < 1e-14  # pair loading: no net charge
    for step in range(8):
        run.step()
        rho = run.rho()
        cc = (rho - rho_prev) / P.dt + orc.div_down(P, run.J)
        assert np.max(np.abs(cc)) < 1e-12, step
        gauss = orc.div_down(P, run.E) - rho / P.eps0
        assert np.max(np.abs(gauss)) < 1e-12, step
        assert np.max(np.abs(orc.div_up(P, run.B))) < 1e-12
        assert run.flags == 0
        rho_prev = rho


def test_gauss_with_background_and_lattice(orc):
    # quiet lattice electrons over a uniform ion background: rho = 0 exactly at t = 0
    wl = I.two_stream(n=(8, 4, 4), per_dim=(2, 2, 2), dx=0.1)
    P = _wl_params(orc, wl)
    run = orc.Run(P, _species(wl))
    assert np.max(np.abs(run.rho())) < 1e-12
    for _ in range(5):
        run.step()
    gauss = orc.div_down(P, run.E) - run.rho()
    assert np.max(np.abs(gauss)) < 1e-11


def test_species_moments_closed_form(orc):
    P = orc.make_params(n=(2, 2, 2), d=(0.5, 1.0, 2.0))
    u = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 1e-9]])
    K, mom = orc.species_moments(P, 2.0, 0.25, u)
    V = 1.0
    exp_K = 0.25 * V * 2.0 * ((math.sqrt(26.0) - 1.0) + (math.sqrt(1 + 1e-18) - 1.0))
    assert abs(K - exp_K) < 1e-14
    assert np.allclose(mom, 0.25 * V * 2.0 * u.sum(axis=1), rtol=0, atol=1e-15)


def test_field_energy_closed_form(orc):
    P = orc.make_params(n=(4, 3, 2), d=(1.0, 2.0, 0.5))
    E = np.ones((3, 2, 3, 4)) * np.array([1.0, 2.0, 3.0])[:, None, None, None]
    B = np.ones((3, 2, 3, 4)) * 0.5
    UE, UB, UEx = orc.field_energy(P, E, B)
    V = 1.0 * 2.0 * 0.5
    assert abs(UE - 0.5 * 24 * V * 14.0) < 1e-12
    assert abs(UB - 0.5 * 24 * V * 0.75) < 1e-12
    assert abs(UEx - 0.5 * 24 * V * 1.0) < 1e-12


def test_lattice_load_deposits_uniform_density(orc):
    # sum of integer shifts of a B-spline is one => a lattice with k particles per cell per
    # dimension deposits exactly k^3 * w q everywhere, for every weight order
    for O in (1, 2, 3):
        P = orc.make_params(n=(6, 4, 3), shape_order=O)
        pos = I.lattice_positions((6, 4, 3), (2, 3, 1))
        rho = orc.deposit_rho(P, -1.0, 1.0 / 6.0, pos)
        assert np.max(np.abs(rho + 1.0)) < 1e-14


def test_maxwell_juttner_mean_gamma():
    # <gamma> = 3 theta + K1(1/theta)/K2(1/theta) = 3.370441 at theta = 1
    from scipy.special import kv
    idx = np.arange(200000, dtype=np.uint64)
    mag = I.maxwell_juttner_speed(7, 99, idx, 1.0)
    g = np.sqrt(1 + mag * mag)
    exact = 3.0 + kv(1, 1.0) / kv(2, 1.0)
    assert abs(exact - 3.370441) < 1e-6
    assert abs(g.mean() - exact) < 3 * g.std() / math.sqrt(g.size)


def test_philox_known_answers():
    # Known-answer vectors of Philox-4x32-10 (Random123 distribution)
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, exp in cases:
        assert tuple(int(x) for x in I.philox4x32(*ctr, *key)) == exp


@pytest.mark.parametrize("origin", ["nearest", "floor"])
def test_split_roundtrip(origin):
    rng = np.random.default_rng(0)
    n = (16, 8, 4)
    pos = rng.uniform(0, 1, (3, 1000)) * np.array(n)[:, None]
    pos[:, 0] = [15.9999999999, 7.5, 3.5]
    pos[:, 1] = [2.9999999999, 0.4999999999, 0.0]
    cell, off = I.to_split(pos, n, origin=origin)
    lo = -0.5 if origin == "nearest" else 0.0
    assert off.dtype == np.float32 and np.all(off >= lo) and np.all(off < lo + 1.0)
    ijk = np.stack([cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])])
    base = np.floor(pos + 0.5) if origin == "nearest" else np.floor(pos)
    moved = (ijk - base.astype(np.int64)) % np.array(n)[:, None]
    assert np.all((moved == 0) | (moved == 1))  # the cell, or the next one after rounding up
    back = I.from_split(cell, off, n)
    dist = np.abs(back - pos)
    dist = np.minimum(dist, np.array(n)[:, None] - dist)
    assert np.max(dist) < 1e-7


def _two_stream_rate(k, v0, wb2):
    """Largest growth rate at wavenumber k of the symmetric cold relativistic two-stream
    (each beam plasma frequency^2 = wb2, longitudinal mass gamma^3 m): roots of
    1 = wb2/g3 [1/(w - k v0)^2 + 1/(w + k v0)^2]."""
    g3 = (1.0 / math.sqrt(1 - v0 * v0)) ** 3
    a = k * v0
    wp = wb2 / g3
    # (w^2 - a^2)^2 = wp [(w + a)^2 + (w - a)^2] = 2 wp (w^2 + a^2); quadratic in W = w^2
    # W^2 - (2 a^2 + 2 wp) W + a^4 - 2 wp a^2 = 0
    bq = -(2 * a * a + 2 * wp)
    cq = a ** 4 - 2 * wp * a * a
    Wm = (-bq - math.sqrt(bq * bq - 4 * cq)) / 2, (-bq + math.sqrt(bq * bq - 4 * cq)) / 2
    return max(math.sqrt(-W) if W < 0 else 0.0 for W in Wm)


def test_two_stream_theory_numbers():
    # maximum over k: omega_b gamma0^(-3/2) / 2 with omega_b^2 = 1/2 -> 0.342893
    g0 = 1 / math.sqrt(1 - 0.04)
    assert abs(math.sqrt(0.5) * g0 ** -1.5 / 2 - 0.342893) < 1e-6
    ks = np.linspace(0.5, 4.5, 4001)
    best = max(_two_stream_rate(k, 0.2, 0.5) for k in ks)
    assert abs(best - 0.342893) < 1e-5


@pytest.mark.slow
def test_two_stream_growth_rate_oracle(orc):
    # Quasi-1D box 6.4 c/w_pe long (64 cells of 0.1, cubic weights, 6th-order fields), beams at
    # +-0.2c.  The growing eigenmode of linear theory at k = 2 pi 3 / 6.4 is seeded (beam
    # displacement xi_s and velocity dv_s with (p + i k v_s) dv_s = q E / (m gamma0^3),
    # xi_s = dv_s / (p + i k v_s), E = eps cos(k x)); the E_x energy then grows as exp(2 p t).
    n, dx = (64, 1, 1), 0.1
    wl = I.two_stream(n=n, per_dim=(32, 1, 1), dx=dx, v_beam=0.2, uth=0.0)
    k = 2 * math.pi * 3 / (n[0] * dx)
    p = _two_stream_rate(k, 0.2, 0.5)
    g0 = 1 / math.sqrt(1 - 0.04)
    eps = 1e-4
    for s, vs in zip(wl.species, (0.2, -0.2)):
        ph = np.exp(1j * k * s.pos[0] * dx)
        dv = s.q * eps / (s.m * g0 ** 3 * (p + 1j * k * vs))
        xi = dv / (p + 1j * k * vs)
        s.pos[0] = np.mod(s.pos[0] + np.real(xi * ph) / dx, n[0])
        s.u[0] += g0 ** 3 * np.real(dv * ph)
    P = _wl_params(orc, wl)
    E0 = np.zeros((3, 1, 1, n[0]))
    E0[0, 0, 0] = eps * np.cos(k * (np.arange(n[0]) + 0.5) * dx)
    run = orc.Run(P, _species(wl), E=E0)
    hist = [orc.field_energy(P, run.E, run.B)[2]]
    for _ in range(200):
        run.step()
        hist.append(orc.field_energy(P, run.E, run.B)[2])
    W = np.array(hist)
    t = P.dt * np.arange(W.size)
    rate = np.polyfit(t, np.log(W), 1)[0] / 2
    assert abs(rate - p) < 0.03 * p, (rate, p)


def test_mmi_loader_is_neutral_and_boosted():
    # the mixed-mode two-stream set-up: each population's electrons and ions share positions
    # (no charge, no current at t = 0 for equal drifts), the beam's mean four-velocity along z
    # is the boost of a thermal population, and the growth rates reproduce the paper's values
    from paper_1211_4575_amd import inputs as I
    wl = I.mmi(n=(6, 5, 4), ppc=40)
    e_b, i_b, e_p, i_p = wl.species
    assert np.array_equal(e_b.pos, i_b.pos) and np.array_equal(e_p.pos, i_p.pos)
    assert not np.array_equal(e_b.pos, e_p.pos)
    assert e_b.w * e_b.pos.shape[1] / (6 * 5 * 4) == pytest.approx(0.1)
    assert e_p.w * e_p.pos.shape[1] / (6 * 5 * 4) == pytest.approx(0.9)
    # cold beam: gamma close to 4, all moving along +z
    g = np.sqrt(1.0 + (e_b.u ** 2).sum(axis=0))
    assert abs(np.mean(g) - 4.0) < 0.1 and np.all(e_b.u[2] > 0)
    gi = np.sqrt(1.0 + (i_b.u ** 2).sum(axis=0))
    assert abs(np.mean(gi) - 4.0) < 1e-3 and np.max(np.abs(gi - 4.0)) < 0.1  # G beta u_z' spread
    # rest-frame boost: the boosted four-velocity has u_z = G (u_z' + beta gamma')
    up = np.array([[0.1], [0.2], [0.3]])
    b = I.boost_z(up, 4.0)
    beta = np.sqrt(1 - 1 / 16.0)
    assert b[2, 0] == pytest.approx(4.0 * (0.3 + beta * np.sqrt(1.14)))
    assert np.sqrt(1 + (b ** 2).sum()) == pytest.approx(4.0 * (np.sqrt(1.14) + beta * 0.3))
    r = I.mmi_rates()
    assert round(r["mmi"], 3) == 0.201 and round(r["fi"], 3) == 0.153 and round(r["tsi"], 3) == 0.080


def test_mmi_lattice_positions_fill_every_cell_evenly():
    # lattice loading: ppc points per cell on a regular sub-lattice, every cell holding exactly
    # ppc particles of each species, at the same points in every cell; velocities unchanged
    from paper_1211_4575_amd import inputs as I
    n, ppc = (6, 5, 4), 12
    wl = I.mmi(n=n, ppc=ppc, lattice=(2, 2, 3))
    noisy = I.mmi(n=n, ppc=ppc)
    for sp, sn in zip(wl.species, noisy.species):
        cell = np.floor(sp.pos).astype(np.int64)
        lin = cell[0] + n[0] * (cell[1] + n[1] * cell[2])
        assert np.array_equal(np.bincount(lin, minlength=n[0] * n[1] * n[2]), np.full(n[0] * n[1] * n[2], ppc))
        frac = sp.pos - cell
        assert set(np.round(frac[0], 12)) == {0.25, 0.75} and set(np.round(frac[1], 12)) == {0.25, 0.75}
        assert set(np.round(frac[2], 12)) == {round(1 / 6, 12), 0.5, round(5 / 6, 12)}
        assert np.array_equal(sp.u, sn.u)
        # the mean position of a cell's points is its centre
        np.testing.assert_allclose(frac.reshape(3, -1, ppc).mean(axis=2), 0.5, atol=1e-12)
    with pytest.raises(ValueError):
        I.mmi(n=n, ppc=ppc, lattice=(2, 2, 2))


def test_mmi_quiet_start_pairs_cancel_the_thermal_current():
    # quiet start: particles 2k and 2k+1 of every species sit at one position with opposite
    # rest-frame thermal velocities, so each pair of the background (no boost) carries no
    # current and the set-up is the noisy one's even particles, mirrored
    from paper_1211_4575_amd import inputs as I
    wl = I.mmi(n=(6, 5, 4), ppc=40, quiet=True)
    noisy = I.mmi(n=(6, 5, 4), ppc=40)
    for sp, sn in zip(wl.species, noisy.species):
        assert np.array_equal(sp.pos[:, 0::2], sp.pos[:, 1::2])
        assert np.array_equal(sp.pos[:, 0::2], sn.pos[:, 0::2])
        assert np.array_equal(sp.u[:, 0::2], sn.u[:, 0::2])
    for sp in wl.species[2:]:  # background: at rest, so the pair's proper velocities cancel
        assert np.array_equal(sp.u[:, 0::2], -sp.u[:, 1::2])
    # the beam's pairs: opposite rest-frame velocities, then the boost G = 4 along z, so the
    # transverse parts are opposite and the z parts average to G beta gamma', gamma' the shared
    # rest-frame Lorentz factor (recovered from the even member: gamma' = G (gamma - beta u_z))
    G, beta = 4.0, np.sqrt(1 - 1 / 16.0)
    for e_b in wl.species[:2]:
        assert np.array_equal(e_b.u[:2, 0::2], -e_b.u[:2, 1::2])
        ue = e_b.u[:, 0::2]
        gam_rest = G * (np.sqrt(1.0 + (ue ** 2).sum(axis=0)) - beta * ue[2])
        np.testing.assert_allclose(0.5 * (e_b.u[2, 0::2] + e_b.u[2, 1::2]), G * beta * gam_rest, rtol=1e-12)


def test_direct_current_breaks_gauss_and_the_filter_restores_it(orc):
    # the plain-heating workload with the direct current (eq. "jj2"): Gauss's law drifts away
    # from its initial zero; five filter passes per step keep it orders of magnitude lower,
    # and the charge-conserving current keeps it at rounding level
    from paper_1211_4575_amd import inputs as I
    wl = I.plain_heating(n=(8, 8, 8), ppc=8)
    res = {}
    for name, kw in (("direct", dict(current_scheme=1)), ("filtered", dict(current_scheme=1, gauss_passes=5)),
                     ("cc", {})):
        P = orc.make_params(**{**wl.params(), **kw})
        run = orc.Run(P, [dict(q=s.q, m=s.m, w=s.w, pos=s.pos, u=s.u) for s in wl.species])
        worst = 0.0
        for _ in range(10):
            run.step()
            worst = max(worst, np.max(np.abs(orc.div_down(P, run.E) - run.rho())))
        res[name] = worst
    assert res["direct"] > 1e-3
    assert res["filtered"] < 0.05 * res["direct"]
    assert res["cc"] < 1e-12


def test_gauss_filter_cadence(orc):
    # the filter after every third step only: the Gauss error after a filtered step is the one
    # of filtering every step from the same state, and between filtered steps it grows back
    from paper_1211_4575_amd import inputs as I
    wl = I.plain_heating(n=(8, 8, 8), ppc=8)
    sp = [dict(q=s.q, m=s.m, w=s.w, pos=s.pos, u=s.u) for s in wl.species]
    P3 = orc.make_params(**{**wl.params(), "current_scheme": 1, "gauss_passes": 5, "gauss_every": 3})
    P1 = orc.make_params(**{**wl.params(), "current_scheme": 1, "gauss_passes": 5})
    r3, r1 = orc.Run(P3, sp), orc.Run(P1, sp)
    err = []
    for step in range(6):
        r3.step()
        r1.step()
        err.append(np.max(np.abs(orc.div_down(P3, r3.E) - r3.rho())))
        if step == 2:  # the first filtered step of the cadence: the state differs from r1 only
            # by the unfiltered steps 1 and 2, so its error is of the same order as r1's
            e1 = np.max(np.abs(orc.div_down(P1, r1.E) - r1.rho()))
            assert err[2] < 3 * e1
    assert err[1] > err[0] and err[2] < 0.5 * err[1] and err[3] > err[2] and err[5] < 0.5 * err[4]
