"""Pins against numbers the paper prints (tests/golden/paper_values.txt, each with its
passage): the 6th-order stencil coefficients, the penta-diagonal system of the high-order
current (eq. "penta": symmetric, with diagonals a+b+c, b+c and c, in the current's
differences), and the cold-beam growth rates of the mixed-mode test."""
import os

import numpy as np
import pytest

from paper_1211_4575_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _values():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, value = line.split()[:2]
        out[name] = float(value)
    return out


def test_sixth_order_coefficients_match_the_printed_ones(orc):
    v = _values()
    a, b, c = orc.fd_coeffs(6)
    assert b == v["fd6_b"] and c == v["fd6_c"]
    # the printed a is the reading's exception: 75/64 makes the stencil a first derivative
    assert a == 75.0 / 64.0 and a != v["fd6_a_printed"]
    assert a + 3 * b + 5 * c == pytest.approx(1.0, abs=1e-15)
    assert v["fd6_a_printed"] + 3 * b + 5 * c == pytest.approx(1.0186, abs=1e-4)


@pytest.mark.parametrize("fo", [4, 6])
def test_high_order_current_solves_the_printed_banded_system(orc, fo):
    # eq. "jj6d"/"penta": in the differences dJ_i = J_i - J_(i-1) of the high-order current,
    # c (dJ_(i+2) + dJ_(i-2)) + (b + c)(dJ_(i+1) + dJ_(i-1)) + (a + b + c) dJ_i equals the
    # second-order current's difference (the decomposed charge change); for 4th order the
    # system is tri-diagonal (c = 0)
    n = (24, 6, 5)
    P = orc.make_params(n=n, shape_order=3, field_order=fo)
    rng = np.random.default_rng(3)
    J2 = rng.normal(size=(3, n[2], n[1], n[0]))
    Jo = orc.current_high_order(P, J2.copy())
    a, b, c = orc.fd_coeffs(fo)
    for comp, axis in ((0, 2), (1, 1), (2, 0)):  # x along the last array axis
        d2 = J2[comp] - np.roll(J2[comp], 1, axis=axis)
        do = Jo[comp] - np.roll(Jo[comp], 1, axis=axis)
        lhs = (c * (np.roll(do, -2, axis=axis) + np.roll(do, 2, axis=axis))
               + (b + c) * (np.roll(do, -1, axis=axis) + np.roll(do, 1, axis=axis)) + (a + b + c) * do)
        assert np.max(np.abs(lhs - d2)) < 1e-12 * np.max(np.abs(d2))


def test_mixed_mode_theory_rates_match_the_printed_ones():
    v = _values()
    r = I.mmi_rates()
    assert round(r["mmi"], 3) == v["mmi_theory"]
    assert round(r["fi"], 3) == v["fi_theory"]
    assert round(r["tsi"], 3) == v["tsi_theory"]
