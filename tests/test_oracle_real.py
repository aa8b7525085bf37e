"""Oracle pins for the features real (CHEMKIN/Cantera) mechanisms need: NASA
7-coefficient thermo, Troe falloff and collision efficiencies (the paper's
mechanisms come from Cantera input, App. A, with thermo polynomials that
change per species, Sec. 3.2.2).

Each pin checks the oracle against something other than itself: continuity
and derivative identities of the thermo polynomials, the reduction to the
linear-cp and Lindemann forms, exact points of Troe's blending function, a
closed-form decay with efficiencies, complex-step derivatives of the
independent numpy right-hand side, conservation laws and scipy's Radau.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_05974_amd import synth
from tests import mechs, rhs_numpy
from tests import test_oracle_mutations as pins

P = synth.P_ATM


@pytest.fixture(scope="module")
def lib():
    return oracle._LIB if __import__("os").path.exists(oracle._LIB) else oracle.build()


@pytest.mark.parametrize("pin", [pins.pin_nasa_continuity, pins.pin_nasa_reference, pins.pin_nasa_reduces_to_linear,
                                 pins.pin_troe_center_and_limits, pins.pin_troe_complex_step,
                                 pins.pin_efficiency_decay, pins.pin_real_complex_step],
                         ids=lambda f: f.__name__)
def test_pin_holds(lib, pin):
    assert pin(lib)


def test_parser_reads_and_rejects_the_extensions():
    m = synth.make_real_mechanism(12, 40, 4, 5)
    om = oracle.Mech(m.to_text())
    assert (om.S, om.R) == (12, 40)
    bad = [m.to_text().replace("TROE 3", "TROE 5", 1), m.to_text().replace("EFF 3", "EFF -1", 1),
           m.to_text().replace("NASA7 1000.0", "NASA7 -1000.0", 1)]
    for text in bad:
        with pytest.raises(Exception):
            oracle.Mech(text)
    # EFF on an elementary reaction and TROE on a third-body reaction are errors
    tb = mechs.isomer_pair(kind=1)
    text = tb.to_text().replace("\nEND", " TROE 3 0.5 100.0 1000.0\nEND")
    with pytest.raises(Exception):
        oracle.Mech(text)
    el = mechs.isomer_pair(kind=0)
    text = el.to_text().replace("\nEND", " EFF 1 2 2.0\nEND")
    with pytest.raises(Exception):
        oracle.Mech(text)


def test_unit_efficiencies_listed_equal_none_listed():
    m = synth.make_real_mechanism(12, 40, 4, 5)
    ones = synth.make_real_mechanism(12, 40, 4, 5)
    for r in ones.reactions:
        if r.eff:
            r.eff = {k: 1.0 for k in r.eff}
    none = synth.make_real_mechanism(12, 40, 4, 5)
    for r in none.reactions:
        r.eff = None
    a, b = oracle.Mech(ones.to_text()), oracle.Mech(none.to_text())
    rng = np.random.default_rng(4)
    y = np.concatenate([synth.composition(rng, m.n_species, 1.0, 1)[:, 0], [1450.0]])
    assert np.array_equal(a.rhs(y, P), b.rhs(y, P))
    assert np.array_equal(a.jac(y, P), b.jac(y, P))
    assert not np.array_equal(oracle.Mech(m.to_text()).rhs(y, P), a.rhs(y, P))


@pytest.fixture(scope="module")
def real_run():
    m = synth.make_real_mechanism(12, 40, 4, 5)
    om = oracle.Mech(m.to_text())
    w = synth.uniform_batch(m, 24, 77, 800.0, 1800.0, 1e-6, 1e-8, 1e-12)
    T1, Y1, st = om.integrate(w.T, w.Y, w.p, w.dt, w.rtol, w.atol)
    return m, om, w, T1, Y1, st


def test_real_mechanism_integrates_and_conserves(real_run):
    m, om, w, T1, Y1, st = real_run
    assert all(s["status"] == 0 for s in st)
    E = m.atoms.astype(float)
    W = om.weights()
    for i in range(w.n_cells):
        el0 = E.T @ (w.Y[:, i] / W)
        el1 = E.T @ (Y1[:, i] / W)
        clipped = st[i]["n_clip"] > 0
        if not clipped:
            assert np.allclose(el1, el0, rtol=1e-12, atol=0)
            assert abs(Y1[:, i].sum() - 1.0) < 1e-12
        h0 = om.enthalpy(w.T[i], w.Y[:, i])
        h1 = om.enthalpy(T1[i], Y1[:, i])
        cp_scale = abs(h0) + 3e3 * T1[i]
        assert abs(h1 - h0) <= 1e-6 * cp_scale
    # the solution moved (these are not equilibrium states)
    assert np.abs(Y1 - w.Y).max() > 1e-3


def test_real_mechanism_against_radau(real_run):
    from scipy.integrate import solve_ivp
    m, om, w, T1, Y1, st = real_run
    for i in (0, 7, 19):
        y0 = np.concatenate([w.Y[:, i], [w.T[i]]])
        sol = solve_ivp(lambda t, y: om.rhs(y, P), (0, w.dt), y0, method="Radau", jac=lambda t, y: om.jac(y, P),
                        rtol=1e-12, atol=1e-16)
        assert sol.success
        assert np.abs(Y1[:, i] - sol.y[:-1, -1]).max() <= 2e-8
        assert abs(T1[i] - sol.y[-1, -1]) / sol.y[-1, -1] <= 2e-8


def test_temperature_from_enthalpy_with_nasa(real_run):
    m, om, w, T1, Y1, st = real_run
    for T in (350.0, 999.9, 1000.1, 2400.0):
        Y = w.Y[:, 3]
        h = om.enthalpy(T, Y)
        assert abs(om.temperature_from_h(h, Y) / T - 1) < 1e-12
