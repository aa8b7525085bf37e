"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of oracle.c (a dropped term,
a wrong sign or exponent, a missing pivot), builds it, and checks that the pin
meant for that part of the oracle now fails.  The real oracle is untouched.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2405_05974_amd import synth
from tests import mechs, rhs_numpy

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")
P = synth.P_ATM
RU = 8.31446261815324


def build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert old in src, old
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    cmd = list(oracle.BUILD_CMD)
    cmd[cmd.index(oracle._SRC)] = str(mut)
    cmd[cmd.index(oracle._LIB)] = str(lib)
    subprocess.run(cmd, check=True, capture_output=True)
    return str(lib)


# ----------------------------------------------------------------- pins
# Each returns True when the pin holds for the given oracle library.

def pin_gibbs_minimum(lib):
    sp = [("A", (2, 1), 3.5, 1e-4, 0.0, 200.0, False),
          ("B", (1, 1), 3.5, 2e-4, 150000.0, 200.0, False),
          ("C", (1, 0), 3.5, 1e-4, 110000.0, 150.0, False),
          ("N", (0, 2), 3.0, 1e-4, 0.0, 190.0, True)]
    mm = mechs.tiny(sp, [synth.Reaction([0], [1, 2], 1e9, 0.0, 10.0, True, 0)])
    om = oracle.Mech(mm.to_text(), lib_path=lib)
    W = om.weights()
    T = 1500.0
    Y0 = np.array([0.3, 0.0, 0.0, 0.7])
    _, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, 10.0, 1e-11, 1e-24, fixed_T=True, max_steps=200000)
    n = Y1[:, 0] / W
    _, _, _, G = om.thermo(T)
    g = G / (RU * T)
    nA0, nI = Y0[0] / W[0], Y0[3] / W[3]
    from scipy.optimize import brentq

    def dG(xi):
        return g[1] + g[2] - g[0] + math.log(xi * xi / ((nA0 - xi) * (nA0 + xi + nI)))

    xi = brentq(dG, 1e-14 * nA0, nA0 * (1 - 1e-14), xtol=1e-20, rtol=1e-15)
    return st[0]["status"] == 0 and abs(n[1] / xi - 1) < 1e-7


def pin_decay(lib, kind):
    T = 1200.0
    conc = P / (RU * T) * 1e-6
    if kind == "third_body":
        m = mechs.isomer_pair(A=1e10, b=0.0, Ea=3.0, kind=1)
        k = mechs.kf_arrhenius(1e10, 0.0, 3.0, T) * conc
    else:
        m = mechs.isomer_pair(A=2e3, b=0.1, Ea=4.0, kind=2, low=(1e9, 0.0, 4.0))
        kinf = mechs.kf_arrhenius(2e3, 0.1, 4.0, T)
        Pr = mechs.kf_arrhenius(1e9, 0.0, 4.0, T) * conc / kinf
        k = kinf * Pr / (1 + Pr)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    Y0 = np.array([0.25, 0.05, 0.70])
    dt = 2.5 / k
    _, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, dt, 1e-12, 1e-20)
    return st[0]["status"] == 0 and abs(Y1[0, 0] / (0.25 * math.exp(-2.5)) - 1) < 1e-8


def pin_complex_step(lib):
    m = synth.config_mechanism(1)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    rng = np.random.default_rng(5)
    y = np.concatenate([synth.composition(rng, m.n_species, 1.0, 1)[:, 0], [1400.0]])
    f_or = om.rhs(y, P)
    if not np.allclose(rhs_numpy.rhs(m, y, P), f_or, rtol=1e-10, atol=1e-12 * np.abs(f_or).max()):
        return False
    Jcs = rhs_numpy.jac_complex_step(m, y, P)
    if np.abs(om.jac(y, P) - Jcs).max() > 1e-9 * np.abs(Jcs).max():
        return False
    mm = mechs.mixed_kinds()
    om2 = oracle.Mech(mm.to_text(), lib_path=lib)
    y2 = np.array([0.1, 0.05, 0.08, 0.02, 0.75, 1500.0])
    Jcs2 = rhs_numpy.jac_complex_step(mm, y2, P)
    return np.abs(om2.jac(y2, P) - Jcs2).max() <= 1e-9 * np.abs(Jcs2).max()


def pin_thermo_reference(lib):
    m = synth.config_mechanism(1)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    H, Sm, _, _ = om.thermo(298.15)
    Hp, Sp, _, _ = om.thermo(1000.0 + 0.1)
    Hm, Smm, _, _ = om.thermo(1000.0 - 0.1)
    _, _, Cp, _ = om.thermo(1000.0)
    return (np.allclose(H, m.hf, atol=1e-9) and np.allclose(Sm, m.s0, atol=1e-12)
            and np.allclose((Sp - Smm) / 0.2, Cp / 1000.0, rtol=1e-7))


def pin_lu(lib):
    import ctypes as C
    l = C.CDLL(lib)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(11, 11))
    A[0, 0] = 0.0
    b = rng.normal(size=11)
    a = np.ascontiguousarray(A).copy()
    piv = np.zeros(11, dtype=np.int32)
    l.orc_lu(11, a.ctypes.data_as(C.POINTER(C.c_double)), piv.ctypes.data_as(C.POINTER(C.c_int)))
    x = b.copy()
    l.orc_lu_solve(11, a.ctypes.data_as(C.POINTER(C.c_double)), piv.ctypes.data_as(C.POINTER(C.c_int)),
                   x.ctypes.data_as(C.POINTER(C.c_double)))
    return bool(np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12))


def pin_radau(lib):
    from scipy.integrate import solve_ivp
    m = synth.config_mechanism(1)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    rng = np.random.default_rng(42)
    y0 = np.concatenate([synth.composition(rng, m.n_species, 1.0, 1)[:, 0], [1250.0]])
    ref = oracle.Mech(m.to_text())          # the real oracle's rhs drives Radau
    sol = solve_ivp(lambda t, y: ref.rhs(y, P), (0, 1e-6), y0, method="Radau", jac=lambda t, y: ref.jac(y, P),
                    rtol=1e-12, atol=1e-16)
    T1, Y1, st = om.integrate(y0[-1:], y0[:-1, None], P, 1e-6, 1e-10, 1e-16)
    return (st[0]["status"] == 0 and np.abs(Y1[:, 0] - sol.y[:-1, -1]).max() <= 2e-8
            and abs(T1[0] - sol.y[-1, -1]) / sol.y[-1, -1] <= 2e-8)


def pin_enthalpy_inversion(lib):
    m = synth.config_mechanism(1)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    rng = np.random.default_rng(7)
    ok = True
    for T in (400.0, 1300.0, 2700.0):
        Y = synth.composition(rng, m.n_species, 1.0, 1)[:, 0]
        ok = ok and abs(om.temperature_from_h(om.enthalpy(T, Y), Y) / T - 1) <= 1e-12
    return bool(ok)


def pin_enthalpy_conservation(lib):
    m = synth.config_mechanism(1)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    w = synth.uniform_batch(m, 4, 1001, 1000, 1600, 1e-6, 1e-8, 1e-12)
    T, Y, st = om.integrate(w.T, w.Y, w.p, w.dt, w.rtol, w.atol)
    ok = (st["status"] == 0).all()
    for i in range(4):
        h0 = om.enthalpy(w.T[i], w.Y[:, i])
        ok = ok and abs(om.enthalpy(T[i], Y[:, i]) - h0) <= 1e-7 * (abs(h0) + 1.5e6)
    return bool(ok)


def pin_difference_quotient(lib):
    m = synth.config_mechanism(1)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    rng = np.random.default_rng(9)
    y = np.concatenate([synth.composition(rng, m.n_species, 1.0, 1)[:, 0], [1400.0]])
    Jcs = rhs_numpy.jac_complex_step(m, y, P)
    w = 1.0 / (1e-8 * np.abs(y) + 1e-12)
    f = om.rhs(y, P)
    Jfd = om.jac_fd(y, P, w, 1.0 / math.sqrt(np.mean((f * w) ** 2)))
    return bool(np.linalg.norm(Jfd - Jcs) / np.linalg.norm(Jcs) < 1e-5)


# -------------------------------------------- real-mechanism features (f4)

def nasa_species_mech(c3=2e-8, c4=-3e-12, c5=2e-16, delta=6e-8):
    """Two isomers with NASA 7-coefficient thermo whose two ranges differ."""
    sp = [("A", (2, 1), 3.5, 2e-4, 1000.0, 200.0, False),
          ("B", (2, 1), 4.1, 1e-4, -5000.0, 210.0, False),
          ("N", (0, 2), 3.0, 1e-4, 0.0, 190.0, True)]
    m = mechs.tiny(sp, [synth.Reaction([0], [1], 1e6, 0.5, 5.0, True, 0)])
    m.nasa = [synth.nasa7_from_linear(m.a0[k], m.a1[k], m.hf[k], m.s0[k], c3, c4, c5, delta) for k in range(3)]
    return m


def pin_nasa_continuity(lib):
    """cp, H and S continuous at T_mid with differing ranges; dH/dT = cp and
    dS/dT = cp/T on both sides (Richardson-extrapolated central differences)."""
    om = oracle.Mech(nasa_species_mech().to_text(), lib_path=lib)
    Tm = 1000.0
    below = om.thermo(Tm)                  # T <= T_mid: the low range
    above = om.thermo(Tm * (1 + 1e-15))
    for a, b in zip(below[:3], above[:3]):
        if not np.allclose(a, b, rtol=1e-12, atol=0):
            return False
    for T in (600.0, 1700.0):
        def d(i, h):
            return (om.thermo(T + h)[i] - om.thermo(T - h)[i]) / (2 * h)
        dH = (4 * d(0, 0.05) - d(0, 0.1)) / 3
        dS = (4 * d(1, 0.05) - d(1, 0.1)) / 3
        _, _, Cp, _ = om.thermo(T)
        if not (np.allclose(dH, Cp, rtol=1e-8) and np.allclose(dS, Cp / T, rtol=1e-8)):
            return False
    return True


def pin_nasa_reference(lib):
    """The low range holds the 298.15 K anchors the coefficients were built
    on: H = h_f and S = s0 there (the high range differs at 298.15 K)."""
    m = nasa_species_mech()
    om = oracle.Mech(m.to_text(), lib_path=lib)
    H, Sm, _, _ = om.thermo(298.15)
    return bool(np.allclose(H, m.hf, rtol=0, atol=1e-8) and np.allclose(Sm, m.s0, rtol=0, atol=1e-11))


def pin_troe_complex_step(lib):
    """Jacobian of a Troe falloff pair against complex-step derivatives of the
    numpy rhs across the falloff range (Pr from ~1e-3 to ~1e3)."""
    m = troe_pair((0.6, 200.0, 2500.0, 5000.0), eff={2: 3.0})
    om = oracle.Mech(m.to_text(), lib_path=lib)
    y = np.array([0.2, 0.1, 0.7, 1300.0])
    for p in (1e2, 1e4, 1e6, 1e8):
        Jcs = rhs_numpy.jac_complex_step(m, y, p)
        J = om.jac(y, p)
        row = np.abs(J - Jcs).max(axis=1) / np.maximum(np.abs(Jcs).max(axis=1), 1e-300)
        if row.max() > 1e-9:
            return False
    return True


def pin_nasa_reduces_to_linear(lib):
    """NASA polynomials built from a linear cp (c3 = c4 = c5 = delta = 0) give
    the linear species' H, S and cp on both ranges."""
    m = nasa_species_mech(0.0, 0.0, 0.0, 0.0)
    lin = nasa_species_mech()
    lin.nasa = None
    om, ol = oracle.Mech(m.to_text(), lib_path=lib), oracle.Mech(lin.to_text(), lib_path=lib)
    for T in (300.0, 999.0, 1500.0, 2600.0):
        for a, b in zip(om.thermo(T)[:3], ol.thermo(T)[:3]):
            if not np.allclose(a, b, rtol=1e-12, atol=1e-9):
                return False
    return True


def troe_pair(troe, low=(1e12, -0.5, 2.0), eff=None):
    m = mechs.isomer_pair(A=2e5, b=0.3, Ea=6.0, kind=2, low=low)
    m.reactions[0].troe = troe
    m.reactions[0].eff = eff
    return m


def pin_troe_center_and_limits(lib):
    """Troe's blending at points where its shape function f1 is known
    exactly: F = F_cent where log10 Pr = -c (f1 = 0, the centre of the
    falloff curve); f1 = 1/d where log10 Pr + c = n/(2d); f1 = -1/(1+d)
    where log10 Pr + c = -n (log F = log F_cent / (1 + f1^2)); and F_cent = 1
    reduces it to the Lindemann form bit for bit."""
    T = 1300.0
    troe = (0.6, 200.0, 2500.0, 5000.0)
    Fc = 0.4 * math.exp(-T / 200.0) + 0.6 * math.exp(-T / 2500.0) + math.exp(-5000.0 / T)
    kinf = mechs.kf_arrhenius(2e5, 0.3, 6.0, T)
    k0 = mechs.kf_arrhenius(1e12, -0.5, 2.0, T)
    om = oracle.Mech(troe_pair(troe).to_text(), lib_path=lib)
    Y = np.array([0.2, 0.1, 0.7])

    def kf_at(Pr):
        conc = Pr * kinf / k0                      # [M] in mol/cm^3 (unit efficiencies)
        p = conc * 1e6 * RU * T
        return om.rates(T, Y, p)[0][0], conc
    c = -0.4 - 0.67 * math.log10(Fc)
    Pr_c = 10.0 ** (-c)
    kc, _ = kf_at(Pr_c)
    if abs(kc / (kinf * Pr_c / (1 + Pr_c) * Fc) - 1) > 1e-12:
        return False
    n = 0.75 - 1.27 * math.log10(Fc)
    for u, f1 in ((n / (2 * 0.14), 1 / 0.14), (-n, -1 / 1.14)):
        Pr = 10.0 ** (u - c)
        k, _ = kf_at(Pr)
        if abs(k / (kinf * Pr / (1 + Pr) * Fc ** (1.0 / (1.0 + f1 * f1))) - 1) > 1e-11:
            return False
    flat = oracle.Mech(troe_pair((0.0, 1e300, 1.0)).to_text(), lib_path=lib)
    lind = oracle.Mech(troe_pair(None).to_text(), lib_path=lib)
    p = 3e5
    return bool(flat.rates(T, Y, p)[0][0] == lind.rates(T, Y, p)[0][0])


def pin_efficiency_decay(lib):
    """Irreversible third-body A -> B at fixed T with the inert colliding at
    efficiency 5 and B at 0: Y_A decays as exp(-k_f [M] t) with
    [M] = C_A + 5 C_N, both constant in time."""
    T = 1200.0
    m = mechs.isomer_pair(A=1e10, b=0.0, Ea=3.0, kind=1)
    m.reactions[0].eff = {1: 0.0, 2: 5.0}
    om = oracle.Mech(m.to_text(), lib_path=lib)
    W = om.weights()
    Y0 = np.array([0.25, 0.05, 0.70])
    rho = P * 10.0 / (RU * 1e7 * T) / np.sum(Y0 / W)
    CA, CN = rho * Y0[0] / W[0], rho * Y0[2] / W[2]
    # [M] changes as A turns into B (efficiency 1 -> 0): solve dCA/dt = -k CA (CA + 5 CN) in closed form
    k = mechs.kf_arrhenius(1e10, 0.0, 3.0, T)
    a = 5.0 * CN
    t = 2.0 / (k * (CA + a))
    CA_t = a * CA * math.exp(-k * a * t) / (a + CA * (1 - math.exp(-k * a * t)))
    _, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, t, 1e-12, 1e-20, fixed_T=True)
    return st[0]["status"] == 0 and abs(Y1[0, 0] / (CA_t * W[0] / rho) - 1) < 1e-8


def pin_real_complex_step(lib):
    """The analytic Jacobian of a mechanism with NASA thermo, Troe falloff and
    efficiencies against complex-step derivatives of the numpy rhs, on both
    thermo ranges and at two pressures."""
    m = synth.make_real_mechanism(12, 40, 4, 5)
    om = oracle.Mech(m.to_text(), lib_path=lib)
    rng = np.random.default_rng(11)
    for T in (750.0, 1600.0):
        y = np.concatenate([synth.composition(rng, m.n_species, 1.0, 1)[:, 0], [T]])
        for p in (P, 6e6):
            f_or = om.rhs(y, p)
            if not np.allclose(rhs_numpy.rhs(m, y, p), f_or, rtol=1e-10, atol=1e-12 * np.abs(f_or).max()):
                return False
            Jcs = rhs_numpy.jac_complex_step(m, y, p)
            J = om.jac(y, p)
            row = np.abs(J - Jcs).max(axis=1) / np.maximum(np.abs(Jcs).max(axis=1), 1e-300)
            if row.max() > 1e-9:
                return False
    return True


# ---------------------------------------------- quasi-steady-state species (f3)

def pin_qss_numpy(lib):
    """The reduced rhs and its Jacobian (QSS closure, one-sided linearisation,
    chain rule through the closure) against the numpy reduced rhs, which
    reads the closure matrix off its own affine QSS production rates, and
    complex-step derivatives of it; on the hand-built QSS mechanism with its
    quadratic couplings, below and above 1000 K and at two pressures."""
    for third in (False, True):
        if not _qss_numpy_case(lib, mechs.qss_tiny(third=third)):
            return False
    return True


def _qss_numpy_case(lib, m):
    om = oracle.Mech(m.to_text(), lib_path=lib)
    rng = np.random.default_rng(3)
    for T in (800.0, 1400.0, 2200.0):
        for p in (P, 6e6):
            Y = np.concatenate([0.3 * rng.dirichlet(np.ones(5)), [0.7]])
            y = np.concatenate([Y, [T]])
            f, fn = om.rhs(y, p), rhs_numpy.rhs_qss(m, y, p)
            if np.abs(f - fn).max() > 1e-12 * np.abs(fn).max():
                return False
            J, Jc = om.jac(y, p), rhs_numpy.jac_complex_step(m, y, p)
            row = np.abs(J - Jc).max(axis=1) / np.maximum(np.abs(Jc).max(axis=1), 1e-300)
            if row.max() > 1e-11:
                return False
    return True


def _qss_full_and_reduced(lib, dh):
    m = mechs.qss_tiny(coupling=False, dh_qss=dh)
    red = oracle.Mech(m.to_text(), lib_path=lib)
    full_m = mechs.qss_tiny(coupling=False, dh_qss=dh)
    full_m.qss = None
    full = oracle.Mech(full_m.to_text(), lib_path=lib)
    return m, red, full


def pin_qss_validity(lib):
    """Quasi-steady state is the limit of a fast, scarce intermediate: with
    no quadratic coupling, the reduced integration approaches the full one
    (X and Y integrated, started at their closure values) as X and Y are made
    less stable, from ~1e-5 in T/T to the integration tolerance."""
    T0 = np.array([1150.0, 1300.0])
    Y0 = np.array([[0.1, 0.05], [0.1, 0.1], [0.05, 0.05], [0.02, 0.05], [0.03, 0.05], [0.7, 0.7]])
    diffs = []
    for dh in (0.0, 6e4):
        m, red, full = _qss_full_and_reduced(lib, dh)
        W = full.weights()
        ts = m.transported
        Yf = np.zeros((m.n_species, 2))
        for i in range(2):
            Cq, _, _ = red.qss_rates(T0[i], Y0[:, i], P)
            rho = P * 10 / (RU * 1e7 * T0[i]) / np.sum(Y0[:, i] / W[ts])
            Yf[ts, i] = Y0[:, i]
            Yf[m.qss, i] = Cq * W[m.qss] / rho
        Yf /= Yf.sum(axis=0)
        T1, Y1, s1 = red.integrate(T0, Y0, P, 2e-4, 1e-10, 1e-16)
        T2, Y2, s2 = full.integrate(T0, Yf, P, 2e-4, 1e-10, 1e-16)
        if s1["status"].any() or s2["status"].any():
            return False
        diffs.append(max((np.abs(T1 - T2) / T2).max(), np.abs(Y1 - Y2[ts]).max()))
    return diffs[0] > 1e-6 and diffs[1] < 1e-8 and diffs[1] < 1e-3 * diffs[0]


def pin_qss_closure_zero(lib):
    """At the closure's concentrations the full mechanism (regular rate
    code, QSS species as ordinary species) produces no net X or Y, and its
    transported production rates are the reduced ones.  The full state holds
    every concentration of the reduced one plus the QSS ones, so its pressure
    is raised by the QSS share of the moles (ideal gas)."""
    m, red, full = _qss_full_and_reduced(lib, 3e4)
    W = full.weights()
    ts = m.transported
    for T in (1100.0, 1700.0):
        Y0 = np.array([0.08, 0.07, 0.06, 0.05, 0.04, 0.7])
        Cq, wd, bad = red.qss_rates(T, Y0, P)
        rho = P * 10 / (RU * 1e7 * T) / np.sum(Y0 / W[ts])
        C = np.zeros(m.n_species)
        C[ts] = rho * Y0 / W[ts]
        C[m.qss] = Cq
        Yf = C * W / np.sum(C * W)
        pf = P * np.sum(C) / np.sum(C[ts])
        kf, kr, Q, wf = full.rates(T, Yf, pf)
        gross = np.abs(full.nu()) @ np.abs(Q)
        if bad or np.abs(wf[m.qss]).max() > 1e-12 * gross[m.qss].max():
            return False
        if np.abs(wf[ts] - wd).max() > 1e-9 * gross[ts].max():
            return False
    return True


MUTATIONS = [
    ("standard-state exponent sign", "pow(c0, (double)dnu)", "pow(c0, (double)-dnu)", pin_gibbs_minimum),
    ("third body drops [M]", "if (x->type == 1) q *= Mj;", "if (x->type == 9) q *= Mj;",
     lambda lib: pin_decay(lib, "third_body")),
    ("Lindemann blend", "kf = kinf * Pr / (1.0 + Pr);", "kf = kinf * Pr;",
     lambda lib: pin_decay(lib, "falloff")),
    ("chain-rule sign of rho", "- m->W[k] * wd[k] / (rho * rho) * drho[j];",
     "+ m->W[k] * wd[k] / (rho * rho) * drho[j];", pin_complex_step),
    ("T-column derivative of K_c", "double dlnKc = sumH / (ORC_RU * T * T) - dnu / T;",
     "double dlnKc = sumH / (ORC_RU * T * T);", pin_complex_step),
    ("entropy temperature term", "a1 * (T - ORC_TREF));\n  *cp", "a1 * T);\n  *cp", pin_thermo_reference),
    ("LU without pivoting", "if (fabs(a[i * n + k]) > best)", "if (0 && fabs(a[i * n + k]) > best)", pin_lu),
    ("BDF psi coefficients", "ss += g[j] * D[j][i];", "ss += g[k] * D[j][i];", pin_radau),
    ("enthalpy inversion sign", "double c = h - al;", "double c = al - h;", pin_enthalpy_inversion),
    ("sign of the temperature equation", "f[S] = fixed_T ? 0.0 : -num / den;", "f[S] = fixed_T ? 0.0 : num / den;",
     pin_enthalpy_conservation),
    ("difference quotient off by the increment", "ytmp[j] = y[j] + inc;", "ytmp[j] = y[j] + 2.0 * inc;",
     pin_difference_quotient),
    ("NASA ranges swapped", "T <= c[0] ? c + 1 : c + 8;", "T <= c[0] ? c + 8 : c + 1;", pin_nasa_reference),
    ("NASA enthalpy constant dropped", "a[4] * T4 * T / 5.0 + a[5]);", "a[4] * T4 * T / 5.0);",
     pin_nasa_continuity),
    ("NASA entropy log term", "*s = ORC_RU * (a[0] * log(T) +", "*s = ORC_RU * (a[0] * T +",
     pin_nasa_reduces_to_linear),
    ("Troe centre offset sign", "double cc = -0.4 - 0.67 * Lc", "double cc = -0.4 + 0.67 * Lc",
     pin_troe_center_and_limits),
    ("Troe derivative in log Pr", "double df1_dlp = nn / (v * v);", "double df1_dlp = 1.0 / v;",
     pin_troe_complex_step),
    ("efficiency offset", "M += (x->effv[i] - 1.0) * C[x->effk[i]];", "M += x->effv[i] * C[x->effk[i]];",
     pin_efficiency_decay),
    ("efficiency in the Jacobian", "double eps = (x->type == 0) ? 0.0 : orc_efficiency(m, x, c);   /* d[M]_j/dC_c */",
     "double eps = (x->type == 0) ? 0.0 : 1.0;", pin_real_complex_step),
    ("heat-capacity slope in the T row", "dden += C[k] * dCp[k];", "dden += 0.0 * dCp[k];",
     pin_real_complex_step),
    ("QSS closure constant term sign", "else b[q] -= nu * c;", "else b[q] += nu * c;", pin_qss_closure_zero),
    ("QSS linearisation threshold", "x->drop_f = nqr >= 2;", "x->drop_f = nqr >= 3;", pin_qss_numpy),
    ("QSS chain-rule sign", "ared -= A[ka * S + m->qsp[q]] * X[q * (ST + 1) + c];",
     "ared += A[ka * S + m->qsp[q]] * X[q * (ST + 1) + c];", pin_qss_numpy),
    ("QSS species as colliders", "if (m->isq[c] >= 0) return 0.0;", "if (m->isq[c] >= 0) return 1.0;",
     pin_qss_numpy),
    ("QSS reverse coefficient sign", "if (n >= 0) A[q * nq + n] -= nu * c;", "if (n >= 0) A[q * nq + n] += nu * c;",
     pin_qss_validity),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    assert pin(oracle._LIB if os.path.exists(oracle._LIB) else oracle.build()), f"pin fails on the real oracle: {name}"
    lib = build_mutant(tmp_path, old, new)
    try:
        caught = not pin(lib)
    except Exception:
        caught = True          # the mutant crashed or produced unusable output
    assert caught, f"planted mistake not caught: {name}"
