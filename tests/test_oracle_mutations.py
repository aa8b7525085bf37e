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


MUTATIONS = [
    ("standard-state exponent sign", "pow(c0, (double)dnu)", "pow(c0, (double)-dnu)", pin_gibbs_minimum),
    ("third body drops [M]", "if (x->type == 1) q *= Mconc;", "if (x->type == 9) q *= Mconc;",
     lambda lib: pin_decay(lib, "third_body")),
    ("Lindemann blend", "kf = kinf * Pr / (1.0 + Pr);", "kf = kinf * Pr;",
     lambda lib: pin_decay(lib, "falloff")),
    ("chain-rule sign of rho", "- m->W[k] * wd[k] / (rho * rho) * drho[j];",
     "+ m->W[k] * wd[k] / (rho * rho) * drho[j];", pin_complex_step),
    ("T-column derivative of K_c", "double dlnKc = sumH / (ORC_RU * T * T) - dnu / T;",
     "double dlnKc = sumH / (ORC_RU * T * T);", pin_complex_step),
    ("entropy temperature term", "a1 * (T - ORC_TREF));\n    if (H)", "a1 * T);\n    if (H)", pin_thermo_reference),
    ("LU without pivoting", "if (fabs(a[i * n + k]) > best)", "if (0 && fabs(a[i * n + k]) > best)", pin_lu),
    ("BDF psi coefficients", "ss += g[j] * D[j][i];", "ss += g[k] * D[j][i];", pin_radau),
    ("enthalpy inversion sign", "double c = h - al;", "double c = al - h;", pin_enthalpy_inversion),
    ("sign of the temperature equation", "f[S] = fixed_T ? 0.0 : -num / den;", "f[S] = fixed_T ? 0.0 : num / den;",
     pin_enthalpy_conservation),
    ("difference quotient off by the increment", "ytmp[j] = y[j] + inc;", "ytmp[j] = y[j] + 2.0 * inc;",
     pin_difference_quotient),
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
