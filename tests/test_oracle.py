"""Pins for the CPU oracle: each check is fixed by mathematics or physics, not
by re-typing the oracle's own formulas.

* thermo: dH/dT = Cp, dS/dT = Cp/T, Gibbs-Helmholtz, reference values
* K_c: isomer special case exp(-dHf/RT); kinetic equilibrium == Gibbs-energy
  minimum (pins the standard-state factor and its exponent sum(nu))
* rates/integration: closed-form decays for elementary, third-body and
  Lindemann reactions, and the A <-> B relaxation
* Jacobian (Eq. 7): complex-step derivative of an independent rhs, the paper's
  Eq. 10 error metric against central differences, first-order convergence of
  one-sided differences (App. C); the integrator's difference-quotient
  Jacobian modes against the complex-step Jacobian and the truth reference
* LU: numpy.linalg.solve; enthalpy inversion: numpy.roots
* integrator: conservation of elements, sum(Y) and enthalpy (to tolerance); detailed balance
  at long times; convergence order 1 and 2 with fixed steps; agreement with
  scipy's Radau within tolerance
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

import oracle
from paper_2405_05974_amd import synth
from tests import mechs, rhs_numpy

RU = 8.31446261815324
P = synth.P_ATM


@pytest.fixture(scope="module")
def g10():
    m = synth.config_mechanism(1)
    return m, oracle.Mech(m.to_text())


def state(m, T, seed=0, alpha=1.0):
    rng = np.random.default_rng(seed)
    Y = synth.composition(rng, m.n_species, alpha, 1)[:, 0]
    return np.concatenate([Y, [T]])


# ------------------------------------------------------------------ parsing

def test_parser_rejects_unbalanced_and_malformed(g10):
    m, _ = g10
    txt = m.to_text()
    with pytest.raises(ValueError):
        oracle.Mech(txt.replace("REACTIONS 25", "REACTIONS 26"))
    bad = mechs.isomer_pair()
    bad.reactions[0].products = [2]       # A -> inert: atoms differ
    with pytest.raises(ValueError, match="balanced"):
        oracle.Mech(bad.to_text())
    with pytest.raises(ValueError):
        oracle.Mech("chem-mech 2\n")


def test_weights_from_atoms(g10):
    m, om = g10
    W = om.weights()
    assert np.allclose(W, m.atoms @ np.array([1.008, 12.011, 15.999]), rtol=1e-15)


# ------------------------------------------------------------------- thermo

def test_thermo_identities(g10):
    m, om = g10
    for T in (300.0, 1000.0, 2500.0):
        h = 1e-4 * T
        Hp, Sp, _, Gp = om.thermo(T + h)
        Hm, Sm_, _, Gm = om.thermo(T - h)
        H, Sm, Cp, G = om.thermo(T)
        assert np.allclose((Hp - Hm) / (2 * h), Cp, rtol=1e-9)          # dH/dT = Cp
        assert np.allclose((Sp - Sm_) / (2 * h), Cp / T, rtol=1e-7)     # dS/dT = Cp/T
        gh = ((Gp / (T + h)) - (Gm / (T - h))) / (2 * h)                  # d(G/T)/dT = -H/T^2
        assert np.allclose(gh, -H / T ** 2, rtol=1e-6, atol=1e-9 * np.abs(H).max() / T ** 2)
        assert np.allclose(G, H - T * Sm, rtol=1e-14, atol=1e-9)
    H, Sm, _, _ = om.thermo(298.15)
    assert np.allclose(H, m.hf, atol=1e-9) and np.allclose(Sm, m.s0, atol=1e-12)


def test_enthalpy_inversion_matches_polynomial_root(g10):
    m, om = g10
    rng = np.random.default_rng(3)
    for T in rng.uniform(250, 3500, 20):
        Y = state(m, T, int(T))[:-1]
        h = om.enthalpy(T, Y)
        Tb = om.temperature_from_h(h, Y)
        assert abs(Tb - T) <= 1e-12 * T
        # the mixture enthalpy is an exact quadratic in T: recover it from three
        # evaluations and ask numpy for the root closest to T
        ts = np.array([300.0, 1500.0, 3000.0])
        coef = np.polyfit(ts, [om.enthalpy(t, Y) for t in ts], 2)
        coef[-1] -= h
        roots = np.roots(coef)
        r = roots[np.argmin(np.abs(roots - T))].real
        assert abs(r - Tb) <= 1e-7 * T


# -------------------------------------------------------------------- rates

def test_kc_isomer_special_case():
    dhf = 12345.0
    m = mechs.isomer_pair(rev=True, dhf=dhf)
    om = oracle.Mech(m.to_text())
    for T in (500.0, 1200.0, 2400.0):
        Y = np.array([0.2, 0.3, 0.5])
        kf, kr, Q, wdot = om.rates(T, Y, P)
        assert kf[0] == pytest.approx(mechs.kf_arrhenius(1e6, 0.5, 5.0, T), rel=1e-13)
        # equal cp and s0: K_c = exp(-(H_B - H_A)/RT) = exp(-dhf/RT)
        assert kr[0] / kf[0] == pytest.approx(math.exp(dhf / (RU * T)), rel=1e-12)
        assert wdot[0] == pytest.approx(-Q[0], rel=1e-15) and wdot[1] == pytest.approx(Q[0], rel=1e-15)


def test_element_and_mass_conservation_of_rates(g10):
    m, om = g10
    W = om.weights()
    for T in (800.0, 1500.0, 2200.0):
        y = state(m, T, 7)
        _, _, Q, wdot = om.rates(T, y[:-1], P)
        scale = np.abs(Q).max() * 4 * 3
        for e in range(m.atoms.shape[1]):
            assert abs(m.atoms[:, e] @ wdot) <= 1e-13 * scale
        assert abs(W @ wdot) <= 1e-13 * scale * W.max()
        nu = om.nu()
        assert np.allclose(nu @ Q, wdot, rtol=1e-13, atol=1e-13 * scale)


def _kinetic_equilibrium(om, T, Y0):
    T1, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, 10.0, 1e-11, 1e-24, fixed_T=True, max_steps=200000)
    assert st[0]["status"] == 0
    return Y1[:, 0]


def test_kc_standard_state_via_gibbs_minimum():
    # A <-> B + C (dnu = +1) with an inert diluent at fixed T and p.  The
    # composition where the kinetics stop must minimise the mixture Gibbs energy
    # sum n_k (G_k/RT + ln(x_k p/p0)) along the reaction extent.
    sp = [("A", (2, 1), 3.5, 1e-4, 0.0, 200.0, False),
          ("B", (1, 1), 3.5, 2e-4, 150000.0, 200.0, False),
          ("C", (1, 0), 3.5, 1e-4, 110000.0, 150.0, False),
          ("N", (0, 2), 3.0, 1e-4, 0.0, 190.0, True)]
    mm = mechs.tiny(sp, [synth.Reaction([0], [1, 2], 1e9, 0.0, 10.0, True, 0)])
    om = oracle.Mech(mm.to_text())
    W = om.weights()
    for T, p in ((1500.0, P), (1500.0, 5 * P), (1900.0, P)):
        Y0 = np.array([0.3, 0.0, 0.0, 0.7])
        T1, Y1, st = om.integrate(np.array([T]), Y0[:, None], p, 10.0, 1e-11, 1e-24, fixed_T=True, max_steps=200000)
        assert st[0]["status"] == 0
        n = Y1[:, 0] / W
        _, _, _, G = om.thermo(T)
        g = G / (RU * T)
        nA0, nI = Y0[0] / W[0], Y0[3] / W[3]

        def dG(xi):   # derivative of the Gibbs energy along the extent
            nA, nB, nC = nA0 - xi, xi, xi
            ntot = nA + nB + nC + nI
            return g[1] + g[2] - g[0] + math.log(nB * nC / (nA * ntot) * p / P)

        xi = brentq(dG, 1e-14 * nA0, nA0 * (1 - 1e-14), xtol=1e-20, rtol=1e-15)
        assert 1e-3 * nA0 < xi < (1 - 1e-3) * nA0
        assert n[1] == pytest.approx(xi, rel=1e-7)
        assert n[0] == pytest.approx(nA0 - xi, rel=1e-7)


# ------------------------------------------------------ closed-form decays

@pytest.mark.parametrize("kind", ["elementary", "third_body", "falloff_mid", "falloff_low", "falloff_high"])
def test_irreversible_isomerisation_closed_form(kind):
    T = 1200.0
    Y0 = np.array([0.25, 0.05, 0.70])
    conc = P / (RU * T) * 1e-6        # [M] = p/RT in mol/cm^3
    if kind == "elementary":
        m = mechs.isomer_pair(A=1e5, b=0.3, Ea=8.0)
        k = mechs.kf_arrhenius(1e5, 0.3, 8.0, T)
    elif kind == "third_body":
        m = mechs.isomer_pair(A=1e10, b=0.0, Ea=3.0, kind=1)
        k = mechs.kf_arrhenius(1e10, 0.0, 3.0, T) * conc
    else:
        A0 = {"falloff_mid": 1e9, "falloff_low": 1e3, "falloff_high": 1e17}[kind]
        m = mechs.isomer_pair(A=2e3, b=0.1, Ea=4.0, kind=2, low=(A0, 0.0, 4.0))
        kinf = mechs.kf_arrhenius(2e3, 0.1, 4.0, T)
        k0 = mechs.kf_arrhenius(A0, 0.0, 4.0, T)
        Pr = k0 * conc / kinf
        k = kinf * Pr / (1 + Pr)
        if kind == "falloff_low":
            assert k == pytest.approx(k0 * conc, rel=1e-5)
        if kind == "falloff_high":
            assert k == pytest.approx(kinf, rel=1e-5)
    om = oracle.Mech(m.to_text())
    dt = 2.5 / k
    # isomers with identical thermo: no heat release, T stays put adiabatically
    T1, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, dt, 1e-12, 1e-20)
    assert st[0]["status"] == 0
    assert abs(T1[0] - T) <= 1e-10 * T
    assert Y1[0, 0] == pytest.approx(Y0[0] * math.exp(-k * dt), rel=1e-8)
    assert Y1[0, 0] + Y1[1, 0] == pytest.approx(Y0[0] + Y0[1], rel=1e-13)


def test_reversible_relaxation_closed_form():
    T, dt, dhf = 1000.0, 1e-3, 4000.0
    m = mechs.isomer_pair(A=1e3, b=0.0, Ea=2.0, rev=True, dhf=dhf)
    om = oracle.Mech(m.to_text())
    kf = mechs.kf_arrhenius(1e3, 0.0, 2.0, T)
    kr = kf * math.exp(dhf / (RU * T))
    Y0 = np.array([0.3, 0.0, 0.7])
    Yeq = Y0[0] * kr / (kf + kr)
    T1, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, dt, 1e-12, 1e-20, fixed_T=True)
    expect = Yeq + (Y0[0] - Yeq) * math.exp(-(kf + kr) * dt)
    assert Y1[0, 0] == pytest.approx(expect, rel=1e-8)


def test_adiabatic_equilibrium_root():
    # A <-> B isomers with different formation enthalpy, adiabatic: the long-time
    # state solves Y_B/Y_A = K_c(T) = exp(-dhf/RT) together with h(T, Y) = h0.
    dhf = -30000.0
    m = mechs.isomer_pair(A=1e6, b=0.0, Ea=10.0, rev=True, dhf=dhf)
    om = oracle.Mech(m.to_text())
    T0, Y0 = 1200.0, np.array([0.3, 0.0, 0.7])
    h0 = om.enthalpy(T0, Y0)

    def resid(T):
        x = 1.0 / (1.0 + math.exp(-dhf / (RU * T)))      # fraction left as A
        Y = np.array([0.3 * x, 0.3 * (1 - x), 0.7])
        return om.enthalpy(T, Y) - h0

    Teq = brentq(resid, T0, T0 + 3000.0, xtol=1e-12)
    T1, Y1, st = om.integrate(np.array([T0]), Y0[:, None], P, 10.0, 1e-11, 1e-20)
    assert st[0]["status"] == 0
    assert T1[0] == pytest.approx(Teq, rel=1e-9)
    assert Y1[1, 0] / Y1[0, 0] == pytest.approx(math.exp(-dhf / (RU * Teq)), rel=1e-7)


# ----------------------------------------------------------------- Jacobian

@pytest.mark.parametrize("T", [700.0, 1400.0, 2300.0])
@pytest.mark.parametrize("fixed_T", [False, True])
def test_jacobian_complex_step(g10, T, fixed_T):
    m, om = g10
    y = state(m, T, int(T) + 11)
    f_np = rhs_numpy.rhs(m, y, P, fixed_T)
    f_or = om.rhs(y, P, fixed_T)
    assert np.allclose(f_np, f_or, rtol=1e-10, atol=1e-12 * np.abs(f_or).max())
    Jcs = rhs_numpy.jac_complex_step(m, y, P, fixed_T)
    J = om.jac(y, P, fixed_T)
    scale = np.abs(Jcs).max()
    assert np.abs(J - Jcs).max() <= 1e-9 * scale
    # row-wise relative check where rows are not tiny
    for i in range(J.shape[0]):
        rs = np.abs(Jcs[i]).max()
        if rs > 1e-6 * scale:
            assert np.abs(J[i] - Jcs[i]).max() <= 1e-8 * rs


def test_jacobian_falloff_and_third_body_complex_step():
    sp = [("A", (2, 1), 3.5, 2e-4, 1000.0, 200.0, False),
          ("B", (2, 1), 3.9, 1e-4, -20000.0, 210.0, False),
          ("C", (1, 1), 4.1, 3e-4, 50000.0, 180.0, False),
          ("D", (1, 0), 2.6, 1e-5, 200000.0, 160.0, False),
          ("N", (0, 2), 3.0, 1e-4, 0.0, 190.0, True)]
    rx = [synth.Reaction([0], [1], 1e9, 0.2, 12.0, True, 2, (1e15, -0.5, 8.0)),
          synth.Reaction([2, 3], [0], 1e12, 0.0, 3.0, True, 1),
          synth.Reaction([1, 1], [0, 0], 1e10, 0.5, 20.0, False, 0),
          synth.Reaction([2, 3, 3], [1, 3], 1e16, -1.0, 1.0, True, 0)]
    mm = mechs.tiny(sp, rx)
    om = oracle.Mech(mm.to_text())
    y = np.array([0.1, 0.05, 0.08, 0.02, 0.75, 1500.0])
    assert np.allclose(rhs_numpy.rhs(mm, y, P), om.rhs(y, P), rtol=1e-10)
    Jcs = rhs_numpy.jac_complex_step(mm, y, P)
    J = om.jac(y, P)
    assert np.abs(J - Jcs).max() <= 1e-9 * np.abs(Jcs).max()


def test_jacobian_eq9_and_one_sided_fd_order(g10):
    m, om = g10
    errs = []
    for s in range(20):
        T = 900.0 + 60.0 * s
        y = state(m, T, 100 + s)
        J = om.jac(y, P)
        Jfd = np.zeros_like(J)
        for j in range(y.size):
            e = 1e-4 * max(abs(y[j]), 1e-6)
            yp, ym = y.copy(), y.copy()
            yp[j] += e
            ym[j] -= e
            Jfd[:, j] = (om.rhs(yp, P) - om.rhs(ym, P)) / (2 * e)
        errs.append(np.linalg.norm(J - Jfd) / np.linalg.norm(Jfd))
    assert np.mean(errs) < 1e-5          # Eq. 10 with central differences
    # App. C: one-sided differences approach the analytic Jacobian at first order
    y = state(m, 1300.0, 5)
    J = om.jac(y, P)
    j = 3
    hs = np.array([1e-2, 1e-3, 1e-4]) * y[j]
    e = []
    for h in hs:
        yp = y.copy()
        yp[j] += h
        col = (om.rhs(yp, P) - om.rhs(y, P)) / h
        e.append(np.linalg.norm(col - J[:, j]) / np.linalg.norm(J[:, j]))
    slope = np.polyfit(np.log(hs), np.log(e), 1)[0]
    assert 0.8 < slope < 1.2


def test_difference_quotient_jacobian(g10):
    """The integrator's finite-difference Jacobian (Sec. 3.2): one-sided
    quotients with the increment max(sqrt(u)|y_j|, m/w_j).  Against the
    complex-step Jacobian its relative Frobenius error (Eq. 10) is of the
    order of the increment, sqrt(u) ~ 1.5e-8, times the curvature of f."""
    for cfg in (1, 4):
        m = synth.config_mechanism(cfg)
        om = oracle.Mech(m.to_text())
        errs = []
        for s, T in enumerate((900.0, 1400.0, 2200.0)):
            y = state(m, T, 40 + s)
            Jcs = rhs_numpy.jac_complex_step(m, y, P)
            w = 1.0 / (1e-8 * np.abs(y) + 1e-12)
            f = om.rhs(y, P)
            h = 1.0 / math.sqrt(np.mean((f * w) ** 2))      # a step the integrator would take here
            Jfd = om.jac_fd(y, P, w, h)
            errs.append(np.linalg.norm(Jfd - Jcs) / np.linalg.norm(Jcs))
        assert max(errs) < 1e-5, (cfg, errs)
        assert min(errs) > 1e-12          # a difference quotient, not the analytic Jacobian


@pytest.mark.parametrize("mode", [1, 2])
def test_integration_with_difference_quotient_jacobian(g10, g10_run, mode):
    """With the finite-difference Jacobian (all columns, or only the T column
    as in Sec. 3.2.2) Newton converges to the same corrector equations: the
    result matches the tight-tolerance truth to a small multiple of rtol, at
    the price of extra right-hand sides (N per Jacobian, or one)."""
    m, om = g10
    w, T, Y, st = g10_run
    idx = np.arange(0, 48, 4)
    Tt, Yt, _ = om.integrate(w.T[idx], w.Y[:, idx], w.p, w.dt, 1e-12, 1e-20)
    Tf, Yf, sf = om.integrate(w.T[idx], w.Y[:, idx], w.p, w.dt, w.rtol, w.atol, jac_mode=mode)
    assert (sf["status"] == 0).all()
    assert np.abs(Yf - Yt).max() <= 1e-7
    assert (np.abs(Tf - Tt) / Tt).max() <= 1e-7
    extra = sf["n_rhs"] - sf["n_newton"] - 1          # right-hand sides beyond the Newton residuals
    per_jac = m.n_species + 1 if mode == 1 else 1
    assert (extra == per_jac * sf["n_jac"]).all()


def test_difference_quotient_scatter_under_summation_order():
    """The finite-difference Jacobian modes reproduce only to the integration
    accuracy: with nothing changed but the order of the reactions (so the
    summation order of the production rates, a rounding-level change), the
    oracle's own results on a config-1 sample move by far more than rounding,
    yet stay within the integration-accuracy bar of the GPU tests (1e-7 in Y,
    1e-6 in T/T from the truth, twice that between two runs).  The default
    analytic-Jacobian integrator, for contrast, moves only slightly."""
    import copy
    w = synth.config_workload(1)
    idx = np.arange(0, w.n_cells, 16)
    T0, Y0 = w.T[idx], w.Y[:, idx]
    om = oracle.Mech(w.mech.to_text())
    Tt, Yt, _ = om.integrate(T0, Y0, w.p, w.dt, 1e-12, 1e-20)
    rng = np.random.default_rng(7)
    perms = [rng.permutation(w.mech.n_reactions) for _ in range(4)]
    mechs_p = []
    for perm in perms:
        m2 = copy.deepcopy(w.mech)
        m2.reactions = [m2.reactions[i] for i in perm]
        mechs_p.append(oracle.Mech(m2.to_text()))
    spread = {}
    for mode in (0, 1, 2):
        To, Yo, _ = om.integrate(T0, Y0, w.p, w.dt, w.rtol, w.atol, jac_mode=mode)
        dT = dY = dTt = dYt = 0.0
        for o2 in mechs_p:
            Tq, Yq, sq = o2.integrate(T0, Y0, w.p, w.dt, w.rtol, w.atol, jac_mode=mode)
            assert (sq["status"] == 0).all()
            dT = max(dT, (np.abs(Tq - To) / To).max())
            dY = max(dY, np.abs(Yq - Yo).max())
            dTt = max(dTt, (np.abs(Tq - Tt) / Tt).max())
            dYt = max(dYt, np.abs(Yq - Yt).max())
        spread[mode] = dT
        assert dY <= 2e-7 and dT <= 2e-6, (mode, dY, dT)
        assert dYt <= 1e-7 and dTt <= 1e-6, (mode, dYt, dTt)
    # far more than rounding in the difference-quotient modes, while the
    # analytic-Jacobian default stays inside its own 1e-8 parity bar
    assert spread[1] > 5e-8 and spread[2] > 5e-8, spread
    assert spread[0] <= 1e-8, spread


# ----------------------------------------------------------- linear algebra

def test_lu_matches_numpy():
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 11, 31, 54):
        A = rng.normal(size=(n, n))
        if n > 1:
            A[0, 0] = 0.0                 # forces a pivot in column 0
        b = rng.normal(size=n)
        a, piv, info = oracle.lu(A)
        assert info == 0
        x = oracle.lu_solve(a, piv, b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
        L = np.tril(a, -1) + np.eye(n)
        U = np.triu(a)
        PA = A.copy()
        for k in range(n):
            PA[[k, piv[k]]] = PA[[piv[k], k]]
        assert np.abs(PA - L @ U).max() <= 1e-14 * n * np.abs(A).max()
        assert np.abs(L).max() <= 1.0 + 1e-15     # partial pivoting bound
    a, piv, info = oracle.lu(np.zeros((3, 3)))
    assert info == 1


# --------------------------------------------------------------- integrator

@pytest.fixture(scope="module")
def g10_run(g10):
    m, om = g10
    w = synth.uniform_batch(m, 48, 1001, 1000, 1600, 1e-5, 1e-8, 1e-12)
    T, Y, st = om.integrate(w.T, w.Y, w.p, w.dt, w.rtol, w.atol, nthreads=0)
    return w, T, Y, st


def test_integration_invariants(g10, g10_run):
    m, om = g10
    w, T, Y, st = g10_run
    assert (st["status"] == 0).all()
    W = om.weights()
    # Linear invariants (total mass, element totals) are exact in exact
    # arithmetic (c^T D_j = 0 for every backward difference), so in cells the
    # positivity projection never touched they hold to rounding, which grows
    # with the Newton iterates.  Zeroing a component's differences breaks
    # c^T D_j = 0 for the following steps: there they hold to the integration
    # tolerance only.
    clip = st["n_clip"] > 0
    assert (clip == (st["clip_mass"] > 0)).all() and (~clip).sum() >= 24
    dev = np.abs(Y.sum(axis=0) - 1.0)
    assert dev[~clip].max() <= 1e-10 and np.median(dev) <= 1e-14 and dev.max() <= 1e-8
    for e in range(m.atoms.shape[1]):
        z0 = (m.atoms[:, e] / W) @ w.Y
        z1 = (m.atoms[:, e] / W) @ Y
        rel = np.abs(z1 - z0) / np.abs(z0).max()
        assert rel[~clip].max() <= 1e-10 and np.median(rel) <= 1e-14 and rel.max() <= 1e-8
    # Enthalpy is conserved by the ODE (adiabatic, constant pressure) but not
    # exactly by BDF, since it is nonlinear in T: the drift is an integration
    # error and shrinks with the tolerance.
    scale = np.array([om.enthalpy(w.T[i], w.Y[:, i]) for i in range(48)])
    cpT = 1.5e6                        # J/kg, cp * T of these mixtures
    drift = np.array([abs(om.enthalpy(T[i], Y[:, i]) - scale[i]) for i in range(48)]) / (np.abs(scale) + cpT)
    assert drift.max() <= 1e-7
    Tt, Yt, _ = om.integrate(w.T[:8], w.Y[:, :8], w.p, w.dt, 1e-12, 1e-20)
    drift_t = np.array([abs(om.enthalpy(Tt[i], Yt[:, i]) - scale[i]) for i in range(8)]) / (np.abs(scale[:8]) + cpT)
    assert drift_t.max() <= 1e-11
    assert (Y >= 0).all()              # the positivity projection
    assert (T > w.T).mean() > 0.5       # these mixtures release heat


def test_integration_against_tight_reference(g10, g10_run):
    m, om = g10
    w, T, Y, st = g10_run
    Tt, Yt, _ = om.integrate(w.T[:12], w.Y[:, :12], w.p, w.dt, 1e-12, 1e-20)
    # global error of an rtol = 1e-8 run: a small multiple of rtol
    assert np.abs(Y[:, :12] - Yt).max() <= 1e-8
    assert (np.abs(T[:12] - Tt) / Tt).max() <= 3e-8
    T2, Y2, _ = om.integrate(w.T[:12], w.Y[:, :12], w.p, w.dt, 1e-6, 1e-12)
    e2 = np.abs(Y2 - Yt).max()
    e1 = np.abs(Y[:, :12] - Yt).max()
    assert e1 < e2 / 10                 # tighter tolerance, smaller error


def test_newton_matrix_reuse(g10, g10_run):
    """Keeping the factored Newton matrix while it is recent (the option)
    changes how Newton converges, not what it converges to: the result stays
    within a small multiple of rtol of the truth, like the fresh-every-attempt
    run (the default), while most attempts skip the Jacobian and the
    factorisation."""
    m, om = g10
    w, Tf0, Yf0, sf0 = g10_run
    idx = np.arange(0, 48, 3)
    Tt, Yt, _ = om.integrate(w.T[idx], w.Y[:, idx], w.p, w.dt, 1e-12, 1e-20)
    T, Y, st = om.integrate(w.T, w.Y, w.p, w.dt, w.rtol, w.atol, jac_reuse=True)
    Tf, Yf, sf = Tf0[idx], Yf0[:, idx], sf0[idx]
    assert (sf["n_jac"] == sf["attempts"]).all()
    for Ta, Ya in ((T[idx], Y[:, idx]), (Tf, Yf)):
        assert np.abs(Ya - Yt).max() <= 1e-7
        assert (np.abs(Ta - Tt) / Tt).max() <= 2e-7
    assert st["n_jac"][idx].sum() < 0.3 * st["attempts"][idx].sum()
    # linear invariants hold for any Jacobian with the same left null space
    # (exactly where the positivity projection never fired)
    dm = np.abs(Y[:, idx].sum(axis=0) - 1.0)
    clean = st["n_clip"][idx] == 0
    assert clean.any() and dm[clean].max() <= 1e-13 and dm.max() <= 1e-8


def test_q_max_two_also_converges(g10, g10_run):
    m, om = g10
    w, T, Y, st = g10_run
    T2, Y2, st2 = om.integrate(w.T[:8], w.Y[:, :8], w.p, w.dt, 1e-8, 1e-12, q_max=2)
    assert (st2["status"] == 0).all() and st2["steps"].mean() > st["steps"][:8].mean()
    assert np.abs(Y2 - Y[:, :8]).max() <= 2e-7


def test_radau_cross_check(g10):
    m, om = g10
    y0 = state(m, 1250.0, 42)
    dt = 1e-5

    def f(t, y):
        return om.rhs(y, P)

    def jac(t, y):
        return om.jac(y, P)

    sol = solve_ivp(f, (0, dt), y0, method="Radau", jac=jac, rtol=1e-12, atol=1e-16)
    T1, Y1, st = om.integrate(y0[-1:], y0[:-1, None], P, dt, 1e-10, 1e-16)
    assert sol.success and st[0]["status"] == 0
    yr = sol.y[:, -1]
    assert np.abs(Y1[:, 0] - yr[:-1]).max() <= 2e-8
    assert abs(T1[0] - yr[-1]) / yr[-1] <= 2e-8


@pytest.mark.parametrize("q,order", [(1, 1.0), (2, 2.0)])
def test_fixed_step_convergence_order(q, order):
    # A <-> B relaxation at fixed T has a closed form; fixed steps of h = dt/n
    m = mechs.isomer_pair(A=3e3, b=0.0, Ea=2.0, rev=True, dhf=3000.0)
    om = oracle.Mech(m.to_text())
    T, dt = 1000.0, 2e-4
    kf = mechs.kf_arrhenius(3e3, 0.0, 2.0, T)
    kr = kf * math.exp(3000.0 / (RU * T))
    Y0 = np.array([0.3, 0.0, 0.7])
    Yeq = Y0[0] * kr / (kf + kr)
    exact = Yeq + (Y0[0] - Yeq) * math.exp(-(kf + kr) * dt)
    errs, ns = [], [16, 32, 64, 128]
    for n in ns:
        _, Y1, st = om.integrate(np.array([T]), Y0[:, None], P, dt, 1e-8, 1e-14, q_max=q, fixed_T=True,
                                 fixed_step_n=n)
        assert st[0]["steps"] == n
        errs.append(abs(Y1[0, 0] - exact))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert abs(slope - order) < 0.15


def test_detailed_balance_at_long_times(g10):
    m, om = g10
    T = 2000.0
    y = state(m, T, 9, alpha=2.0)
    T1, Y1, st = om.integrate(np.array([T]), y[:-1, None], P, 5.0, 1e-11, 1e-22, fixed_T=True, max_steps=400000)
    assert st[0]["status"] == 0
    W = om.weights()
    Y = Y1[:, 0]
    rho = P * 10 / (RU * 1e7 * T) / np.sum(Y / W)
    C = rho * Y / W
    kf, kr, _, _ = om.rates(T, Y, P)
    nu = om.nu()
    checked = 0
    for j in range(om.R):
        sp = np.nonzero(nu[:, j])[0]
        if (C[sp] > 1e-15).all():            # concentrations resolved above atol
            lhs = nu[:, j] @ np.log(C)
            assert abs(lhs - math.log(kf[j] / kr[j])) <= 1e-6
            checked += 1
    assert checked >= 8


def test_failure_flags(g10):
    m, om = g10
    w = synth.uniform_batch(m, 4, 1001, 1000, 1600, 1e-5, 1e-8, 1e-12)
    T = w.T.copy()
    T[1] = float("nan")
    T[2] = -5.0
    T1, Y1, st = om.integrate(T, w.Y, w.p, w.dt, w.rtol, w.atol, max_steps=5)
    assert list(st["status"][1:3]) == [3, 3]
    assert st["status"][0] == 1 and st["attempts"][0] == 5      # max_steps exhausted
    assert np.isnan(T1[1]) and T1[2] == -5.0                     # bad cells left untouched
