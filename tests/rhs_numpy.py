"""A second, independent right-hand side in numpy (test helper).

It reads the mechanism from the generator's data classes (not from either
parser) and accepts complex states, so that complex-step differentiation of it
gives the Jacobian to rounding (Squire & Trapp).  It is compared with the
oracle's rhs value by value before its derivatives are trusted.
"""
import numpy as np

RU = 8.31446261815324
TREF = 298.15
PATM = 101325.0


def species_thermo(mech, T):
    """H, S, Cp per species (J/mol, J/(mol K)); complex T allowed."""
    S = mech.n_species
    a0, a1, hf, s0 = mech.a0, mech.a1, mech.hf, mech.s0
    H = hf + RU * (a0 * (T - TREF) + a1 * (T ** 2 - TREF ** 2) / 2)
    Sm = s0 + RU * (a0 * np.log(T / TREF) + a1 * (T - TREF))
    Cp = RU * (a0 + a1 * T)
    if mech.nasa is None:
        return H, Sm, Cp
    H = np.array(H, dtype=complex if np.iscomplexobj(T) else float)
    Sm = np.array(Sm, dtype=H.dtype)
    Cp = np.array(Cp, dtype=H.dtype)
    for k in range(S):
        if mech.nasa[k] is None:
            continue
        c = np.asarray(mech.nasa[k], dtype=float)
        a = c[1:8] if np.real(T) <= c[0] else c[8:15]
        powers = np.array([T ** i for i in range(5)])                 # 1, T, .., T^4
        Cp[k] = RU * np.dot(a[:5], powers)
        H[k] = RU * (np.dot(a[:5] / np.arange(1, 6), powers * T) + a[5])
        Sm[k] = RU * (a[0] * np.log(T) + np.dot(a[1:5] / np.arange(1, 5), powers[1:]) + a[6])
    return H, Sm, Cp


def troe_factor(troe, T, Pr):
    alpha, T3, T1 = troe[0], troe[1], troe[2]
    Fc = (1 - alpha) * np.exp(-T / T3) + alpha * np.exp(-T / T1)
    if len(troe) == 4:
        Fc = Fc + np.exp(-troe[3] / T)
    logFc = np.log10(Fc)
    c = -0.4 - 0.67 * logFc
    n = 0.75 - 1.27 * logFc
    x = np.log10(Pr) + c
    f1 = x / (n - 0.14 * x)
    return 10.0 ** (logFc / (1 + f1 * f1))


def rhs(mech, y, p, fixed_T=False):
    S = mech.n_species
    Y = y[:S]
    T = y[S]
    W = mech.atoms @ np.array([m for _, m in mech.elements])
    H, Sm, Cp = species_thermo(mech, T)
    G = H - T * Sm
    # density in g/cm^3 and concentrations in mol/cm^3
    Wbar = 1.0 / np.sum(Y / W)
    rho = p * 10.0 * Wbar / (RU * 1e7 * T)
    C = rho * Y / W
    M = np.sum(C)
    wdot = np.zeros(S, dtype=np.result_type(y, float))
    for r in mech.reactions:
        eps = np.ones(S)
        for k, e in (r.eff or {}).items():
            eps[k] = e
        Mr = np.dot(eps, C)
        kinf = r.A * T ** r.b * np.exp(-r.Ea * 4184.0 / (RU * T))
        kf = kinf
        if r.kind == 2:
            A0, b0, Ea0 = r.low
            k0 = A0 * T ** b0 * np.exp(-Ea0 * 4184.0 / (RU * T))
            Pr = k0 * Mr / kinf
            kf = kinf * Pr / (1 + Pr)
            if r.troe is not None:
                kf = kf * troe_factor(r.troe, T, Pr)
        pf = np.prod([C[i] for i in r.reactants])
        pr = np.prod([C[i] for i in r.products])
        if r.reversible:
            nu = np.zeros(S)
            for i in r.reactants:
                nu[i] -= 1
            for i in r.products:
                nu[i] += 1
            # equilibrium constant in pressure units, converted to mol/cm^3
            Kp = np.exp(-np.sum(nu * G) / (RU * T))
            Kc = Kp * (PATM / (RU * T) * 1e-6) ** np.sum(nu)
            q = kf * pf - kf / Kc * pr
        else:
            q = kf * pf
        if r.kind == 1:
            q = q * Mr
        for i in r.reactants:
            wdot[i] -= q
        for i in r.products:
            wdot[i] += q
    f = np.zeros(S + 1, dtype=np.result_type(y, float))
    f[:S] = W * wdot / rho
    f[S] = 0.0 if fixed_T else -np.sum(H * wdot) / np.sum(C * Cp)
    return f


def rhs_qss(mech, y, p, fixed_T=False):
    """Reduced right-hand side with quasi-steady-state species (y = Y of the
    transported species, then T).  Directions with two or more QSS species
    among their reactants are dropped.  With those gone the QSS production
    rates are affine in the QSS concentrations, so the closure matrix and
    vector are read off numerically: b0 = wdot_Q(C_Q = 0) and
    A[:, n] = wdot_Q(C_Q = e_n) - b0; then C_Q = -A^-1 b0.  [M] sums the
    transported species only."""
    S = mech.n_species
    qs = list(mech.qss)
    ts = mech.transported
    T = y[-1]
    Yt = y[:-1]
    W = mech.atoms @ np.array([m for _, m in mech.elements])
    H, Sm, Cp = species_thermo(mech, T)
    G = H - T * Sm
    Wbar = 1.0 / np.sum(Yt / W[ts])
    rho = p * 10.0 * Wbar / (RU * 1e7 * T)
    dt = np.result_type(y, float)
    C = np.zeros(S, dtype=dt)
    C[ts] = rho * Yt / W[ts]
    isq = np.zeros(S, dtype=bool)
    isq[qs] = True
    consts = []
    for r in mech.reactions:
        eps = np.ones(S)
        for k, e in (r.eff or {}).items():
            eps[k] = e
        eps[qs] = 0.0
        Mr = np.dot(eps, C)
        kinf = r.A * T ** r.b * np.exp(-r.Ea * 4184.0 / (RU * T))
        kf = kinf
        if r.kind == 2:
            A0, b0_, Ea0 = r.low
            k0 = A0 * T ** b0_ * np.exp(-Ea0 * 4184.0 / (RU * T))
            Pr = k0 * Mr / kinf
            kf = kinf * Pr / (1 + Pr)
            if r.troe is not None:
                kf = kf * troe_factor(r.troe, T, Pr)
        nu = np.zeros(S)
        for i in r.reactants:
            nu[i] -= 1
        for i in r.products:
            nu[i] += 1
        kr = 0.0
        if r.reversible:
            Kc = np.exp(-np.sum(nu * G) / (RU * T)) * (PATM / (RU * T) * 1e-6) ** np.sum(nu)
            kr = kf / Kc
        keep_f = sum(isq[i] for i in r.reactants) < 2
        keep_r = r.reversible and sum(isq[i] for i in r.products) < 2
        consts.append((nu, kf if keep_f else 0.0, kr if keep_r else 0.0, Mr if r.kind == 1 else 1.0))

    def wdot_all(Cv):
        wd = np.zeros(S, dtype=np.result_type(Cv, float))
        for r, (nu, kf, kr, mf) in zip(mech.reactions, consts):
            q = kf * np.prod([Cv[i] for i in r.reactants]) - kr * np.prod([Cv[i] for i in r.products])
            wd = wd + nu * (mf * q)
        return wd

    nq = len(qs)
    C0 = C.copy()
    b0 = wdot_all(C0)[qs]
    A = np.zeros((nq, nq), dtype=np.result_type(b0, float))
    for n in range(nq):
        Cn = C0.copy()
        Cn[qs[n]] = 1.0
        A[:, n] = wdot_all(Cn)[qs] - b0
    C[qs] = np.linalg.solve(A, -b0)
    wd = wdot_all(C)
    f = np.zeros(len(ts) + 1, dtype=np.result_type(y, float))
    f[:-1] = W[ts] * wd[ts] / rho
    f[-1] = 0.0 if fixed_T else -np.sum(H[ts] * wd[ts]) / np.sum(C[ts] * Cp[ts])
    return f


def jac_complex_step(mech, y, p, fixed_T=False, h=1e-30, fn=None):
    """J[i, j] = Im f(y + i h e_j) / h (|h| * |y| far below rounding)."""
    fn = fn or (rhs_qss if getattr(mech, "qss", None) else rhs)
    n = y.shape[0]
    J = np.zeros((n, n))
    for j in range(n):
        yc = y.astype(complex)
        step = h * max(1.0, abs(y[j]))
        yc[j] += 1j * step
        J[:, j] = fn(mech, yc, p, fixed_T).imag / step
    return J
