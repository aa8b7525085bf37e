"""Seeded synthetic inputs: mechanisms and per-cell reactor states.

This module is shared by the GPU library's tests/bench and by the CPU oracle's
tests.  It holds none of the integration method's arithmetic: it draws random
numbers, checks integer atom balance while drawing reactions, and writes the
mechanism text format that both sides parse on their own.

Mechanism generator G(S, R, E, seed)
-------------------------------------
The paper states the kinetics only as a mechanism of N species and M
reactions with forward/backward stoichiometric coefficients (Sec. 2.1, Eq. 1)
and rates of progress built from rate constants (Eq. 2); its own mechanisms
(n-dodecane, methane, n-heptane) are not available, so a synthetic family of
the same structure stands in:

* E elements taken in the order H, C, O, N (masses in g/mol).
* S species; atom counts per element drawn uniformly from {0..3}, an all-zero
  vector is redrawn.  The last species (index S-1) is inert: it takes part in
  no reaction but collides as a third body.
* Linear heat capacity per species, cp/R = a0 + a1*T, a0 ~ U[2.5, 6],
  a1 ~ U[0, 1e-3] 1/K; formation enthalpy h_f ~ U[-3e5, 3e5] J/mol and
  standard entropy s0 ~ U[150, 250] J/(mol K), both at 298.15 K.
* R reversible reactions with 1-2 reactants and 1-2 products drawn from the
  reactive species (repeats allowed, e.g. 2A), atom balanced.  All balanced
  candidate reactions are enumerated; if fewer than R exist the whole species
  set is redrawn from the same stream.  R distinct candidates are picked
  without replacement and each is oriented by a fair coin.
* log10 A ~ U[8, 14] (mol, cm, s units), b ~ U[-1, 2], Ea ~ U[0, 40] kcal/mol.
* Exactly round(0.2 R) reactions, picked uniformly, are third-body reactions
  with unit efficiencies for every species.

Mechanism text format (version 1), one record per line, '#' starts a comment::

    chem-mech 1
    ELEMENTS <E>
    <symbol> <mass g/mol>                                  (E lines)
    SPECIES <S>
    <name> <inert 0|1> <n_e0> .. <n_e(E-1)> <a0> <a1> <hf J/mol> <s0 J/mol/K>
      or
    <name> <inert 0|1> <n_e0> .. <n_e(E-1)> NASA7 <T_mid> <c1..c7 for T <= T_mid> <c1..c7 above>
    REACTIONS <R>
    <rev 0|1> <type 0|1|2> <nr> <r_1..r_nr> <np> <p_1..p_np> <A> <b> <Ea kcal/mol> [<A0> <b0> <Ea0>]
        [TROE <3|4> <alpha> <T3> <T1> [<T2>]] [EFF <n> <k_1> <eps_1> .. <k_n> <eps_n>]
    END

type 0 = elementary, 1 = third body (+M), 2 = falloff (+M) whose
low-pressure limit (A0, b0, Ea0) follows (Lindemann form, times Troe's
broadening factor when TROE follows; T3, T1, T2 are CHEMKIN's T***, T*, T**).
EFF lists collision efficiencies other than 1 in [M] for types 1 and 2.
An optional record `QSS <n> <k_1> .. <k_n>` before END names the species
treated as quasi-steady (algebraic; the state holds the others in order).
NASA7 gives CHEMKIN's 7-coefficient polynomials in two ranges split at T_mid.  Reactant and
product lists hold 0-based species indices, a repeated index meaning a
stoichiometric coefficient of 2 (at most 3 entries per side).  Floats are
written with 17 significant digits so that every parser reads back the same
doubles.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ELEMENT_TABLE: Tuple[Tuple[str, float], ...] = (
    ("H", 1.008), ("C", 12.011), ("O", 15.999), ("N", 14.007))

P_ATM = 101325.0  # Pa


@dataclasses.dataclass
class Reaction:
    reactants: List[int]
    products: List[int]
    A: float
    b: float
    Ea: float                 # kcal/mol
    reversible: bool = True
    kind: int = 0             # 0 elementary, 1 third body, 2 falloff (Lindemann, or Troe with `troe`)
    low: Optional[Tuple[float, float, float]] = None   # (A0, b0, Ea0 kcal/mol)
    troe: Optional[Tuple[float, ...]] = None           # (alpha, T3, T1[, T2]) of a Troe falloff
    eff: Optional[Dict[int, float]] = None             # collision efficiencies other than 1


@dataclasses.dataclass
class Mechanism:
    elements: List[Tuple[str, float]]
    names: List[str]
    atoms: np.ndarray         # [S, E] int
    a0: np.ndarray
    a1: np.ndarray
    hf: np.ndarray
    s0: np.ndarray
    inert: np.ndarray         # [S] bool
    reactions: List[Reaction]
    label: str = ""
    nasa: Optional[List[Optional[Tuple[float, ...]]]] = None   # per species: (T_mid, 7 low, 7 high) or None
    qss: Optional[List[int]] = None     # quasi-steady-state species (algebraic, not in the state)

    @property
    def transported(self) -> List[int]:
        """Species of the integrated state, in order (all but the QSS ones)."""
        q = set(self.qss or [])
        return [k for k in range(self.n_species) if k not in q]

    @property
    def n_state_species(self) -> int:
        return self.n_species - len(self.qss or [])

    @property
    def n_species(self) -> int:
        return len(self.names)

    @property
    def n_reactions(self) -> int:
        return len(self.reactions)

    def to_text(self) -> str:
        return write_mechanism(self)


def _f(x: float) -> str:
    return repr(float(x)) if math.isfinite(x) else "nan"


def write_mechanism(m: Mechanism) -> str:
    out = [f"chem-mech 1", f"# {m.label}" if m.label else "# synthetic mechanism",
           f"ELEMENTS {len(m.elements)}"]
    for sym, mass in m.elements:
        out.append(f"{sym} {_f(mass)}")
    out.append(f"SPECIES {m.n_species}")
    for k, name in enumerate(m.names):
        atoms = " ".join(str(int(v)) for v in m.atoms[k])
        if m.nasa is not None and m.nasa[k] is not None:
            out.append(f"{name} {int(bool(m.inert[k]))} {atoms} NASA7 " + " ".join(_f(v) for v in m.nasa[k]))
            continue
        out.append(f"{name} {int(bool(m.inert[k]))} {atoms} {_f(m.a0[k])} {_f(m.a1[k])} "
                   f"{_f(m.hf[k])} {_f(m.s0[k])}")
    out.append(f"REACTIONS {m.n_reactions}")
    for r in m.reactions:
        fields = [str(int(r.reversible)), str(int(r.kind)), str(len(r.reactants))]
        fields += [str(int(i)) for i in r.reactants]
        fields += [str(len(r.products))] + [str(int(i)) for i in r.products]
        fields += [_f(r.A), _f(r.b), _f(r.Ea)]
        if r.kind == 2:
            assert r.low is not None
            fields += [_f(v) for v in r.low]
            if r.troe is not None:
                fields += ["TROE", str(len(r.troe))] + [_f(v) for v in r.troe]
        if r.eff:
            assert r.kind in (1, 2)
            fields += ["EFF", str(len(r.eff))]
            for k in sorted(r.eff):
                fields += [str(int(k)), _f(r.eff[k])]
        out.append(" ".join(fields))
    if m.qss:
        out.append(f"QSS {len(m.qss)} " + " ".join(str(int(k)) for k in m.qss))
    out.append("END")
    return "\n".join(out) + "\n"


def _balanced_pool(atoms: np.ndarray, reactive: int) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """All unordered pairs {left side, right side} of 1-2 reactive species with
    equal integer atom vectors and different multisets."""
    sides: List[Tuple[int, ...]] = [(i,) for i in range(reactive)]
    sides += [(i, j) for i in range(reactive) for j in range(i, reactive)]
    groups = {}
    for s in sides:
        key = tuple(int(v) for v in atoms[list(s)].sum(axis=0))
        groups.setdefault(key, []).append(s)
    pool = []
    for key in sorted(groups):
        members = groups[key]
        for a in range(len(members)):
            for b in range(a + 1, len(members)):
                pool.append((members[a], members[b]))
    return pool


def make_mechanism(S: int, R: int, E: int, seed: int, max_redraws: int = 1000) -> Mechanism:
    """G(S, R, E, seed): see the module docstring for the recipe and draw order."""
    if not (2 <= S <= 63 and 1 <= E <= len(ELEMENT_TABLE) and R >= 1):
        raise ValueError("unsupported G(S,R,E)")
    rng = np.random.default_rng(seed)
    elements = list(ELEMENT_TABLE[:E])
    for _attempt in range(max_redraws):
        atoms = np.zeros((S, E), dtype=np.int64)
        for k in range(S):
            while True:
                v = rng.integers(0, 4, size=E)
                if v.sum() > 0:
                    break
            atoms[k] = v
        pool = _balanced_pool(atoms, S - 1)
        if len(pool) >= R:
            break
    else:
        raise RuntimeError(f"G({S},{R},{E},{seed}): no balanced reaction set after {max_redraws} redraws")
    a0 = rng.uniform(2.5, 6.0, size=S)
    a1 = rng.uniform(0.0, 1e-3, size=S)
    hf = rng.uniform(-3e5, 3e5, size=S)
    s0 = rng.uniform(150.0, 250.0, size=S)
    pick = rng.choice(len(pool), size=R, replace=False)
    flip = rng.integers(0, 2, size=R)
    log10A = rng.uniform(8.0, 14.0, size=R)
    b = rng.uniform(-1.0, 2.0, size=R)
    Ea = rng.uniform(0.0, 40.0, size=R)
    n_tb = int(round(0.2 * R))
    tb = set(int(i) for i in rng.choice(R, size=n_tb, replace=False))
    reactions = []
    for j in range(R):
        left, right = pool[int(pick[j])]
        if flip[j]:
            left, right = right, left
        reactions.append(Reaction(list(left), list(right), float(10.0 ** log10A[j]),
                                  float(b[j]), float(Ea[j]), True, 1 if j in tb else 0))
    inert = np.zeros(S, dtype=bool)
    inert[S - 1] = True
    names = [f"S{k}" for k in range(S - 1)] + ["INERT"]
    return Mechanism(elements, names, atoms, a0, a1, hf, s0, inert, reactions,
                     label=f"G({S},{R},{E},seed {seed})")


# ------------------------------------------- real-mechanism features (f4) ----

TREF = 298.15
EFF_CHOICES = (0.0, 0.4, 0.7, 2.0, 5.0, 12.0)


def nasa7_from_linear(a0: float, a1: float, hf: float, s0: float, c3: float, c4: float, c5: float,
                      delta: float, t_mid: float = 1000.0) -> Tuple[float, ...]:
    """NASA 7-coefficient thermo whose low-range cp/R is a0 + a1 T + c3 T^2 +
    c4 T^3 + c5 T^4, anchored at h_f and s0 (298.15 K), and whose high range
    adds delta (T - t_mid)^2 to cp/R, with the enthalpy and entropy constants
    chosen so that cp, H and S are continuous at t_mid.  Polynomial bookkeeping
    on the coefficient vectors (numpy.polynomial), written once here for the
    inputs."""
    P = np.polynomial.polynomial
    ru = 8.31446261815324
    cp_lo = np.array([a0, a1, c3, c4, c5])
    # H/R = int cp/R dT + c6;   S/R = c1 ln T + int (cp/R - c1)/T dT + c7
    h_poly = P.polyint(cp_lo)                      # zero constant term
    s_poly = P.polyint(cp_lo[1:])                  # of (cp/R - c1)/T
    c6 = hf / ru - P.polyval(TREF, h_poly)
    c7 = s0 / ru - (cp_lo[0] * math.log(TREF) + P.polyval(TREF, s_poly))
    shift = delta * np.array([t_mid * t_mid, -2.0 * t_mid, 1.0, 0.0, 0.0])   # delta (T - t_mid)^2
    cp_hi = cp_lo + shift
    h_hi = P.polyint(cp_hi)
    s_hi = P.polyint(cp_hi[1:])
    c6_hi = (P.polyval(t_mid, h_poly) + c6) - P.polyval(t_mid, h_hi)
    c7_hi = (cp_lo[0] * math.log(t_mid) + P.polyval(t_mid, s_poly) + c7) - \
        (cp_hi[0] * math.log(t_mid) + P.polyval(t_mid, s_hi))
    return (float(t_mid), *map(float, cp_lo), float(c6), float(c7), *map(float, cp_hi), float(c6_hi), float(c7_hi))


def make_real_mechanism(S: int, R: int, E: int, seed: int, troe_fraction: float = 0.1) -> Mechanism:
    """G(S,R,E,seed) with the features of real (CHEMKIN/Cantera) mechanisms
    added from a second stream seeded seed + 7919, leaving G's own draws as
    they are:

    * every species gets NASA 7-coefficient thermo: the low range adds
      c3 T^2 + c4 T^3 + c5 T^4 (c3 ~ U[-5e-8, 5e-8], c4 ~ U[-5e-12, 5e-12],
      c5 ~ U[-5e-16, 5e-16]) to G's linear cp/R, the range splits at 1000 K,
      and the high range adds delta (T - 1000)^2 with delta ~ U[-1e-7, 1e-7],
      continuous in cp, H and S;
    * round(troe_fraction R) elementary reactions become Troe falloff
      reactions: A0 = A 10^U[3,7], b0 ~ U[-2, 0], Ea0 = Ea U[0, 1]; alpha ~
      U[0.1, 0.9], T3 ~ U[30, 500] K, T1 ~ U[500, 5000] K, and with
      probability 1/2 T2 ~ U[1000, 8000] K;
    * every third-body and falloff reaction lists efficiencies for 3 distinct
      species drawn uniformly, each from {0, 0.4, 0.7, 2, 5, 12}."""
    m = make_mechanism(S, R, E, seed)
    rng = np.random.default_rng(seed + 7919)
    nasa = []
    for k in range(S):
        c3, c4, c5 = rng.uniform(-5e-8, 5e-8), rng.uniform(-5e-12, 5e-12), rng.uniform(-5e-16, 5e-16)
        delta = rng.uniform(-1e-7, 1e-7)
        nasa.append(nasa7_from_linear(m.a0[k], m.a1[k], m.hf[k], m.s0[k], c3, c4, c5, delta))
    m.nasa = nasa
    elementary = [j for j, r in enumerate(m.reactions) if r.kind == 0]
    n_troe = min(len(elementary), int(round(troe_fraction * R)))
    troe_ids = sorted(int(j) for j in rng.choice(elementary, size=n_troe, replace=False)) if n_troe else []
    for j in troe_ids:
        r = m.reactions[j]
        r.kind = 2
        r.low = (float(r.A * 10.0 ** rng.uniform(3.0, 7.0)), float(rng.uniform(-2.0, 0.0)),
                 float(r.Ea * rng.uniform(0.0, 1.0)))
        troe = [float(rng.uniform(0.1, 0.9)), float(rng.uniform(30.0, 500.0)), float(rng.uniform(500.0, 5000.0))]
        if rng.uniform() < 0.5:
            troe.append(float(rng.uniform(1000.0, 8000.0)))
        r.troe = tuple(troe)
    for r in m.reactions:
        if r.kind in (1, 2):
            ks = rng.choice(S, size=min(3, S), replace=False)
            r.eff = {int(k): float(EFF_CHOICES[int(rng.integers(0, len(EFF_CHOICES)))]) for k in ks}
    m.label = f"G_real({S},{R},{E},seed {seed})"
    return m


# ------------------------------------------- quasi-steady-state species (f3) ----

def _qss_branching(r: Reaction, qss: set) -> bool:
    """A direction of r with exactly one QSS reactant yields two or more QSS
    species (integer bookkeeping on the reaction lists)."""
    sides = [(r.reactants, r.products)] + ([(r.products, r.reactants)] if r.reversible else [])
    return any(sum(i in qss for i in rs) == 1 and sum(i in qss for i in ps) >= 2 for rs, ps in sides)


def _qss_leaks(reactions: List[Reaction], qss: set) -> bool:
    """Every QSS species is consumed by some direction with it as the only
    QSS reactant and no QSS product."""
    leak = {k: False for k in qss}
    for r in reactions:
        sides = [(r.reactants, r.products)] + ([(r.products, r.reactants)] if r.reversible else [])
        for rs, ps in sides:
            qr = [i for i in rs if i in qss]
            if len(qr) == 1 and not any(i in qss for i in ps):
                leak[qr[0]] = True
    return all(leak.values())


def make_qss_mechanism(S: int, R: int, E: int, seed: int, n_qss: int, speedup: float = 1e2,
                       dh_f: float = 1.5e5, max_draws: int = 200) -> Mechanism:
    """G(S,R,E,seed) with n_qss of its reactive species made quasi-steady
    (the paper's reduced mechanisms are not available, so a selection rule on
    the synthetic family stands in).  From a second stream seeded
    seed + 104729: n_qss species are drawn uniformly among the reactive
    species that take part in at least two reactions.  Reactions with a
    direction that turns one QSS species into two are removed (kept, they
    can make the closure singular); the draw is repeated until every QSS
    species keeps a direction that consumes it into transported species
    only.  With that, every column of the closure matrix is diagonally
    dominant, so the closure is regular at every state.  Each chosen species'
    formation enthalpy is raised by dh_f J/mol (a short-lived,
    low-concentration intermediate), and the pre-exponential factor of every
    reaction involving one is multiplied by `speedup` (fast).  Reactions with
    two QSS species on one side stay: their quadratic couplings are left to
    the one-sided linearisation."""
    m = make_mechanism(S, R, E, seed)
    rng = np.random.default_rng(seed + 104729)
    count = np.zeros(S, dtype=int)
    for r in m.reactions:
        for k in set(r.reactants) | set(r.products):
            count[k] += 1
    cand = [k for k in range(S - 1) if count[k] >= 2]
    if len(cand) < n_qss:
        raise ValueError("not enough QSS candidates")
    for _ in range(max_draws):
        pick = set(int(k) for k in rng.choice(cand, size=n_qss, replace=False))
        kept = [r for r in m.reactions if not _qss_branching(r, pick)]
        if _qss_leaks(kept, pick):
            break
    else:
        raise RuntimeError("no admissible QSS set")
    m.reactions = kept
    m.qss = sorted(pick)
    m.hf = m.hf.copy()
    for k in m.qss:
        m.hf[k] += dh_f
    for r in m.reactions:
        if pick & (set(r.reactants) | set(r.products)):
            r.A *= speedup
    m.label = f"G_qss({S},{R},{E},seed {seed},{n_qss} QSS; {len(m.reactions)} reactions kept)"
    return m


# ---------------------------------------------------------------- states ----

def composition(rng: np.random.Generator, S: int, alpha: float, n: int = 1,
                inert_fraction: float = 0.7) -> np.ndarray:
    """[S, n] mass fractions: the inert species holds `inert_fraction`, the
    reactive species share the rest by a Dirichlet(alpha) draw per column; a
    final division by the column sum only removes rounding."""
    Y = np.empty((S, n))
    d = rng.dirichlet(np.full(S - 1, alpha), size=n).T     # [S-1, n]
    Y[:S - 1] = (1.0 - inert_fraction) * d
    Y[S - 1] = inert_fraction
    Y /= Y.sum(axis=0, keepdims=True)
    return Y


@dataclasses.dataclass
class Workload:
    """One batch of reactor cells (SoA: Y[k, i] species-major)."""
    mech: Mechanism
    T: np.ndarray           # [n]
    Y: np.ndarray           # [S, n]
    p: float
    dt: float
    rtol: float
    atol: float
    name: str = ""
    shape: Optional[Tuple[int, ...]] = None

    @property
    def n_cells(self) -> int:
        return int(self.T.shape[0])


def uniform_batch(mech: Mechanism, n: int, seed: int, T_lo: float, T_hi: float,
                  dt: float, rtol: float, atol: float, alpha: float = 1.0,
                  name: str = "") -> Workload:
    """n cells with T ~ U[T_lo, T_hi] and Y = 0.7 inert + 0.3 Dirichlet(alpha)."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(T_lo, T_hi, size=n)
    Y = composition(rng, mech.n_species, alpha, n)
    return Workload(mech, T, np.ascontiguousarray(Y), P_ATM, dt, rtol, atol, name=name)


def flame_profile(mech: Mechanism, shape: Tuple[int, int, int], seed: int, Y_eq: np.ndarray,
                  dt: float, rtol: float, atol: float, name: str = "",
                  x_centre: float = 128.0, width: float = 8.0, noise_K: float = 5.0) -> Workload:
    """A planar tanh flame through a box of nx*ny*nz cells.

    x is the integer index along the longest (slowest-varying) axis, the cell
    order being i = z + nz*(y + ny*x).  w = (1 + tanh((x - x_centre)/width))/2,
    T = 300 + 1900 w + N(0, noise_K) per cell, Y = (1 - w) Y_cold + w Y_eq
    where Y_cold is one Dirichlet(2) draw over the reactive species with 0.7
    inert (drawn first from the stream) and Y_eq is the equilibrium
    composition supplied by the caller."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    Y_cold = cold_mixture(rng, mech.n_species)
    n = nx * ny * nz
    x = np.repeat(np.arange(nx, dtype=np.float64), ny * nz)
    w = 0.5 * (1.0 + np.tanh((x - x_centre) / width))
    T = 300.0 + 1900.0 * w + rng.normal(0.0, noise_K, size=n)
    Y = (1.0 - w)[None, :] * Y_cold[:, None] + w[None, :] * np.asarray(Y_eq, dtype=np.float64)[:, None]
    return Workload(mech, T, np.ascontiguousarray(Y), P_ATM, dt, rtol, atol, name=name, shape=shape)


def cold_mixture(rng: np.random.Generator, S: int) -> np.ndarray:
    """The unburnt mixture of the flame profile: 0.7 inert + 0.3 Dirichlet(2)."""
    return composition(rng, S, 2.0, 1)[:, 0]


@dataclasses.dataclass
class Box:
    L: int
    T: np.ndarray
    Y: np.ndarray
    dt: float


def amr_boxes(mech: Mechanism, n_boxes: int, seed: int, L_lo: int = 8, L_hi: int = 64,
              T_lo: float = 900.0, T_hi: float = 2300.0, noise_K: float = 20.0,
              dt_lo: float = 1e-7, dt_hi: float = 1e-5, max_cells: Optional[int] = None) -> List[Box]:
    """Uneven cubic boxes: edge L = round(exp(U[ln L_lo, ln L_hi])); per box a
    temperature T_b ~ U[T_lo, T_hi] plus N(0, noise_K) per cell, one
    Dirichlet(1) composition with 0.7 inert, and dt_b log-uniform in
    [dt_lo, dt_hi].  `max_cells` caps each box (for scaled-down runs)."""
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(n_boxes):
        L = int(round(math.exp(rng.uniform(math.log(L_lo), math.log(L_hi)))))
        n = L ** 3
        if max_cells is not None:
            n = min(n, max_cells)
        Tb = rng.uniform(T_lo, T_hi)
        Yb = composition(rng, mech.n_species, 1.0, 1)[:, 0]
        dtb = math.exp(rng.uniform(math.log(dt_lo), math.log(dt_hi)))
        T = Tb + rng.normal(0.0, noise_K, size=n)
        Y = np.ascontiguousarray(np.repeat(Yb[:, None], n, axis=1))
        boxes.append(Box(L, T, Y, dtb))
    return boxes


def poisson_trace(seed: int, rate_hz: float, duration_s: float) -> np.ndarray:
    """Open-loop arrival times (s) with exponential inter-arrival gaps."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out)


# --------------------------------------------------------- named configs ----

CONFIG_MECH = {
    1: (10, 25, 3, 0),
    2: (10, 25, 3, 1),
    3: (53, 325, 4, 2),
    4: (30, 180, 4, 3),
}


def config_mechanism(cfg: int) -> Mechanism:
    return make_mechanism(*CONFIG_MECH[cfg])


def config_seed(cfg: int) -> int:
    return 1000 + cfg


def load_composition_file(path: str) -> np.ndarray:
    """Read a composition written one value per line ('#' comments)."""
    vals = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                vals.append(float(line))
    return np.asarray(vals)


def config_workload(cfg: int, yeq_dir: Optional[str] = None, shape: Optional[Tuple[int, int, int]] = None,
                    n: Optional[int] = None) -> Workload:
    """The named workloads (cell counts can be reduced with `shape`/`n`):

    1: G(10,25,3,s0), 4096 cells, T ~ U[1000,1600], Dirichlet(1) + 0.7 inert,
       dt 1e-5 s, rtol 1e-8, atol 1e-12
    2: G(10,25,3,s1) planar flame in a 64x64x256 box (x = the 256 axis),
       dt 2e-6 s, rtol 1e-8, atol 1e-12
    3: G(53,325,4,s2) planar flame in a 16x64x256 box, dt 1e-6 s, rtol 1e-6,
       atol 1e-12
    """
    m = config_mechanism(cfg)
    seed = config_seed(cfg)
    if cfg == 1:
        return uniform_batch(m, n or 4096, seed, 1000.0, 1600.0, 1e-5, 1e-8, 1e-12, name="config1")
    if cfg in (2, 3):
        if yeq_dir is None:
            raise ValueError("flame workloads need the directory of the equilibrium composition files")
        S, R, E, s = CONFIG_MECH[cfg]
        Yeq = load_composition_file(f"{yeq_dir}/yeq_G{S}_{R}_{E}_s{s}.txt")
        if cfg == 2:
            shape = shape or (256, 64, 64)
            return flame_profile(m, shape, seed, Yeq, 2e-6, 1e-8, 1e-12, name="config2")
        shape = shape or (256, 64, 16)
        return flame_profile(m, shape, seed, Yeq, 1e-6, 1e-6, 1e-12, name="config3")
    raise ValueError(f"no batch workload for config {cfg}")
