"""Tiny hand-written mechanisms for closed-form tests (built with the shared
generator's data classes, so both sides read them through the text format)."""
import numpy as np

from paper_2405_05974_amd import synth

RU = 8.31446261815324
KCAL = 4184.0


def tiny(species, reactions, elements=(("H", 1.008), ("C", 12.011))):
    """species: list of (name, atoms tuple, a0, a1, hf, s0, inert)."""
    names = [s[0] for s in species]
    atoms = np.array([s[1] for s in species], dtype=np.int64)
    a0 = np.array([s[2] for s in species], dtype=float)
    a1 = np.array([s[3] for s in species], dtype=float)
    hf = np.array([s[4] for s in species], dtype=float)
    s0 = np.array([s[5] for s in species], dtype=float)
    inert = np.array([s[6] for s in species], dtype=bool)
    return synth.Mechanism(list(elements), names, atoms, a0, a1, hf, s0, inert, reactions, label="tiny")


def isomer_pair(A=1e6, b=0.5, Ea=5.0, rev=False, kind=0, low=None, dhf=0.0, a1=2e-4):
    """A <-> B isomers (same atoms, cp and s0) plus an inert diluent."""
    sp = [("A", (2, 1), 3.5, a1, 1000.0, 200.0, False),
          ("B", (2, 1), 3.5, a1, 1000.0 + dhf, 200.0, False),
          ("N", (0, 2), 3.0, 1e-4, 0.0, 190.0, True)]
    rx = [synth.Reaction([0], [1], A, b, Ea, rev, kind, low)]
    return tiny(sp, rx)


def kf_arrhenius(A, b, Ea_kcal, T):
    return A * T ** b * np.exp(-Ea_kcal * KCAL / (RU * T))


def mixed_kinds():
    """Five species, four reactions: Lindemann falloff, third body, an
    irreversible 2B -> 2A, and a three-reactant reaction; dnu != 0 included."""
    sp = [("A", (2, 1), 3.5, 2e-4, 1000.0, 200.0, False),
          ("B", (2, 1), 3.9, 1e-4, -20000.0, 210.0, False),
          ("C", (1, 1), 4.1, 3e-4, 50000.0, 180.0, False),
          ("D", (1, 0), 2.6, 1e-5, 200000.0, 160.0, False),
          ("N", (0, 2), 3.0, 1e-4, 0.0, 190.0, True)]
    rx = [synth.Reaction([0], [1], 1e9, 0.2, 12.0, True, 2, (1e15, -0.5, 8.0)),
          synth.Reaction([2, 3], [0], 1e12, 0.0, 3.0, True, 1),
          synth.Reaction([1, 1], [0, 0], 1e10, 0.5, 20.0, False, 0),
          synth.Reaction([2, 3, 3], [1, 3], 1e16, -1.0, 1.0, True, 0)]
    return tiny(sp, rx)


def qss_tiny(low=(1e16, 0.0, 2.0), speed=1.0, coupling=True, dh_qss=0.0, third=False):
    """Six transported species, two QSS species X and Y and an inert, over
    the elements H and C, built so that every part of the closure is
    exercised: a QSS group of two (X and Y turn into each other through
    reactions 3, 4, 5 and 7), leaks of X (8, a falloff reaction with
    efficiencies) and of Y (9), a direction producing two QSS species (2),
    a quadratic coupling X + Y (6, forward direction removed by the one-sided
    linearisation) and a third-body reaction with efficiencies (10).  `speed`
    multiplies the pre-exponential factor of every reaction of X or Y: their
    concentrations stay, their relaxation times shrink.  coupling=False
    replaces reaction 2 by A + C = X + E and leaves out reaction 6: no
    quadratic coupling, nothing linearised (and X, Y do not collide).
    dh_qss raises the formation enthalpies of X and Y (J/mol): less stable,
    scarcer and shorter-lived, while the flux through them stays.
    third=True adds a third QSS species Z, made from X (X + B -> Z) and
    leaking into A + Z = C + E: a group of its own that depends on the X, Y
    group; it is listed first in the QSS record, so its solve order comes
    from the dependencies, not from the record."""
    sp = [("A", (2, 0), 3.5, 2e-4, 0.0, 130.0, False),
          ("B", (0, 2), 3.6, 1e-4, 0.0, 200.0, False),
          ("C", (1, 1), 4.0, 2e-4, 40000.0, 200.0, False),
          ("D", (2, 2), 5.5, 3e-4, 20000.0, 230.0, False),
          ("E", (2, 1), 4.8, 2e-4, 60000.0, 220.0, False),
          ("X", (1, 0), 2.5, 0.0, 218000.0 + dh_qss, 115.0, False),
          ("Y", (0, 1), 2.5, 1e-5, 300000.0 + dh_qss, 158.0, False),
          ("N", (0, 3), 3.5, 1e-4, 0.0, 190.0, True)]
    A, B, C, D, E, X, Y = range(7)
    R = synth.Reaction
    rx = [R([A, B], [C, C], 1e11, 0.0, 20.0),
          R([A], [X, X], 1e11, 0.0, 60.0),
          R([X, B], [C, Y], 2e13, 0.0, 4.0),
          R([Y, A], [C, X], 1e13, 0.5, 6.0),
          R([X, C], [A, Y], 5e12, 0.0, 8.0),
          R([X, Y], [C], 1e13, 0.0, 0.0),
          R([X, D], [A, C, Y], 1e12, 0.0, 3.0),
          R([X, C], [E], 3e12, 0.0, 1.0, True, 2, low),
          R([Y, E], [D], 2e13, 0.0, 2.0),
          R([C, C], [D], 1e14, -0.5, 0.0, True, 1)]
    rx[7].troe = (0.5, 200.0, 2000.0)
    rx[7].eff = {B: 2.5, D: 0.0}
    rx[9].eff = {A: 2.0, X: 5.0}
    for r in rx:
        if X in r.reactants + r.products or Y in r.reactants + r.products:
            r.A *= speed
            if r.low is not None:
                r.low = (r.low[0] * speed, r.low[1], r.low[2])
    if third:
        sp.insert(7, ("Z", (1, 2), 3.0, 1e-4, 150000.0, 200.0, False))
        rx += [R([X, B], [7], 3e12, 0.0, 2.0, False), R([7, A], [C, E], 1e13, 0.0, 3.0)]
    if not coupling:
        rx[1] = R([A, C], [X, E], 1e11, 0.0, 40.0)
        # X and Y collide with efficiency 0, so that [M] is the same whether
        # or not they are integrated as ordinary species
        rx[7].eff = {B: 2.5, D: 0.0, X: 0.0, Y: 0.0}
        rx[9].eff = {A: 2.0, X: 0.0, Y: 0.0}
        del rx[5]
    m = tiny(sp, rx)
    m.qss = [7, X, Y] if third else [X, Y]
    return m
