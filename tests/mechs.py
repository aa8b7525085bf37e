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
