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
