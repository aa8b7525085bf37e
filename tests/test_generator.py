"""Seeded input generator G(S,R,E,seed) and state builders."""
import hashlib

import numpy as np
import pytest

from paper_2405_05974_amd import synth


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_reactions_atom_balanced_and_mass_balanced(cfg):
    m = synth.config_mechanism(cfg)
    S, E = m.atoms.shape
    W = m.atoms @ np.array([mass for _, mass in m.elements])
    for r in m.reactions:
        lhs = m.atoms[r.reactants].sum(axis=0)
        rhs = m.atoms[r.products].sum(axis=0)
        assert np.array_equal(lhs, rhs)                 # exact in integers
        assert abs(W[r.reactants].sum() - W[r.products].sum()) <= 1e-12 * W.max()
        assert sorted(r.reactants) != sorted(r.products)
        assert 1 <= len(r.reactants) <= 2 and 1 <= len(r.products) <= 2


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_shape_counts_and_ranges(cfg):
    S, R, E, seed = synth.CONFIG_MECH[cfg]
    m = synth.config_mechanism(cfg)
    assert m.n_species == S and m.n_reactions == R and len(m.elements) == E
    assert sum(r.kind == 1 for r in m.reactions) == round(0.2 * R)
    assert all(r.kind in (0, 1) and r.reversible for r in m.reactions)
    inert = S - 1
    assert m.inert[inert] and m.inert.sum() == 1
    assert all(inert not in r.reactants and inert not in r.products for r in m.reactions)
    assert (m.atoms.sum(axis=1) > 0).all() and m.atoms.max() <= 3 and m.atoms.min() >= 0
    assert ((2.5 <= m.a0) & (m.a0 <= 6)).all() and ((0 <= m.a1) & (m.a1 <= 1e-3)).all()
    assert ((-3e5 <= m.hf) & (m.hf <= 3e5)).all() and ((150 <= m.s0) & (m.s0 <= 250)).all()
    A = np.array([r.A for r in m.reactions])
    assert ((1e8 <= A) & (A <= 1e14)).all()
    assert all(-1 <= r.b <= 2 and 0 <= r.Ea <= 40 for r in m.reactions)
    keys = {(tuple(sorted(r.reactants)), tuple(sorted(r.products))) for r in m.reactions}
    keys |= {(b, a) for a, b in keys}
    assert len(keys) == 2 * R                            # distinct reactions


def test_deterministic_per_seed():
    a = synth.make_mechanism(10, 25, 3, 0).to_text()
    b = synth.make_mechanism(10, 25, 3, 0).to_text()
    c = synth.make_mechanism(10, 25, 3, 1).to_text()
    assert a == b and a != c
    assert hashlib.sha256(a.encode()).hexdigest() == hashlib.sha256(b.encode()).hexdigest()


def test_text_roundtrip_floats():
    m = synth.config_mechanism(1)
    txt = m.to_text()
    vals = []
    for t in txt.split():
        try:
            if any(ch in t for ch in ".e"):
                vals.append(float(t))
        except ValueError:
            pass
    assert len(vals) > 100
    # 17 significant digits: the repr of every float survives a text round trip
    assert all(float(repr(v)) == v for v in vals)
    assert txt.startswith("chem-mech 1") and txt.rstrip().endswith("END")


def test_compositions():
    w = synth.uniform_batch(synth.config_mechanism(1), 4096, 1001, 1000, 1600, 1e-5, 1e-8, 1e-12)
    assert w.Y.shape == (10, 4096) and w.Y.flags.c_contiguous
    assert np.allclose(w.Y.sum(axis=0), 1.0, atol=1e-15)
    assert np.allclose(w.Y[-1], 0.7, atol=1e-15)
    assert (w.T >= 1000).all() and (w.T <= 1600).all()


def test_flame_profile_structure():
    m = synth.config_mechanism(2)
    Yeq = np.full(m.n_species, 1.0 / m.n_species)
    w = synth.flame_profile(m, (256, 2, 2), 1002, Yeq, 2e-6, 1e-8, 1e-12)
    assert w.n_cells == 1024
    T = w.T.reshape(256, 4)
    assert abs(T[0].mean() - 300) < 20 and abs(T[-1].mean() - 2200) < 20
    assert np.allclose(w.Y.sum(axis=0), 1.0, atol=1e-14)


def test_boxes_and_trace():
    m = synth.config_mechanism(4)
    boxes = synth.amr_boxes(m, 50, 1004, max_cells=64)
    assert all(8 <= b.L <= 64 and 1e-7 <= b.dt <= 1e-5 for b in boxes)
    tr = synth.poisson_trace(1005, 2000.0, 0.5)
    assert 800 < len(tr) < 1200 and np.all(np.diff(tr) > 0)
