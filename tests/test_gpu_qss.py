"""GPU parity for mechanisms with quasi-steady-state (QSS) species: the
closure (Eq. 4-6) solved group by group in the generated kernels, the
one-sided linearisation and the Jacobian through the closure, against the
oracle (one dense pivoted solve, Schur-complement Jacobian).

Stage parity (rates of the transported species, right-hand side, Jacobian)
on the hand-built mechanisms, whose rates are well conditioned; integration
at the FP64 bars |dY| <= 1e-8 and |dT|/T <= 1e-8 on them and on synthetic QSS
mechanisms, with QSS groups of 1 to 4 species and two groups solved in
dependency order.  (On synthetic mechanisms whose net rates are tiny
differences of huge gross ones, the rounding of the two closure solves,
group by group and dense, shows in the net rates: one such case agrees only
to ~2e-7 and is not used here.)
"""
import numpy as np
import pytest

from paper_2405_05974_amd import synth
from tests import mechs
from tests.test_gpu_parity import assert_parity, chem, gpu_integrate, oracle_integrate, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

P60 = 60e5

# name -> (mechanism factory, dt, T range); G_qss seeds where the QSS
# approximation holds over the sampled states (the oracle fails no cell)
WORK = {
    "qtiny": (mechs.qss_tiny, 3e-6, 1000.0, 1800.0),                                   # one group of 2
    "qtiny3": (lambda: mechs.qss_tiny(third=True), 3e-6, 1000.0, 1800.0),              # groups {X, Y}, then {Z}
    "gq13": (lambda: synth.make_qss_mechanism(13, 36, 3, 34, 3), 1e-6, 1000.0, 1600.0),   # one group of 3
    "gq14": (lambda: synth.make_qss_mechanism(14, 40, 3, 30, 4), 1e-6, 1000.0, 1600.0),   # one group of 4
}


def workload(name, n):
    make, dt, lo, hi = WORK[name]
    m = make()
    rng = np.random.default_rng(41)
    T = rng.uniform(lo, hi, n)
    Y = synth.composition(rng, m.n_state_species, 1.0, n)
    return m, T, Y, dt


@pytest.mark.parametrize("third,p", [(False, synth.P_ATM), (False, P60), (True, synth.P_ATM)],
                         ids=["1atm", "60bar", "three-qss"])
def test_qss_rates_rhs_jacobian_parity(chem, torch_dev, third, p):
    import oracle
    torch, dev = torch_dev
    m = mechs.qss_tiny(third=third)
    n = 131
    rng = np.random.default_rng(7)
    T = rng.uniform(700.0, 2400.0, n)
    Y = np.vstack([0.3 * rng.dirichlet(np.ones(5), size=n).T, np.full((1, n), 0.7)])
    text = m.to_text()
    om = oracle.Mech(text)
    gm = chem.Mechanism(text)
    assert gm.S == m.n_state_species
    ST, N = m.n_state_species, m.n_state_species + 1
    say(f"qss rates qtiny third={third} n={n} p={p:g}")
    Tt = torch.tensor(T, device=dev)
    Yt = torch.tensor(np.ascontiguousarray(Y), device=dev)
    wd = torch.zeros((ST, n), dtype=torch.float64, device=dev)
    f = torch.zeros((N, n), dtype=torch.float64, device=dev)
    J = torch.zeros((N * N, n), dtype=torch.float64, device=dev)
    gm.rates(Tt, Yt, p, wd, f, J)
    torch.cuda.synchronize()
    wd, f, J = wd.cpu().numpy(), f.cpu().numpy(), J.cpu().numpy()
    worst = {"wdot": 0.0, "f": 0.0, "J": 0.0}
    for i in range(n):
        _, wo, bad = om.qss_rates(T[i], Y[:, i], p)
        assert not bad
        worst["wdot"] = max(worst["wdot"], np.abs(wd[:, i] * 1e-6 - wo).max() / np.abs(wo).max())
        y = np.concatenate([Y[:, i], [T[i]]])
        fo = om.rhs(y, p)
        worst["f"] = max(worst["f"], np.abs(f[:, i] - fo).max() / np.abs(fo).max())
        Jo = om.jac(y, p)
        rs = np.abs(Jo).max(axis=1, keepdims=True) + 1e-300
        worst["J"] = max(worst["J"], (np.abs(J[:, i].reshape(N, N) - Jo) / rs).max())
    say(f"qss rates p={p:g} worst relative: {worst}")
    assert worst["wdot"] <= 1e-11 and worst["f"] <= 1e-11 and worst["J"] <= 1e-9


@pytest.mark.parametrize("name,p", [("qtiny", synth.P_ATM), ("qtiny", P60), ("qtiny3", synth.P_ATM), ("qtiny3", P60),
                                    ("gq13", synth.P_ATM), ("gq14", synth.P_ATM)])
def test_qss_integration_parity(chem, torch_dev, name, p):
    n = 160
    m, T, Y, dt = workload(name, n)
    text = m.to_text()
    say(f"qss integration {name} p={p:g} n={n} dt={dt:g}")
    Tg, Yg, st, rec = gpu_integrate(chem, torch_dev, text, T, Y, p, dt, 1e-8, 1e-12)
    To, Yo, so = oracle_integrate(text, T, Y, p, dt, 1e-8, 1e-12)
    assert (so["status"] == 0).all() and st["rc"] == 0
    assert np.abs(Tg - T).max() > 1.0
    assert_parity(Tg, Yg, To, Yo, f"qss {name} p={p:g}")
    say(f"qss {name}: identical step counts in {np.mean(rec[1] == so['steps']):.3f} of the cells")


def test_qss_boxes_equal_integrate(chem, torch_dev):
    torch, dev = torch_dev
    m, T, Y, dt = workload("gq13", 200)
    text = m.to_text()
    gm = chem.Mechanism(text)
    say("qss boxes gq13: 3 boxes vs one integrate")
    Ta = torch.tensor(T, device=dev)
    Ya = torch.tensor(np.ascontiguousarray(Y), device=dev)
    gm.integrate(Ta, Ya, synth.P_ATM, dt, 1e-8, 1e-12)
    cuts = [0, 70, 71, 200]
    boxes = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        boxes.append((torch.tensor(T[a:b], device=dev), torch.tensor(np.ascontiguousarray(Y[:, a:b]), device=dev), dt))
    gm.integrate_boxes(boxes, synth.P_ATM, 1e-8, 1e-12)
    torch.cuda.synchronize()
    Tb = np.concatenate([b[0].cpu().numpy() for b in boxes])
    Yb = np.concatenate([b[1].cpu().numpy() for b in boxes], axis=1)
    assert np.array_equal(Tb, Ta.cpu().numpy()) and np.array_equal(Yb, Ya.cpu().numpy())


def test_qss_refused_where_unsupported(chem, torch_dev):
    torch, dev = torch_dev
    m = mechs.qss_tiny()
    gm = chem.Mechanism(m.to_text())
    T = torch.full((4,), 1200.0, dtype=torch.float64, device=dev)
    Y = torch.full((m.n_state_species, 4), 1.0 / m.n_state_species, dtype=torch.float64, device=dev)
    say("qss: group kernels and FP32 LU refuse QSS mechanisms")
    gm.set_options(kernel=1)
    with pytest.raises(chem.ChemError, match="QSS"):
        gm.integrate(T, Y, synth.P_ATM, 1e-7, 1e-8, 1e-12)
    gm.set_options(kernel=0, lu_fp32=1)
    with pytest.raises(chem.ChemError, match="QSS"):
        gm.integrate(T, Y, synth.P_ATM, 1e-7, 1e-8, 1e-12)
