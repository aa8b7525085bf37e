"""GPU parity for real-mechanism features: NASA 7-coefficient thermo, Troe
falloff and collision efficiencies (G_real mechanisms), in both kernel
families, against the oracle on the same seeded inputs.

Stage parity (rates, right-hand side, analytic Jacobian) at rounding-level
tolerances on states spanning both thermo ranges and the falloff region; the
integration at the FP64 bars |dY| <= 1e-8 and |dT|/T <= 1e-8.
"""
import numpy as np
import pytest

from paper_2405_05974_amd import synth
from tests.test_gpu_parity import assert_parity, chem, check_rates, gpu_integrate, oracle_integrate, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

P60 = 60e5

REAL = {
    "real10": (10, 25, 3, 6),     # N = 11: the generated lane-per-cell kernels serve it
    "real12": (12, 40, 4, 5),     # N = 13: group kernels, 16 lanes per cell
    "real30": (30, 120, 4, 8),    # N = 31: group kernels, 32 lanes per cell
}


def real(name):
    return synth.make_real_mechanism(*REAL[name])


@pytest.mark.parametrize("name,kernel,p", [("real10", 2, synth.P_ATM), ("real10", 1, synth.P_ATM),
                                           ("real10", 2, P60), ("real12", 1, synth.P_ATM), ("real12", 1, P60),
                                           ("real30", 1, synth.P_ATM)],
                         ids=["real10-lane", "real10-group", "real10-lane-60bar", "real12-group",
                              "real12-group-60bar", "real30-group"])
def test_real_rates_rhs_jacobian_parity(chem, torch_dev, name, kernel, p):
    m = real(name)
    n = 131
    rng = np.random.default_rng(17)
    T = rng.uniform(300.0, 3000.0, n)
    T[:4] = [999.0, 1000.0, 1000.0 + 1e-9, 1001.0]      # both sides of the thermo range split
    Y = synth.composition(rng, m.n_species, 0.5, n)
    check_rates(chem, torch_dev, m, T, Y, p, kernel, name)


@pytest.mark.parametrize("name,kernel,p", [("real10", 2, synth.P_ATM), ("real10", 1, synth.P_ATM),
                                           ("real10", 2, P60), ("real12", 1, synth.P_ATM), ("real12", 1, P60),
                                           ("real30", 1, synth.P_ATM)],
                         ids=["real10-lane", "real10-group", "real10-lane-60bar", "real12-group",
                              "real12-group-60bar", "real30-group"])
def test_real_integration_parity(chem, torch_dev, name, kernel, p):
    m = real(name)
    n = 200 if name != "real30" else 96
    w = synth.uniform_batch(m, n, 23, 800.0, 1800.0, 1e-6, 1e-8, 1e-12)
    say(f"real integration {name} kernel={kernel} p={p:g} n={n}")
    Tg, Yg, st, rec = gpu_integrate(chem, torch_dev, m.to_text(), w.T, w.Y, p, w.dt, w.rtol, w.atol, kernel=kernel)
    To, Yo, so = oracle_integrate(m.to_text(), w.T, w.Y, p, w.dt, w.rtol, w.atol)
    assert st["rc"] == 0 and all(s["status"] == 0 for s in so)
    assert np.abs(Tg - w.T).max() > 1.0          # the cells react (heat release crosses the range split)
    assert_parity(Tg, Yg, To, Yo, f"real {name} kernel={kernel} p={p:g}")
    steps_o = np.array([s["steps"] for s in so])
    say(f"real {name}: identical step counts in {np.mean(rec[1] == steps_o):.3f} of the cells")


def test_real_lane_and_group_agree(chem, torch_dev):
    m = real("real10")
    w = synth.uniform_batch(m, 128, 29, 900.0, 1700.0, 1e-6, 1e-8, 1e-12)
    say("real10 lane vs group")
    Ta, Ya, _, _ = gpu_integrate(chem, torch_dev, m.to_text(), w.T, w.Y, w.p, w.dt, w.rtol, w.atol, kernel=2)
    Tb, Yb, _, _ = gpu_integrate(chem, torch_dev, m.to_text(), w.T, w.Y, w.p, w.dt, w.rtol, w.atol, kernel=1)
    assert_parity(Ta, Ya, Tb, Yb, "real10 lane vs group")
