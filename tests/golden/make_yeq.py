"""Write the equilibrium compositions used by the flame-profile workloads.

The hot side of the planar flame holds the composition that the oracle's
kinetics reach from the cold mixture at a fixed 2200 K and 1 atm (a long
fixed-temperature integration, horizon 1 s, rtol 1e-10, atol 1e-20).  The
values depend only on the oracle and the seeded generator; this script calls
nothing else.  Run:  python tests/golden/make_yeq.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2405_05974_amd import synth  # noqa: E402


def yeq_path(cfg: int) -> str:
    S, R, E, seed = synth.CONFIG_MECH[cfg]
    return os.path.join(HERE, f"yeq_G{S}_{R}_{E}_s{seed}.txt")


def main(cfgs=(2, 3)):
    for cfg in cfgs:
        m = synth.config_mechanism(cfg)
        om = oracle.Mech(m.to_text())
        rng = np.random.default_rng(synth.config_seed(cfg))
        Yc = synth.cold_mixture(rng, m.n_species)
        T, Y, st = om.integrate(np.array([2200.0]), Yc[:, None], synth.P_ATM, 1.0, 1e-10, 1e-20,
                                fixed_T=True, max_steps=10 ** 7)
        assert st[0]["status"] == 0, st
        with open(yeq_path(cfg), "w") as fh:
            fh.write(f"# equilibrium composition of {m.label} at 2200 K, 1 atm (oracle, fixed T, 1 s)\n")
            fh.write(f"# cold mixture: 0.7 inert + 0.3 Dirichlet(2), rng seed {synth.config_seed(cfg)}\n")
            fh.write(f"# steps {int(st[0]['steps'])}\n")
            for v in Y[:, 0]:
                fh.write(repr(float(v)) + "\n")
        print(cfg, yeq_path(cfg), int(st[0]["steps"]))


if __name__ == "__main__":
    main(tuple(int(a) for a in sys.argv[1:]) or (2, 3))
