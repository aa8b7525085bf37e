"""The allocation-free entry point (chem_integrate_noalloc) against
chem_integrate on the same inputs: two calls in a row, the second smaller,
for both kernel families.  The two run the same kernels, so results and
statistics must agree exactly; the oracle bar (|dY| <= 1e-8, |dT|/T <= 1e-8)
is checked on the first call as well.
"""
import numpy as np
import pytest

from paper_2405_05974_amd import synth

pytestmark = pytest.mark.gpu

STAT_KEYS = ("n_cells", "n_steps_total", "n_steps_max", "n_attempts", "n_rhs", "n_jac", "n_newton_iters",
             "n_err_test_fails", "n_newton_fails", "n_cells_failed")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _run_pair(chem, torch, dev, gm, w, n, noalloc):
    T = torch.tensor(w.T[:n].copy(), dtype=torch.float64, device=dev)
    Y = torch.tensor(np.ascontiguousarray(w.Y[:, :n]), dtype=torch.float64, device=dev)
    if noalloc:
        st = gm.integrate_noalloc(T, Y, w.p, w.dt, w.rtol, w.atol)
    else:
        st = gm.integrate(T, Y, w.p, w.dt, w.rtol, w.atol)
    torch.cuda.synchronize()
    return T.cpu().numpy(), Y.cpu().numpy(), st


@pytest.mark.parametrize("kernel", ["lane", "group"])
def test_noalloc_equals_integrate_twice_second_smaller(kernel):
    import torch
    import oracle
    from paper_2405_05974_amd import chem
    chem.load_library()
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    m = synth.config_mechanism(1)
    w = synth.uniform_batch(m, 1000, 11, 1000.0, 1600.0, 1e-6, 1e-8, 1e-12)
    gm = chem.Mechanism(m.to_text())
    gm.set_options(kernel=2 if kernel == "lane" else 1)
    # a first ordinary call loads the generated module (the allocation-free call refuses to)
    say(f"noalloc {kernel}: warm-up chem_integrate on 64 cells")
    _run_pair(chem, torch, dev, gm, w, 64, noalloc=False)
    om = oracle.Mech(m.to_text())
    for n in (1000, 333):
        say(f"noalloc {kernel}: n={n} chem_integrate")
        Ta, Ya, sa = _run_pair(chem, torch, dev, gm, w, n, noalloc=False)
        say(f"noalloc {kernel}: n={n} chem_integrate_noalloc")
        Tb, Yb, sb = _run_pair(chem, torch, dev, gm, w, n, noalloc=True)
        assert np.array_equal(Ta, Tb) and np.array_equal(Ya, Yb), (kernel, n)
        for k in STAT_KEYS:
            assert sa[k] == sb[k], (kernel, n, k, sa[k], sb[k])
        assert sb["rc"] == sa["rc"] == 0
        if n == 1000:
            To, Yo, _ = om.integrate(w.T[:n], w.Y[:, :n], w.p, w.dt, w.rtol, w.atol)
            dY = float(np.abs(Yb - Yo).max())
            dT = float((np.abs(Tb - To) / To).max())
            say(f"noalloc {kernel}: vs oracle max|dY|={dY:.3e} max|dT|/T={dT:.3e}")
            assert dY <= 1e-8 and dT <= 1e-8


def test_noalloc_rejects_what_it_cannot_do_without_allocating():
    import torch
    from paper_2405_05974_amd import chem
    chem.load_library()
    dev = torch.device("cuda:0")
    m = synth.config_mechanism(1)
    gm = chem.Mechanism(m.to_text())
    T = torch.full((4,), 1200.0, dtype=torch.float64, device=dev)
    Y = torch.full((m.n_species, 4), 1.0 / m.n_species, dtype=torch.float64, device=dev)
    say("noalloc: refusals (module not loaded, retry option, size limit)")
    gm.set_options(kernel=2)
    with pytest.raises(chem.ChemError, match="not loaded"):
        gm.integrate_noalloc(T, Y, 101325.0, 1e-7, 1e-8, 1e-12)
    gm.set_options(kernel=1, retry=1)
    with pytest.raises(chem.ChemError, match="retry"):
        gm.integrate_noalloc(T, Y, 101325.0, 1e-7, 1e-8, 1e-12)
    gm.set_options(retry=0)
    lib = chem.load_library()
    rc = lib.chem_integrate_noalloc(gm.h, chem.NOALLOC_MAX_CELLS + 1, chem._ptr(T), chem._ptr(Y), 101325.0, 1e-7,
                                    1e-8, 1e-12, None)
    assert rc == chem.CHEM_ERR_ARG and b"allocation-free limit" in lib.chem_last_error()
