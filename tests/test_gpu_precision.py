"""The two precision forms against the FP64 oracle, observable by observable
(needs an MI355X).

Step 1 (the trajectories still agree): the relative error of every
observable of each form against the oracle.  Time averages over steps
200..1000 (the trajectories have decorrelated, so the comparison is
statistical): kinetic temperature, pressure, mean many-body density and
potential energy per particle of each form against the oracle's own time
averages.  The table is printed (pytest -s shows it) and the bars asserted:
FP64 form within 1e-12 at step 1, FP32 form within 1e-5; both forms' time
averages within 1% of the oracle's; pressure, a small difference of large
terms with large fluctuations in a 6,000-particle box, within four standard
errors of the difference of the two sample means.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import orc_params, say

pytestmark = pytest.mark.gpu

KEYS = ("ke", "kT", "pressure", "virial", "epot", "mean_rho")


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_observable_errors_per_form(mdpd):
    w = W.bulk(L=10.0, seed=0)
    say("precision forms vs oracle", w.n)
    forms = {"fp64": mdpd.FP64, "fp32_forces": mdpd.FP32_FORCES}
    o = oracle.System(orc_params(w, search=1), w.x, w.v)
    systems = {k: mdpd.System(w, precision=p) for k, p in forms.items()}
    o.step(1)
    ref = o.observables()
    rows = []
    for k, s in systems.items():
        s.step(1)
        ob = s.observables()
        errs = {q: rel(ob[q], ref[q]) for q in KEYS}
        rows.append((k, errs))
        bar = 1e-12 if k == "fp64" else 1e-5
        for q, e in errs.items():
            assert e < bar, (k, q, e)
    print("\nstep 1, relative error vs the FP64 oracle")
    for k, errs in rows:
        print(f"  {k:12s} " + "  ".join(f"{q} {e:.1e}" for q, e in errs.items()))
    # time averages, and the drift of the total momentum (zero at the start:
    # the Maxwell velocities have their mean removed; with no walls and no
    # body force every pair force cancels in exact arithmetic)
    acc = {k: [] for k in ["oracle", *systems]}
    pmax = {k: 0.0 for k in ["oracle", *systems]}
    for block in range(100):
        o.step(10)
        for s in systems.values():
            s.step(10)
        ob = o.observables()
        pmax["oracle"] = max(pmax["oracle"], float(np.abs([ob["px"], ob["py"], ob["pz"]]).max()))
        for k, s in systems.items():
            pmax[k] = max(pmax[k], float(np.abs(s.observables()["momentum"]).max()))
        if block >= 20:
            acc["oracle"].append([o.observables()[q] for q in KEYS])
            for k, s in systems.items():
                acc[k].append([s.observables()[q] for q in KEYS])
    arr = {k: np.array(v) for k, v in acc.items()}
    mean = {k: dict(zip(KEYS, np.mean(v, axis=0))) for k, v in arr.items()}
    var = {k: dict(zip(KEYS, np.var(v, axis=0, ddof=1) / v.shape[0])) for k, v in arr.items()}
    print("time averages over steps 210..1000 (standard error of the mean in brackets)")
    for k, m in mean.items():
        print(f"  {k:12s} " + "  ".join(f"{q} {v:.5g} ({np.sqrt(var[k][q]):.2g})" for q, v in m.items()))
    print("largest |total momentum component| over 1000 steps (thermal scale sqrt(N m kT) = "
          f"{np.sqrt(w.n * w.mass * w.kT):.1f}): " + "  ".join(f"{k} {v:.2e}" for k, v in pmax.items()))
    assert pmax["oracle"] < 1e-9 and pmax["fp64"] < 1e-9, pmax
    assert pmax["fp32_forces"] < 0.05, pmax
    for k in systems:
        assert rel(mean[k]["kT"], mean["oracle"]["kT"]) < 0.01, k
        assert rel(mean[k]["mean_rho"], mean["oracle"]["mean_rho"]) < 0.01, k
        assert rel(mean[k]["epot"], mean["oracle"]["epot"]) < 0.01, k
        se = np.sqrt(var[k]["pressure"] + var["oracle"]["pressure"])
        assert abs(mean[k]["pressure"] - mean["oracle"]["pressure"]) < 4.0 * se, (k, se)
    for s in systems.values():
        s.close()
