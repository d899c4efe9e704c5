"""Precision contract of the FP32 path against the FP64 oracle.

* Per-step error: from the same seeded load (the FP32 state is the FP64
  state rounded), one step of the GPU in FP32 and of the oracle in FP64 must
  give deposits, ion density, potential and field within 1e-5 of the profile's
  scale.  (Collisions change velocities only, so one step's deposits are
  still comparable; later steps diverge particle by particle.)
* Statistical agreement: time-averaged electron/ion density profiles and the
  EEDF of independent FP32 GPU and FP64 oracle ensembles agree within their
  ensemble errors.
"""
import numpy as np
import pytest

import oracle
from paper_1508_02892_amd import hd, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("model", [0, 1])
def test_fp32_step_within_1e5_of_fp64_oracle(model):
    base = dict(ion_model=model, n_cells=128, n_macro=60_000, t_e0_eV=6.0, v_amp_V=300.0,
                phase_rad=0.7)
    dev = hd.Discharge(W.small(precision=0, **base))
    orc = oracle.Oracle(W.small(precision=1, **base))
    for step in (0, 1):
        if step:
            dev.step(1)
            orc.step(1)
        m = dev.moments()
        g = orc.grid()
        errs = {"cnt": _rel(m["cnt"], g["cnt"]), "n_i": _rel(m["n_i"], g["n_i"]),
                "phi": _rel(m["phi"], g["phi"]), "E": _rel(m["E"], g["E"])}
        print("FP32 vs FP64, step", step, errs)
        for k, v in errs.items():
            assert v <= TOL, (step, k, v)


def _ensemble_gpu(p, seeds, steps):
    ne, ni, ee = [], [], []
    for s in seeds:
        d = hd.Discharge(dict(p, seed=s, precision=0))
        d.step(steps)
        m = d.moments()
        ne.append(m["n_e_avg"])
        ni.append(m["n_i_avg"])
        ee.append(m["eedf_counts"].astype(np.float64))
        d.close()
    return np.array(ne), np.array(ni), np.array(ee)


def _ensemble_oracle(p, seeds, steps):
    ne, ni, ee = [], [], []
    for s in seeds:
        o = oracle.Oracle(dict(p, seed=s, precision=1))
        o.step(steps)
        a = o.accum()
        d = o.derived()
        nn = p["n_cells"] + 1
        dV = np.full(nn, d["dz"])
        dV[0] = dV[-1] = d["dz"] / 2
        n_acc = o.counters()["n_acc"]
        ne.append(a["acc_cnt"].astype(np.float64) * (d["w"] * 2.0 ** -32) / dV / n_acc)
        ni.append(a["acc_ni"] / n_acc)
        ee.append(a["eedf"].astype(np.float64))
    return np.array(ne), np.array(ni), np.array(ee)


def test_time_averages_agree_statistically():
    p = W.small(n_cells=64, n_macro=20_000, t_e0_eV=4.0, v_amp_V=120.0, eedf_every=8,
                load_lo=0.1, load_hi=0.9)
    K, steps = 8, 400
    g_ne, g_ni, g_ee = _ensemble_gpu(p, range(100, 100 + K), steps)
    o_ne, o_ni, o_ee = _ensemble_oracle(p, range(200, 200 + K), steps)
    for name, a, b in (("n_e", g_ne, o_ne), ("n_i", g_ni, o_ni)):
        diff = a.mean(0) - b.mean(0)
        se = np.sqrt(a.var(0, ddof=1) / K + b.var(0, ddof=1) / K) + 1e-9 * np.abs(b).max()
        z = np.abs(diff) / se
        print(name, "max z", z.max())
        assert z.max() < 5.0, name
    # EEDF: samples within a run are correlated (the same particles every
    # eedf_every steps), so bins are compared by their seed-to-seed spread
    gf = g_ee / g_ee.sum(1, keepdims=True)
    of = o_ee / o_ee.sum(1, keepdims=True)
    se = np.sqrt(gf.var(0, ddof=1) / K + of.var(0, ddof=1) / K)
    m = (gf.mean(0) + of.mean(0)) > 1e-3
    z = np.abs(gf.mean(0) - of.mean(0))[m] / se[m]
    print("eedf bins", m.sum(), "max z", z.max())
    assert z.max() < 5.0
    centre = (np.arange(gf.shape[1] - 1) + 0.5) * p["eedf_emax_eV"] / p["n_eedf_bins"]
    ge = (gf[:, :-1] * centre).sum(1) / gf[:, :-1].sum(1)
    oe = (of[:, :-1] * centre).sum(1) / of[:, :-1].sum(1)
    print("mean energy", ge.mean(), oe.mean())
    assert abs(ge.mean() / oe.mean() - 1) < 0.01
