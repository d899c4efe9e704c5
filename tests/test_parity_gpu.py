"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

The precision contract makes the device and the oracle perform the same
IEEE operations in the same order, so every discrete outcome (cell index,
collision channel, child and secondary creation, array order after sorts) and
every stored value (particle state, fixed-point deposits, FP64 field and ion
fluid, counters, averages, EEDF) must be bitwise identical.
"""
import numpy as np
import pytest

import oracle
from paper_1508_02892_amd import hd, workloads as W

pytestmark = pytest.mark.gpu


def _fields_equal(g, o, live_only=True):
    assert len(g["cell"]) == len(o["cell"]), (len(g["cell"]), len(o["cell"]))
    np.testing.assert_array_equal(g["cell"], o["cell"])
    live = o["cell"] >= 0
    for k in ("off", "vx", "vy", "vz", "id"):
        a, b = g[k], o[k]
        if live_only:
            a, b = a[live], b[live]
        np.testing.assert_array_equal(a, b, err_msg=k)


def compare(dev_m, dev_p, orc: oracle.Oracle, dev_ep=None):
    o = orc.particles()
    _fields_equal(dev_p, o)
    g = orc.grid()
    np.testing.assert_array_equal(dev_m["cnt"], g["cnt"], err_msg="cnt")
    for k in ("n_i", "phi", "E"):
        np.testing.assert_array_equal(dev_m[k], g[k], err_msg=k)
    np.testing.assert_array_equal(dev_m["gamma_i"], g["gamma"], err_msg="gamma")
    S = len(orc.params.get("species", []))
    for q in range(S):
        sp = orc.species(q)
        np.testing.assert_array_equal(dev_m["n_species"][q * orc.nn:(q + 1) * orc.nn], sp["n"],
                                      err_msg="n of species %d" % q)
        np.testing.assert_array_equal(dev_m["gamma_species"][q * orc.nn:(q + 1) * orc.nn],
                                      sp["gamma"], err_msg="gamma of species %d" % q)
    if dev_ep is not None:
        np.testing.assert_array_equal(dev_ep, g["Ep"], err_msg="Ep")
    c = orc.counters()
    np.testing.assert_array_equal(dev_m["coll"], c["coll"])
    np.testing.assert_array_equal(dev_m["absorbed"], c["absorbed"])
    np.testing.assert_array_equal(dev_m["emitted"], c["emitted"])
    assert dev_m["created"] == c["created"]
    assert dev_m["overflow"] == c["overflow"]
    assert dev_m["n_acc"] == c["n_acc"]
    assert dev_m["pushed"] == c["pushed"]
    assert dev_m["step"] == orc.step_index
    pw = orc.power()
    assert dev_m["volt_amp"] == pw["volt_amp"]
    assert dev_m["p_abs"] == pw["p_abs"]
    assert dev_m["rf_periods"] == pw["rf_periods"]
    a = orc.accum()
    np.testing.assert_array_equal(dev_m["eedf_counts"], a["eedf"])
    if c["n_acc"]:
        d = orc.derived()
        dV = np.full(orc.nn, d["dz"])
        dV[0] = dV[-1] = d["dz"] / 2
        scale = (d["w"] * 2.0 ** -32) / dV
        np.testing.assert_array_equal(dev_m["n_e_avg"],
                                      a["acc_cnt"].astype(np.float64) * scale / c["n_acc"])
        np.testing.assert_array_equal(dev_m["n_i_avg"], a["acc_ni"] / c["n_acc"])


def run_pair(p, steps, chunks=None):
    dev = hd.Discharge(p)
    orc = oracle.Oracle(p, contract=True)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())
    for n in (chunks or [steps]):
        dev.step(n)
        orc.step(n)
        compare(dev.moments(), dev.particles(), orc, dev.push_field())
    return dev, orc


@pytest.mark.parametrize("precision", [0, 1])
def test_device_arithmetic_is_correctly_rounded(precision):
    rng = np.random.default_rng(precision)
    dt = oracle.pdtype(precision)
    a = np.concatenate([rng.random(20000), rng.random(20000) * 1e6, rng.random(2000) * 1e-30,
                        [0.0, 1.0, 0.5, 2.0 ** -24, 1 - 2.0 ** -24, 3.0]]).astype(dt)
    b = (rng.random(len(a)) + 0.01).astype(dt)
    out = hd.diag_arith(precision, a, b)
    np.testing.assert_array_equal(out[:, 0], np.sqrt(a))
    np.testing.assert_array_equal(out[:, 1], a / b)
    np.testing.assert_array_equal(out[:, 2], np.rint(a * dt(2.0 ** 32)))
    np.testing.assert_array_equal(out[:, 3], np.floor(a))


@pytest.mark.parametrize("precision,model", [(1, 0), (0, 0), (0, 1), (1, 1)])
def test_initial_state_matches(precision, model):
    p = W.small(precision=precision, ion_model=model, n_cells=64, n_macro=5000)
    dev = hd.Discharge(p)
    orc = oracle.Oracle(p, contract=True)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())


@pytest.mark.parametrize("precision,model", [(1, 0), (0, 0), (0, 1), (1, 1), (0, 2), (1, 3)])
def test_steps_match_small(precision, model):
    # 5,000 electrons = 4 full chunks and a ragged one; 40 steps cross two sorts
    # and two EEDF samples, single steps and captured intervals.
    p = W.small(precision=precision, ion_model=model, n_cells=64, n_macro=5000)
    run_pair(p, 40, chunks=[1, 2, 13, 16, 8])


def _hot(precision, model, **kw):
    return W.small(precision=precision, ion_model=model, n_cells=64, n_macro=20_000,
                   t_e0_eV=50.0, v_amp_V=2000.0, phase_rad=np.pi / 2, gamma_see=1.0,
                   load_lo=0.0, load_hi=1.0, mu_const=8e-3, **kw)


@pytest.mark.parametrize("precision,model", [(0, 1), (1, 0)])
def test_ionization_emission_and_walls_match(precision, model):
    dev, orc = run_pair(_hot(precision, model), 48, chunks=[3, 16, 29])
    c = orc.counters()
    assert c["created"] > 0 and c["emitted"].sum() > 0 and c["absorbed"].sum() > 0


def _fit_case(precision, model):
    base = dict(precision=precision, ion_model=model, n_cells=64, n_macro=20_000, t_e0_eV=50.0,
                phase_rad=np.pi / 2, gamma_see=1.0, load_lo=0.0, load_hi=1.0)
    if model == W.ION_DD_FIT:
        # the vacuum field sits just above the Table 2 branch field; the
        # space charge of the escaping electrons pulls part of the gap below
        return W.small(v_amp_V=184.0, n_e0_m3=1e19, **base), [1, 15, 32]
    # the ions accelerate through the Table 3 branch speed near step 160
    return W.small(v_amp_V=4000.0, mu_const=8e-3, **base), [1, 31, 64, 128]


@pytest.mark.parametrize("precision,model", [(0, W.ION_DD_FIT), (1, W.ION_FULL_FIT),
                                             (0, W.ION_FULL_FIT), (1, W.ION_DD_FIT)])
def test_fitted_transport_matches(precision, model):
    p, chunks = _fit_case(precision, model)
    dev, orc = run_pair(p, sum(chunks), chunks=chunks)
    g = orc.grid()
    if model == W.ION_DD_FIT:
        a, x0 = np.abs(g["E"]), 1.47e6
    else:
        n = g["n_i"]
        a = np.abs(np.where(n > orc.derived()["nfloor"], g["gamma"] / np.maximum(n, 1e-300), 0.0))
        x0 = 2e3
    # both branches of the fit were taken on the last step
    assert (a < x0).sum() >= 5 and (a >= x0).sum() >= 5


@pytest.mark.parametrize("precision,model", [(0, W.ION_FULL), (1, W.ION_DD), (0, W.ION_DD_FIT)])
def test_power_control_matches(precision, model):
    # RF periods of 20 steps, so that five amplitude updates (Eq 2.9) feed
    # back into the field within 100 steps; ionization, emission and wall
    # losses all carry current.  Zero phase puts the period ends at V = 0.
    p = _hot(precision, model, f_rf_Hz=1.0 / (20 * 2e-14), power_W_m2=1e6, power_alpha=0.1)
    p["phase_rad"] = 0.0
    dev, orc = run_pair(p, 100, chunks=[7, 13, 20, 40, 20])
    pw = orc.power()
    assert pw["rf_periods"] == 5 and pw["volt_amp"] != p["v_amp_V"] and pw["p_abs"] != 0.0


def _chem_case(precision, **kw):
    # the complex chemistry with attachment 1,000 times stronger, so that
    # electrons attach within a few dozen steps; hot enough to ionize He and
    # the admixture
    ch = W.chem_channels()
    ch[8] = dict(ch[8], sigma_m2=ch[8]["sigma_m2"] * 1e3)
    base = dict(precision=precision, n_cells=64, n_macro=20_000, t_e0_eV=8.0, v_amp_V=2000.0,
                phase_rad=np.pi / 2, gamma_see=1.0, load_lo=0.0, load_hi=1.0, channels=ch)
    base.update(kw)
    return W.small_chem(**base)


@pytest.mark.parametrize("precision", [0, 1])
def test_complex_chemistry_matches(precision):
    # twelve channels (the generic channel path), attachment into O-,
    # ionization into He+, He2+ and O2+, four drift-diffusion species
    p = _chem_case(precision)
    dev, orc = run_pair(p, 48, chunks=[1, 15, 32])
    c = orc.counters()
    assert c["coll"][8] > 0 and c["coll"][9] > 0 and c["coll"][10] > 0
    assert orc.species(3)["n"].any() and orc.species(2)["n"].any()


def test_c2_full_size_first_steps_match():
    # the complex-chemistry workload at full size: 4,194,304 FP32 electrons,
    # 1,024 cells, 17 steps including one compaction + sort
    p = W.c2()
    dev = hd.Discharge(p)
    orc = oracle.Oracle(p, contract=True)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())
    dev.step(17)
    orc.step(17)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())


def test_mixed_ion_models_in_one_batch():
    # one launch advances constant and fitted, drift-diffusion and full fluids
    ps = [_fit_case(0, m)[0] for m in (W.ION_DD_FIT, W.ION_FULL_FIT)]
    ps = [_hot(0, W.ION_DD, seed=40), _hot(0, W.ION_FULL, seed=41)] + ps + [_chem_case(0, seed=44)]
    b = hd.Batch(ps)
    b.step(7)
    b.step(16)
    for i, p in enumerate(ps):
        orc = oracle.Oracle(p, contract=True)
        orc.step(23)
        compare(b.moments(i), b.particles(i), orc)


def test_many_chunks_per_workgroup_and_sparse_eedf():
    # enough particles that each persistent workgroup takes several chunks
    p = W.small(precision=0, ion_model=1, n_cells=512, n_macro=1_500_000, gap_m=2e-3,
                eedf_every=5)
    run_pair(p, 21, chunks=[5, 16])


def test_c0_full_run_matches():
    p = W.c0()
    dev = hd.Discharge(p)
    orc = oracle.Oracle(p, contract=True)
    dev.step(W.C0_STEPS)
    orc.step(W.C0_STEPS)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())


def test_c1_full_size_first_steps_match():
    # the single large discharge at full size: 8,388,608 FP32 electrons, full
    # ion fluid, 2,048 cells; 17 steps include one compaction + sort
    p = W.c1()
    dev = hd.Discharge(p)
    orc = oracle.Oracle(p, contract=True)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())
    dev.step(17)
    orc.step(17)
    compare(dev.moments(), dev.particles(), orc, dev.push_field())


def test_batch_members_match_alone_and_oracle():
    ps = [W.small(precision=0, ion_model=0, n_cells=n, n_macro=m, seed=s, v_amp_V=v)
          for n, m, s, v in [(64, 3000, 11, 150.0), (128, 9000, 12, 300.0), (96, 1, 13, 50.0),
                             (256, 40000, 14, 250.0)]]
    b = hd.Batch(ps)
    b.step(5)
    b.step(30)
    for i, p in enumerate(ps):
        orc = oracle.Oracle(p, contract=True)
        orc.step(35)
        compare(b.moments(i), b.particles(i), orc)


def test_capacity_overflow_is_reported():
    p = _hot(0, 0)
    p["capacity"] = p["n_macro"] + 10
    dev = hd.Discharge(p)
    dev.step(20)
    with pytest.raises(hd.HdError) as e:
        dev.moments()
    assert e.value.code == -4
    with pytest.raises(hd.HdError):
        dev.step(1)
