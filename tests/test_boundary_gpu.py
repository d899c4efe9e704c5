"""The C ABI's device memory and failure handling, on the GPU.

* A caller-supplied arena (a torch byte tensor) holds the whole device state:
  the run equals the library-allocated run and the oracle bit for bit; too
  small an arena is HD_ENOMEM.
* Capacity overflow: the handle keeps a checkpoint of a sort interval that
  starts close to its capacity; an overflow is rolled back to the last
  complete step (HD_ECAPACITY), hd_grow raises the capacity, and the
  continued run equals an uninterrupted one and the oracle bit for bit.
* A field that stops being finite (an absurd drive amplitude, an ordinary
  parameter) is reported as HD_ENUMERIC and the handle stops stepping.
* The launch-graph path runs: steps replayed from captured graphs are
  counted.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1508_02892_amd import hd, workloads as W

pytestmark = pytest.mark.gpu


def _same_state(a, b):
    ma, pa = a
    mb, pb = b
    for k in pa:
        np.testing.assert_array_equal(pa[k], pb[k], err_msg=k)
    for k in ("cnt", "n_i", "phi", "E", "gamma_i", "n_e_avg", "n_i_avg", "eedf_counts", "coll",
              "absorbed", "emitted"):
        np.testing.assert_array_equal(ma[k], mb[k], err_msg=k)
    for k in ("step", "created", "pushed", "n_acc"):
        assert ma[k] == mb[k], k


def _hot(**kw):
    return W.small(precision=0, ion_model=W.ION_FULL, n_cells=64, n_macro=20_000, t_e0_eV=50.0,
                   v_amp_V=2000.0, phase_rad=np.pi / 2, gamma_see=1.0, load_lo=0.0,
                   load_hi=1.0, mu_const=8e-3, **kw)


def test_arena_holds_the_state():
    p = W.small(precision=0, ion_model=W.ION_FULL, n_cells=128, n_macro=30_000)
    need = hd.required_bytes(p)
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    a = hd.Discharge(p, arena=arena)
    b = hd.Discharge(p)
    for d in (a, b):
        d.step(5)
        d.step(30)
    ra, rb = (a.moments(), a.particles()), (b.moments(), b.particles())
    _same_state(ra, rb)
    orc = oracle.Oracle(p, contract=True)
    orc.step(35)
    np.testing.assert_array_equal(ra[0]["cnt"], orc.grid()["cnt"])
    np.testing.assert_array_equal(ra[0]["phi"], orc.grid()["phi"])
    a.close()
    del arena
    with pytest.raises(hd.HdError) as e:
        hd.Discharge(p, arena=torch.empty(need // 2, dtype=torch.uint8, device="cuda"))
    assert e.value.code == -2


def test_capacity_overflow_rolls_back_and_grows():
    p = _hot(capacity=20_000 + 3_000)
    steps = 48
    ref = oracle.Oracle(p, contract=True)
    ref.step(steps)
    assert ref.counters()["created"] > 3_000  # the run needs more than the capacity
    dev = hd.Discharge(p)
    dev.step(steps)
    with pytest.raises(hd.HdError) as e:
        dev.moments()
    assert e.value.code == -4
    m = dev.moments()  # the handle stands at the last complete step
    assert m["rollbacks"] == 1 and 0 < m["step"] < steps
    with pytest.raises(hd.HdError) as e:
        dev.step(1)  # stopped until the capacity grows
    assert e.value.code == -4
    # the state at the rollback equals the oracle's after the same steps
    part = oracle.Oracle(p, contract=True)
    part.step(m["step"])
    np.testing.assert_array_equal(m["cnt"], part.grid()["cnt"])
    np.testing.assert_array_equal(dev.particles()["id"], part.particles()["id"])
    dev.grow(80_000)
    dev.step(steps - m["step"])
    m2 = dev.moments()
    assert m2["step"] == steps
    o = ref.particles()
    g = dev.particles()
    np.testing.assert_array_equal(g["cell"], o["cell"])
    live = o["cell"] >= 0
    for k in ("off", "vx", "vy", "vz", "id"):
        np.testing.assert_array_equal(g[k][live], o[k][live], err_msg=k)
    for k in ("cnt", "n_i", "phi", "E"):
        np.testing.assert_array_equal(m2[k], ref.grid()[k], err_msg=k)
    dev.close()


def test_non_finite_field_is_reported():
    # 1e308 V at 1 THz: the drive reaches ~1e307 V within a step, so the
    # field at the walls (V / dz) overflows to infinity
    p = W.small(precision=0, n_cells=64, n_macro=5_000, v_amp_V=1e308, f_rf_Hz=1e12,
                phase_rad=0.0)
    dev = hd.Discharge(p)
    dev.step(5)
    with pytest.raises(hd.HdError) as e:
        dev.moments()
    assert e.value.code == -5
    with pytest.raises(hd.HdError):
        dev.step(1)
    dev.close()
    with pytest.raises(hd.HdError) as e:  # already infinite at step 0
        hd.Discharge(dict(p, phase_rad=np.pi / 2))
    assert e.value.code == -5


def test_graph_path_runs():
    p = W.small(precision=0, n_cells=64, n_macro=5_000)
    dev = hd.Discharge(p)
    dev.step(3)   # direct launches up to the interval boundary...
    dev.step(13)
    dev.step(32)  # ...then two captured intervals
    m = dev.moments()
    assert m["step"] == 48 and m["graph_steps"] == 32
    dev.close()
