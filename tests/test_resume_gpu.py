"""Snapshot and resume (hd_save / hd_restore).

A run of 2N steps equals N steps, a snapshot, a fresh handle (of another
capacity) restored from it and N more steps, bit for bit: the random
streams are keyed by particle id and step, so the snapshot -- state record,
particles in use, grids -- is the whole state.  N is not a multiple of the
sort interval, so the resumed run starts inside an interval and crosses
sorts.  The cases cover both particle precisions, the full and the
drift-diffusion ion fluid, and power control (whose amplitude and running
power sums live in the state record).
"""
import numpy as np
import pytest

from paper_1508_02892_amd import hd, workloads as W

pytestmark = pytest.mark.gpu

N = 37


def _hot(precision, model, **kw):
    return W.small(precision=precision, ion_model=model, n_cells=64, n_macro=20_000,
                   t_e0_eV=50.0, v_amp_V=2000.0, phase_rad=np.pi / 2, gamma_see=1.0,
                   load_lo=0.0, load_hi=1.0, mu_const=8e-3, **kw)


CASES = {
    "fp32-full": lambda: _hot(0, W.ION_FULL),
    "fp64-dd": lambda: _hot(1, W.ION_DD),
    "fp32-power": lambda: dict(_hot(0, W.ION_DD_FIT, f_rf_Hz=1.0 / (20 * 2e-14), power_W_m2=1e6,
                                    power_alpha=0.1), phase_rad=0.0),
}


def _same(ma, pa, mb, pb):
    for k in pa:
        np.testing.assert_array_equal(pa[k], pb[k], err_msg=k)
    for k, v in ma.items():
        if k in ("graph_steps", "rollbacks"):  # how the steps were launched
            continue
        if isinstance(v, np.ndarray):
            np.testing.assert_array_equal(v, mb[k], err_msg=k)
        else:
            assert v == mb[k], k


@pytest.mark.parametrize("case", sorted(CASES))
def test_resume_equals_uninterrupted_run(case):
    p = CASES[case]()
    a = hd.Discharge(p)
    a.step(2 * N)
    ref = (a.moments(), a.particles())
    a.close()
    b = hd.Discharge(p)
    b.step(N)
    snap = b.save()
    b.close()
    q = dict(p, capacity=2 * int(p["capacity"]))
    c = hd.Discharge(q)
    c.restore(snap)
    assert c.moments()["step"] == N
    c.step(N)
    _same(*ref, c.moments(), c.particles())
    c.close()


def test_snapshot_is_refused_where_it_does_not_belong():
    p = CASES["fp32-full"]()
    b = hd.Discharge(p)
    b.step(5)
    snap = b.save()
    other = hd.Discharge(dict(p, v_amp_V=1000.0))  # other parameters
    with pytest.raises(hd.HdError) as e:
        other.restore(snap)
    assert e.value.code == -1
    with pytest.raises(hd.HdError) as e:
        b.restore(snap[: len(snap) // 2])  # truncated
    assert e.value.code == -1
    # a handle of the least capacity its parameters allow (n_macro, rounded
    # up to whole sort tiles) against a snapshot of a run that has grown
    # past it
    tight = hd.Discharge(dict(p, capacity=int(p["n_macro"])))
    slots = -(-int(p["n_macro"]) // 4096) * 4096
    while b.moments()["n_slots"] <= slots and b.moments()["step"] < 400:
        b.step(10)
    assert b.moments()["n_slots"] > slots
    with pytest.raises(hd.HdError) as e:
        tight.restore(b.save())
    assert e.value.code == -4  # HD_ECAPACITY
    for h in (b, other, tight):
        h.close()
