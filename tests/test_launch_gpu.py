"""Launch shapes do not change results.

Every shape the autotuner may pick (the electron kernel variant -- how the
particle data are loaded, with or without the nontemporal hint, in 512- or
1,024-thread workgroups -- and its workgroup count, the sort's workgroup
count and tile, the append's workgroup count) must give bitwise the same
run: particles are processed in fixed sub-chunks, deposits are integer
sums, children are appended in parent order and the sort is stable, so no
launch shape can reach a result.  The batch is shaped like the batched
sweep (uneven gaps, grids, voltages and particle counts); two members are
also checked against the oracle, and a run whose first steps were taken by
the autotuner equals a run with a fixed shape.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1508_02892_amd import hd, workloads as W

pytestmark = pytest.mark.gpu

STEPS = 40  # two sorts and a partial interval


def _params():
    ps = W.c3(n_discharges=6, total_electrons=0)
    sizes = [20_000, 150_000, 4_097, 60_000, 90_001, 33_000]
    return [W.scaled(p, n) for p, n in zip(ps, sizes)]


def _run(ps, cfg=None, tune=0):
    b = hd.Batch(ps)
    if cfg is not None:
        b.set_launch(cfg)
    used = b.get_launch()
    if tune:
        used = b.autotune(tune)
        b.step(STEPS - tune)
    else:
        b.step(7)
        b.step(STEPS - 7)
    out = [(b.moments(i), b.particles(i)) for i in range(len(ps))]
    b.close()
    return out, used


def _same(a, b):
    for (ma, pa), (mb, pb) in zip(a, b):
        for k in pa:
            np.testing.assert_array_equal(pa[k], pb[k], err_msg=k)
        for k, v in ma.items():
            if k in ("graph_steps", "rollbacks"):  # how the steps were launched
                continue
            if isinstance(v, np.ndarray):
                np.testing.assert_array_equal(v, mb[k], err_msg=k)
            else:
                assert v == mb[k], k


CONFIGS = [
    {"electron_variant": 1},
    {"electron_variant": 2},
    {"electron_variant": 2, "electron_groups": 100},
    {"electron_variant": 0, "electron_groups": 7},
    {"electron_variant": 1, "electron_groups": 33},
    {"electron_variant": 3},
    {"electron_variant": 4, "electron_groups": 77},
    {"electron_variant": 5, "electron_groups": 200},
    {"electron_variant": 6},
    {"electron_variant": 7},
    {"electron_variant": 7, "electron_groups": 3},
    {"electron_variant": 8},                          # wide workgroups (1,024 threads)
    {"electron_variant": 10, "electron_groups": 5},
    {"electron_variant": 11},
    {"electron_variant": 12, "electron_groups": 50},
    {"electron_variant": 13, "electron_groups": 100},
    {"electron_variant": 14},
    {"electron_variant": 15, "electron_groups": 2},
    {"sort_groups": 3},
    {"sort_tile": 8192},
    {"sort_tile": 8192, "sort_groups": 7},
    {"append_groups": 1},
    {"electron_variant": 1, "electron_groups": 1, "sort_groups": 1000, "append_groups": 64},
]


def test_every_launch_shape_gives_the_same_run():
    ps = _params()
    ref, used = _run(ps, {})
    print("default shape:", used)
    for cfg in CONFIGS:
        got, used = _run(ps, cfg)
        print("shape:", used)
        for k, v in cfg.items():
            assert used[k] == v
        _same(ref, got)
    for i in (0, 2):
        orc = oracle.Oracle(ps[i], contract=True)
        orc.step(STEPS)
        m, p = ref[i]
        o = orc.particles()
        np.testing.assert_array_equal(p["cell"], o["cell"])
        live = o["cell"] >= 0
        for k in ("off", "vx", "vy", "vz", "id"):
            np.testing.assert_array_equal(p[k][live], o[k][live], err_msg=k)
        np.testing.assert_array_equal(m["cnt"], orc.grid()["cnt"])
        np.testing.assert_array_equal(m["phi"], orc.grid()["phi"])


def test_autotuned_run_equals_fixed_shape_run():
    ps = _params()
    ref, _ = _run(ps, {})
    got, chosen = _run(ps, tune=32)
    print("autotuner chose:", chosen)
    _same(ref, got)


def test_invalid_shapes_are_rejected():
    b = hd.Batch(_params()[:2])
    for cfg in ({"electron_variant": 99}, {"electron_variant": -1}, {"electron_groups": 5000},
                {"sort_groups": -1}, {"append_groups": 100000}, {"sort_tile": 2048}, {"sort_tile": 16384},
                {"sort_tile": 6000}):
        with pytest.raises(hd.HdError) as e:
            b.set_launch(cfg)
        assert e.value.code == -1
    with pytest.raises(hd.HdError):
        b.autotune(8)  # below two sort intervals
    b.close()
    # FP64 and the register-prefetch kernel have no wide workgroups
    d = hd.Discharge(W.c0())
    with pytest.raises(hd.HdError) as e:
        d.set_launch({"electron_variant": 8})
    assert e.value.code == -1
    d.close()
    b = hd.Batch(_params()[:2])
    with pytest.raises(hd.HdError) as e:
        b.set_launch({"electron_variant": 9})
    assert e.value.code == -1
    b.close()


def test_c3_full_scale_batch_equals_single_handles():
    # The batched sweep at full size: 64 discharges, 2^26 electrons in all,
    # 256-4096 cells.  After 17 steps (one sort), every member equals the
    # same discharge run alone, bit for bit; three members (the smallest,
    # one in the middle and the largest grid) also equal the oracle.
    ps = W.c3()
    assert sum(p["n_macro"] for p in ps) == 1 << 26
    b = hd.Batch(ps)
    b.step(17)
    for i, p in enumerate(ps):
        d = hd.Discharge(p)
        d.step(17)
        _same([(b.moments(i), b.particles(i))], [(d.moments(), d.particles())])
        d.close()
    picks = {int(np.argmin([p["n_macro"] for p in ps])), len(ps) // 2,
             int(np.argmax([p["n_cells"] for p in ps]))}
    for i in sorted(picks):
        orc = oracle.Oracle(ps[i], contract=True)
        orc.step(17)
        m, p = b.moments(i), b.particles(i)
        o = orc.particles()
        np.testing.assert_array_equal(p["cell"], o["cell"])
        live = o["cell"] >= 0
        for k in ("off", "vx", "vy", "vz", "id"):
            np.testing.assert_array_equal(p[k][live], o[k][live], err_msg=k)
        for k in ("cnt", "n_i", "phi", "E"):
            np.testing.assert_array_equal(m[k], orc.grid()[k], err_msg=k)
    b.close()


_TUNE_CHILD = """
import json, sys
sys.path.insert(0, sys.argv[2])
from paper_1508_02892_amd import hd, workloads as W
ps = [W.scaled(p, n) for p, n in zip(W.c3(n_discharges=3, total_electrons=0), [30000, 50000, 20000])]
b = hd.Batch(ps)
c = b.autotune(32) if sys.argv[1] == "tune" else b.get_launch()
print(json.dumps(c))
b.close()
"""


def test_tune_cache_file_carries_the_choice_across_processes(tmp_path):
    # A process that autotunes appends its choice to the HD_TUNE_CACHE file;
    # a later process with a batch of the same shape starts from the file's
    # last entry for that shape (here rewritten to a shape the tuner would
    # not pick, so that it can only have come from the file).
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, HD_TUNE_CACHE=str(cache))

    def child(mode):
        r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, mode, root], env=env,
                           capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    tuned = child("tune")
    lines = cache.read_text().split("\n")
    key, *vals = lines[0].split()
    assert [int(v) for v in vals] == [tuned[k] for k in ("electron_variant", "electron_groups",
                                                        "sort_groups", "append_groups",
                                                        "sort_tile")]
    assert child("fresh") == tuned
    with open(cache, "a") as f:
        f.write("%s 1 77 333 5 8192\n" % key)
    assert child("fresh") == {"electron_variant": 1, "electron_groups": 77, "sort_groups": 333,
                              "append_groups": 5, "sort_tile": 8192}
    with open(cache, "a") as f:  # a line without the tile keeps the default one
        f.write("%s 2 50 100 4\n" % key)
    assert child("fresh") == {"electron_variant": 2, "electron_groups": 50, "sort_groups": 100,
                              "append_groups": 4, "sort_tile": 4096}


def test_untuned_default_follows_the_mall():
    # Without a cached choice a handle starts cached (variant 0) while its
    # initial particle state fits the 256 MB MALL, else with nontemporal
    # ids, cells and offsets (variant 5); on a grid so large that a narrow
    # workgroup's LDS leaves room for only one per CU, with wide workgroups
    # (variants 8 and 13).
    for cells, gap, wide in ((2048, 1e-3, 0), (4096, 2e-3, 8)):
        p = W.c1(n_cells=cells, gap_m=gap, ion_model=W.ION_DD)
        small = hd.Discharge(W.scaled(p, 4 << 20))
        big = hd.Discharge(W.scaled(p, 12 << 20))
        assert small.get_launch()["electron_variant"] == 0 + wide
        assert big.get_launch()["electron_variant"] == 5 + wide
        small.close()
        big.close()
