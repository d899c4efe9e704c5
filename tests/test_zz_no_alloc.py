"""The no-allocation entry point (hd_swarm_run_noalloc) against the
allocating one (hd_swarm_create / run / results), through the C ABI.

Two calls in a row, the second with a smaller swarm (fewer fields and ions),
so that the shared work space's leftovers from the first call would show;
each must equal the three-call form on the same parameters bit for bit
(the same kernels in the same order).  Sizes beyond the work space are
rejected with HD_EINVAL.
"""
import numpy as np
import pytest

from paper_1508_02892_amd import hd, workloads as W

pytestmark = pytest.mark.gpu


def _alloc(p, n_relax, n_avg):
    s = hd.Swarm(p)
    s.run(n_relax)
    s.run(n_avg, accumulate=True)
    r = s.results()
    s.close()
    return r


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_allocating_swarm_twice(precision):
    big = W.swarm_params([1e5, 6e5, 2e6, 8e6, 0.0], n_ions=40_000, precision=precision, seed=11)
    small = W.swarm_params([3e5, 4e6], n_ions=3_001, precision=precision, seed=12)
    for p, n_relax, n_avg in ((big, 300, 520), (small, 100, 260)):
        got = hd.swarm_run_noalloc(p, n_relax, n_avg)
        ref = _alloc(p, n_relax, n_avg)
        assert len(got) == len(ref) == len(p["e0_V_m"])
        for g, r in zip(got, ref):
            for k in r:
                assert g[k] == r[k], (k, g[k], r[k])
        assert sum(r["collisions"] for r in ref) > 0
        assert all(r["samples"] == n_avg * p["n_ions"] for r in ref)


def test_noalloc_rejects_sizes_beyond_the_work_space():
    p = W.swarm_params([1e6] * 4, n_ions=1_000_000, precision=1)  # 4e6 FP64 ions
    with pytest.raises(hd.HdError) as e:
        hd.swarm_run_noalloc(p, 10, 10)
    assert e.value.code == -1
    assert "work space" in str(e.value)
    q = W.swarm_params([1e6] * 300, n_ions=64, precision=0)  # too many fields
    with pytest.raises(hd.HdError) as e:
        hd.swarm_run_noalloc(q, 10, 10)
    assert e.value.code == -1
