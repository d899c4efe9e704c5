"""Pins of the oracle's cloud-in-cell fixed-point deposit and of the
ion-induced secondary emission."""
import numpy as np
import pytest

import oracle
from paper_1508_02892_amd import workloads as W

E_CH = 1.602176634e-19
ME = 9.1093837015e-31


@pytest.mark.parametrize("precision", [0, 1])
def test_deposit_total_is_exact(precision):
    rng = np.random.default_rng(precision)
    n, nc = 100_000, 64
    cell = rng.integers(0, nc, n)
    off = rng.random(n).astype(oracle.pdtype(precision))
    g = oracle.deposit(precision, cell, off, nc + 1)
    assert int(g.sum()) == n * 2 ** 32
    # brute force on each particle: node c gets 2^32 - rint(off 2^32), c+1 the rest
    ref = np.zeros(nc + 1, dtype=object)
    for c, o in zip(cell[:2000], off[:2000]):
        w1 = int(np.rint(np.float64(o) * 2.0 ** 32))
        ref[c] += 2 ** 32 - w1
        ref[c + 1] += w1
    g2 = oracle.deposit(precision, cell[:2000], off[:2000], nc + 1)
    assert [int(x) for x in g2] == list(ref)
    # order independence
    perm = rng.permutation(n)
    np.testing.assert_array_equal(oracle.deposit(precision, cell[perm], off[perm], nc + 1), g)


def test_deposit_at_node_puts_all_weight_on_it():
    g = oracle.deposit(1, [5, 0], [0.0, 0.0], 8)
    assert g[5] == 2 ** 32 and g[0] == 2 ** 32 and g.sum() == 2 ** 33
    g = oracle.deposit(1, [2], [0.25], 8)
    assert g[2] == 3 * 2 ** 30 and g[3] == 2 ** 30
    assert (oracle.deposit(1, [-1], [0.5], 8) == 0).all()


def _see_disch(precision=1, gamma=0.1):
    return oracle.Oracle(W.small(precision=precision, n_macro=1024, n_cells=64, gamma_see=gamma))


@pytest.mark.parametrize("X", [0.3, 2.7])
def test_emission_count_mean_is_X(X):
    o = _see_disch()
    w = o.derived()["w"]
    F = X * w / (0.1 * 2e-14)
    counts = np.array([len(o.emit(0, F, n)["cell"]) for n in range(4000)])
    lo = int(np.floor(X))
    assert set(np.unique(counts)) <= {lo, lo + 1}
    p = X - lo
    assert abs(counts.mean() - X) < 5 * np.sqrt(p * (1 - p) / len(counts))


@pytest.mark.parametrize("side", [0, 1])
def test_emission_cosine_law_speed_and_position(side):
    o = _see_disch()
    d = o.derived()
    F = 50.0 * d["w"] / (0.1 * 2e-14)
    vx, vy, vz, cell, off = [], [], [], [], []
    for n in range(400):
        e = o.emit(side, F, n)
        vx.append(e["vx"]); vy.append(e["vy"]); vz.append(e["vz"])
        cell.append(e["cell"]); off.append(e["off"])
    vx, vy, vz = (np.concatenate(a) for a in (vx, vy, vz))
    cell, off = np.concatenate(cell), np.concatenate(off)
    v = np.sqrt(vx ** 2 + vy ** 2 + vz ** 2)
    v_exp = np.sqrt(2 * E_CH * 2.0 / ME)
    np.testing.assert_allclose(v, v_exp, rtol=1e-13)
    cos = np.abs(vz) / v
    assert abs(cos.mean() - 2 / 3) < 5 * np.sqrt((1 / 2 - 4 / 9) / len(cos))
    assert (np.sign(vz) == (1 if side == 0 else -1)).all()
    phi = np.arctan2(vy, vx)
    assert abs(np.cos(phi).mean()) < 5 * np.sqrt(0.5 / len(phi))
    z = (cell + off) * d["dz"]
    flight = np.abs(vz) * 2e-14
    dist = z if side == 0 else 64 * d["dz"] - z
    assert (dist <= flight * (1 + 1e-9) + 1e-18).all()
    assert abs((dist / flight).mean() - 0.5) < 0.05
